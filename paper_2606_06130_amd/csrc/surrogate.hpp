// Learned multipath surrogate (surrogate.hip): host entry points behind the
// library's C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sonar {

struct Surrogate;
hipError_t surrogate_create(int64_t max_rows, int n_bins, float r_min, float r_max, int smooth, Surrogate **out);
void surrogate_free(Surrogate *s);
int64_t surrogate_param_count();
int64_t surrogate_max_rows(const Surrogate *s);
int surrogate_bins(const Surrogate *s);
hipError_t surrogate_set_state(Surrogate *s, const float *master, const float *m, const float *v, int64_t step);
hipError_t surrogate_get_state(const Surrogate *s, float *master, float *m, float *v, int64_t *step);
hipError_t surrogate_set_norm(Surrogate *s, const float *mu, const float *sg);
// `geo`: one geometry block of 16 floats per image (device), see sonar.h
hipError_t surrogate_forward(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W, float *coef,
                             hipStream_t st);
hipError_t surrogate_gradient(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W,
                              const float *target, float *dev_grad, float *dev_loss, hipStream_t st);
hipError_t surrogate_train_step(Surrogate *s, const float *gbuf, const float *geo, int n_img, int H, int W,
                                const float *target, float lr, float *dev_loss, hipStream_t st);
hipError_t surrogate_set_loss_weights(Surrogate *s, const float *w);
hipError_t surrogate_target_coef(const Surrogate *s, const float *im, const float *gbuf, int64_t rows,
                                 int standardize, float *coef, hipStream_t st);
hipError_t surrogate_coef_moments(Surrogate *s, const float *coef, int64_t rows, double *host_sum, double *host_sq,
                                  hipStream_t st);
hipError_t surrogate_profile_errors(const Surrogate *s, const float *pred, const float *i1, const float *im,
                                    const float *gbuf, int64_t rows, float *err, float *profile, hipStream_t st);

}  // namespace sonar
