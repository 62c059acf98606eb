"""Independent pings issued on several streams at once (as the benchmark's
jobs do) give the same outputs as the same pings one at a time: the staged
multi-bounce ping keeps all its state in the caller's workspace, and the
surrogate's inference and profile read only shared weights (needs an MI355X)."""
import math
import sys

import numpy as np
import pytest

from paper_2606_06130_amd import scenes as S

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU (it must not pass by skipping)")
    from paper_2606_06130_amd import sonar
    return torch, sonar


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _poses(n):
    return [S.pose((0.3 * i, 0.5 - 0.2 * i, -2.0 - 0.3 * i), yaw=math.radians(8 * i - 12),
                   pitch_down=math.radians(30 + 3 * i), ping=i) for i in range(n)]


def test_staged_multipath_pings_on_four_streams():
    torch, sonar = _gpu()
    scene = sonar.Scene(S.scene_harbor_multipath())
    cfg = S.sensor_harbor_multipath().replace(n_h=128, n_v=64, rays_per_beam=8)
    poses = _poses(4)
    ref = []
    for p in poses:
        o = sonar.alloc_outputs(cfg, incoh=True)
        sonar.ping(scene, cfg, p, out=o, staged=True)
        torch.cuda.synchronize()
        ref.append(o)
    streams = [torch.cuda.Stream() for _ in poses]
    outs = [sonar.alloc_outputs(cfg, incoh=True) for _ in poses]
    for _ in range(3):                     # several rounds so that the streams overlap
        for p, o, st in zip(poses, outs, streams):
            sonar.ping(scene, cfg, p, out=o, staged=True, stream=st)
    torch.cuda.synchronize()
    assert scene.status() == 0
    for i, (a, b) in enumerate(zip(outs, ref)):
        _log("ping", i, "volume norm", float(b["volume"].abs().norm()))
        assert float(b["volume"].abs().norm()) > 0
        assert torch.equal(a["volume"], b["volume"]), i
        assert torch.equal(a["incoh"], b["incoh"]), i


def test_surrogate_pings_on_four_streams():
    torch, sonar = _gpu()
    from paper_2606_06130_amd import surrogate as SU
    scene = sonar.Scene(S.scene_harbor_multipath())
    cfg = S.sensor_harbor_multipath().replace(n_h=128, n_v=64, rays_per_beam=8, max_bounces=1)
    bv, bh = sonar.beams_of(cfg)
    rows = bv * bh
    sur = sonar.Surrogate(rows, cfg.n_range, cfg.r_min, cfg.r_max)
    SU.load_checkpoint(SU.WEIGHTS, sur)
    poses = _poses(4)
    geo = torch.from_numpy(sonar.surrogate_geometry(cfg, poses)).cuda()

    def bufs():
        o = sonar.alloc_outputs(cfg, gbuffer=True, incoh=True)
        return (o, o["gbuffer"].view(1, bv, bh, 8), o["incoh"].view(2, rows, cfg.n_range)[0],
                torch.empty((rows, 64), device="cuda"), torch.empty((rows, cfg.n_range), device="cuda"))

    def run(i, b, st=None):
        o, gv, i1, cf, pf = b
        sonar.ping(scene, cfg, poses[i], out=o, stream=st)
        sur.forward(gv, geo[i:i + 1], out=cf, stream=st)
        sur.profile(cf, i1, gv, im=None, want_profile=True, stream=st, out=pf)

    ref = []
    for i in range(4):
        b = bufs()
        run(i, b)
        torch.cuda.synchronize()
        ref.append(b)
    streams = [torch.cuda.Stream() for _ in poses]
    got = [bufs() for _ in poses]
    for _ in range(3):
        for i in range(4):
            run(i, got[i], streams[i])
    torch.cuda.synchronize()
    for i in range(4):
        assert torch.equal(got[i][3], ref[i][3]), i          # coefficients
        assert torch.equal(got[i][4], ref[i][4]), i          # profile
    _log("surrogate profiles equal on four streams")
