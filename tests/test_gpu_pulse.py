"""Pulse compression (time series and matched filter of each beam column)
on the GPU against the FP64 oracle, through the C-ABI (needs an MI355X)."""
import math
import sys

import numpy as np
import pytest

from oracle import pulse as OP
from paper_2606_06130_amd import scenes as S

pytestmark = pytest.mark.gpu

TOL = 1e-5          # relative L2 per output: FP32 sums of at most 2 x 64 products


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("a GPU test ran without a visible GPU (it must not pass by skipping)")
    from paper_2606_06130_amd import sonar
    return torch, sonar


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    d = np.linalg.norm(np.asarray(a, np.complex128) - b)
    n = np.linalg.norm(b)
    return d / n if n > 0 else d


def _rand_complex(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.normal(size=shape) + 1j * rng.normal(size=shape)).astype(np.complex64)


@pytest.mark.parametrize("n_beams,n_bins,L,want", [
    (37, 300, 16, "both"), (5, 1024, 64, "both"), (3, 7, 9, "both"), (2, 1, 1, "both"),
    (11, 2048, 33, "series"), (11, 257, 5, "matched"), (64, 1024, 16, "both"), (1, 4, 64, "both")])
def test_random_columns_match_oracle(n_beams, n_bins, L, want):
    torch, sonar = _gpu()
    x = _rand_complex((n_beams, n_bins), 100 + n_bins + L)
    p = _rand_complex(L, 7 + L)
    _log("pulse", n_beams, n_bins, L, want)
    xd = torch.from_numpy(x).cuda()
    out = sonar.pulse_compress(xd, p, series=want in ("both", "series"), matched=want in ("both", "matched"))
    torch.cuda.synchronize()
    s_ref, y_ref = OP.compress(x.astype(np.complex128), p.astype(np.complex128))
    if "series" in out:
        assert _rel(out["series"].cpu().numpy(), s_ref) <= TOL
    if "matched" in out:
        assert _rel(out["matched"].cpu().numpy(), y_ref) <= TOL
    assert torch.equal(xd.cpu(), torch.from_numpy(x))                     # input untouched


def _sparse_returns(n_beams, n_bins, seed, per_beam=16):
    """Seeded stand-in for a ping volume: per beam a few returns at random
    bins with log-normal amplitudes and uniform phases, zeros elsewhere."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = np.zeros((n_beams, n_bins), np.complex64)
    k = rng.integers(0, per_beam + 1, n_beams)
    for b in np.nonzero(k)[0]:
        bins = rng.integers(0, n_bins, int(k[b]))
        amp = np.exp(rng.normal(-9.0, 1.5, int(k[b])))
        ph = rng.uniform(0, 2 * math.pi, int(k[b]))
        np.add.at(x[b], bins, (amp * np.exp(1j * ph)).astype(np.complex64))
    return x


def test_harbor_size_sampled_beams():
    """The harbor layout (32,768 beams x 1,024 bins) with the benchmark's
    16-tap LFM pulse, in the launch configuration the benchmark times;
    sampled beams against the oracle."""
    torch, sonar = _gpu()
    cfg, pose = S.sensor_harbor(), S.pose_harbor()
    bv, bh = sonar.beams_of(cfg)
    nb = bv * bh
    x = _sparse_returns(nb, cfg.n_range, 21)
    dt = sonar.pulse_dt(cfg, pose)
    p = sonar.lfm_pulse(40e3, 300e-6, dt)
    assert len(p) == 16
    xd = torch.from_numpy(x).cuda().view(bv, bh, cfg.n_range)
    out = sonar.pulse_compress(xd, p)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(5))
    beams = np.concatenate([[0, nb - 1], rng.choice(nb, 62, replace=False)])
    s = out["series"].view(nb, -1)[torch.from_numpy(beams).cuda()].cpu().numpy()
    y = out["matched"].view(nb, -1)[torch.from_numpy(beams).cuda()].cpu().numpy()
    s_ref, y_ref = OP.compress(x[beams].astype(np.complex128), p.astype(np.complex128))
    assert _rel(s, s_ref) <= TOL and _rel(y, y_ref) <= TOL
    # every beam: the matched output's energy equals that of the series
    # correlated with the pulse, a property that holds at any size; here the
    # cheaper check that empty columns stay exactly zero
    empty = np.nonzero(~np.any(x != 0, axis=1))[0]
    if len(empty):
        e = torch.from_numpy(empty[:256]).cuda()
        assert int(torch.count_nonzero(out["matched"].view(nb, -1)[e])) == 0


def test_graph_replays_match_eager():
    """The call allocates nothing and records no memset: captured once, each
    replay (with eager work in between) reproduces the eager result."""
    torch, sonar = _gpu()
    x = _rand_complex((300, 512), 3)
    p = _rand_complex(24, 4)
    xd = torch.from_numpy(x).cuda()
    eager = sonar.pulse_compress(xd, p)
    torch.cuda.synchronize()
    want = {k: v.clone() for k, v in eager.items()}
    out = {k: torch.empty_like(v) for k, v in want.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        sonar.pulse_compress(xd, p, out=out, stream=s)      # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            sonar.pulse_compress(xd, p, out=out, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        for v in out.values():
            v.fill_(complex(float("nan"), 0.0))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in want:
            assert torch.equal(out[k], want[k]), (rep, k)


def test_ping_then_matched_cfar_runs():
    """Composition: a ping's volume, its matched-filter output, CA-CFAR on
    that output (ranges of the strongest detections stay near those of the
    raw volume's)."""
    torch, sonar = _gpu()
    mesh = S.scene_seabed_boxes()
    cfg, pose = S.sensor_seabed_boxes(), S.pose_seabed_boxes()
    sc = sonar.Scene(mesh)
    vol = sonar.ping(sc, cfg, pose)["volume"]
    p = sonar.lfm_pulse(40e3, 200e-6, sonar.pulse_dt(cfg, pose))
    y = sonar.pulse_compress(vol, p, series=False)["matched"]
    det = sonar.Detector(cfg)
    det(y, pose)
    pts, n = det.fetch()
    torch.cuda.synchronize()
    assert sc.status() == 0 and n > 0
