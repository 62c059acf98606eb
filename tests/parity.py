"""Helpers that compare the HIP path with the oracle (test infrastructure)."""
from __future__ import annotations

import numpy as np

import oracle


def mask_words(n_rays: int, flagged_rays) -> np.ndarray:
    """uint32 bit mask over rays with the given ray indices set."""
    w = np.zeros((n_rays + 31) // 32, np.uint32)
    fr = np.asarray(flagged_rays, np.int64)
    np.bitwise_or.at(w, fr >> 5, (np.uint32(1) << (fr & 31).astype(np.uint32)))
    return w


def ray_ids(beams, n_r):
    beams = np.asarray(beams, np.int64)
    return (beams[:, None] * n_r + np.arange(n_r)[None, :]).reshape(-1)


def flag_summary(flags) -> dict:
    flags = np.asarray(flags)
    out = {"rays": int(flags.size), "flagged": int((flags != 0).sum())}
    for i, nm in enumerate(oracle.FLAG_NAMES):
        c = int(((flags >> i) & 1).sum())
        if c:
            out[nm] = c
    return out


def compare_rays(gpu: dict, orc: dict, rays) -> dict:
    """Bit-exact comparison of hit triangle, bin and visibility on the
    oracle's unflagged rays. ``gpu`` arrays are indexed by global ray id,
    ``orc`` arrays by position in ``rays``."""
    ok = orc["flags"] == 0
    res = {}
    for key in ("tri", "bin", "vis"):
        g = np.asarray(gpu[key])[rays][ok]
        o = np.asarray(orc[key])[ok]
        if key == "vis":
            # visibility is only defined where there was a hit
            g = np.where(np.asarray(orc["tri"])[ok] >= 0, g, 0)
            o = np.where(np.asarray(orc["tri"])[ok] >= 0, o, 0)
        res[key + "_mismatch"] = int((g != o).any(axis=1).sum())
    if "beam" in gpu and "rxb" in orc:
        # the beam each contribution is added to, where there is one
        has = np.asarray(orc["bin"])[ok] >= 0
        g = np.where(has, np.asarray(gpu["beam"])[rays][ok], -1)
        o = np.where(has, np.asarray(orc["rxb"])[ok], -1)
        res["beam_mismatch"] = int((g != o).any(axis=1).sum())
    if "rbin" in gpu and "rbin" in orc:
        # retro-chain returns: bins exact, values to the volume tolerance
        res["rbin_mismatch"] = int((np.asarray(gpu["rbin"])[rays][ok] != np.asarray(orc["rbin"])[ok]).any(axis=1).sum())
        res["retro_err"] = rel_l2(np.asarray(gpu["ramp"])[rays][ok], np.asarray(orc["ramp"])[ok])
        res["retro_returns"] = int((np.asarray(orc["rbin"])[ok] >= 0).sum())
    res.update(flag_summary(orc["flags"]))
    return res


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    nb = np.linalg.norm(b)
    if nb == 0:
        return float(np.linalg.norm(a))
    return float(np.linalg.norm(a - b) / nb)


def compare_points(pts, total, o, beams):
    """GPU points vs the oracle's, beam by beam, skipping beams with a
    threshold- or peak-flagged decision. Returns the number of beams compared."""
    assert total == len(pts)
    by_beam = {}
    for p in pts:
        by_beam.setdefault(int(p["beam"]), []).append(p)
    compared = 0
    for q, b in enumerate(beams):
        if o["beam_flag"][q]:
            continue
        fb = o["flag_bins"][q]
        ob = [x for x in o["bin"][q] if x >= 0]
        gb = [int(p["bin"]) for p in by_beam.get(int(b), [])]
        if any(fb[x] for x in set(ob) | set(gb)):
            continue
        assert gb == ob, (b, gb, ob)
        for p, want in zip(by_beam.get(int(b), []), o["pts"][q]):
            np.testing.assert_allclose([p["x"], p["y"], p["z"]], want[:3], atol=2e-5)
            assert abs(p["db"] - want[3]) < 1e-3
        compared += 1
    # points come out in (beam, range) order
    keys = pts["beam"].astype(np.int64) * 100000 + pts["bin"]
    assert np.all(np.diff(keys) > 0)
    return compared
