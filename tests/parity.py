"""Comparison rules between the HIP path and the oracle (shared by the GPU tests).

Classes: (cls, n_hits, hit ordinals) must be identical for every pixel outside
the edge band E, the pixels with an 8-neighbour of a different oracle class
(several answers are right at class boundaries: the shadow edge, disk edges,
image-order boundaries).  Values, on pixels whose classes match and that lie
outside E: relative error of r_em and g of every recorded hit, of the final
theta, absolute error of the final phi scaled by max(1, |phi|), and the flux as
max |dI| / max(I); the constraint residual separately (gated maximum absolute,
full maximum on escaped rays within 1e-12 absolute or 1e-4 relative: both
depend on the step sequence, which two correct implementations reproduce to
rounding, and the full maximum on the 1/Delta growth of dH/dq near the stop).
"""
import numpy as np


def class_key(o):
    return (o["cls"].astype(np.int64) * 1000 + o["n_hits"] * 100
            + np.clip(o["hit_order"][:, 0], 0, 9) * 10 + np.clip(o["hit_order"][:, 1], 0, 9))


def edge_band(key2d):
    band = np.zeros(key2d.shape, dtype=bool)
    H, W = key2d.shape
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            ys, yd = slice(max(0, dj), H + min(0, dj)), slice(max(0, -dj), H + min(0, -dj))
            xs, xd = slice(max(0, di), W + min(0, di)), slice(max(0, -di), W + min(0, -di))
            band[yd, xd] |= key2d[ys, xs] != key2d[yd, xd]
    return band


def compare(g, o, band, tol, h_tol=None):
    """Return a dict of error statistics; asserts nothing."""
    kg, ko = class_key(g), class_key(o)
    off = ~band
    mism = off & (kg != ko)
    ok = off & (kg == ko)
    res = {"n": len(ko), "band": int(band.sum()), "class_mismatch_off_band": int(mism.sum()),
           "class_mismatch_in_band": int((band & (kg != ko)).sum())}
    errs = {}
    hits = o["n_hits"]
    for name in ("hit_r", "hit_g"):
        e = []
        for k in range(3):
            m = ok & (hits > k)
            if m.any():
                e.append(np.abs(g[name][m, k] / o[name][m, k] - 1.0))
        errs[name] = np.concatenate(e) if e else np.zeros(0)
    th = np.abs(g["final_rtp"][ok, 1] / o["final_rtp"][ok, 1] - 1.0)
    ph = np.abs(g["final_rtp"][ok, 2] - o["final_rtp"][ok, 2]) / np.maximum(1.0, np.abs(o["final_rtp"][ok, 2]))
    errs["final_theta"] = th
    errs["final_phi"] = ph
    imax = max(np.abs(o["intensity"]).max(), 1e-300)
    errs["flux"] = np.abs(g["intensity"][ok] - o["intensity"][ok]) / imax
    # the constraint residual: the gated maximum (states with r >= 1.5 r_+) in
    # absolute terms; the full maximum, which near the stop radius is dominated
    # by the 1/Delta growth of dH/dq, relative to its own size
    errs["h_gate_abs"] = np.abs(g["h_gate"][ok] - o["h_gate"][ok])
    # (captured rays are left out: their last accepted step ends past the stop
    # radius, where H is ill-conditioned)
    # a ray passes the full-maximum check within 1e-12 absolute or 1e-4
    # relative (near the rounding level of H, ~1e-13, only the first is
    # meaningful); h_drift_rel holds the relative difference beyond 1e-12
    esc = ok & (o["cls"] == 0)
    dh = np.abs(g["h_drift"][esc] - o["h_drift"][esc])
    errs["h_drift_rel"] = np.where(dh <= 1e-12, 0.0, dh / (np.abs(o["h_drift"][esc]) + 1e-300))
    for k, v in errs.items():
        res[k] = {"max": float(v.max()) if v.size else 0.0,
                  "p50": float(np.median(v)) if v.size else 0.0,
                  "p99": float(np.quantile(v, 0.99)) if v.size else 0.0, "n": int(v.size)}
    res["tol"] = tol
    return res


def assert_parity(res, tol, h_tol=None):
    assert res["class_mismatch_off_band"] == 0, res
    for k in ("hit_r", "hit_g", "final_theta", "final_phi", "flux"):
        assert res[k]["max"] <= tol, (k, res[k], res)
    if h_tol is not None:
        assert res["h_gate_abs"]["max"] <= h_tol, res["h_gate_abs"]
        if h_tol <= 1e-12:
            assert res["h_drift_rel"]["max"] <= 1e-4, res["h_drift_rel"]
