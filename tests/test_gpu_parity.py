"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

FP64 path: identical classes off the edge band and relative error <= 1e-9 in
emission radius, redshift, final theta (phi: 1e-9 * max(1, |phi|)), flux as
max |dI| / max(I), and |d h_drift| <= 1e-12.  Mixed path: the same rules at
1e-4.  Full-size images are checked on seeded samples of pixels (with their 8
neighbours traced by the oracle for the edge band) in the launch configuration
the benchmark uses.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from parity import assert_parity, class_key, compare, edge_band

pytestmark = pytest.mark.gpu

FP64_TOL, FP64_HTOL, MIXED_TOL = 1e-9, 1e-12, 1e-4
# Tabulated metric: the bicubic Hermite metric is only C^1 across cell edges,
# so the right-hand side has kinks and the step sequence is fragile.  The
# oracle itself moves by up to 1.8e-7 (emission radius) and 1.7e-6 (final
# theta) when its table entries carry 2e-16 relative noise; two correct FP64
# implementations cannot agree more closely than that.  Bar: 1e-5 relative,
# 1e-7 absolute on the gated constraint residual.
TAB_TOL, TAB_HTOL = 1e-5, 1e-7


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_08989_amd import tartarus as T
    T.tartarus_init(0, 0)
    return T


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_trace(T, a, cams, disk, solver, precision=0, launch=None, table=None):
    import torch
    cams = cams if isinstance(cams, list) else [cams]
    n = sum(c["nx"] * c["ny"] for c in cams)
    out = T.alloc_outputs(n)
    metric = T.make_metric(a) if table is None else T.make_metric(a, *table)
    T.tartarus_trace(metric, [T.make_camera(c) for c in cams], T.make_disk(disk), T.make_solver(solver, precision),
                     out, launch=launch)
    torch.cuda.synchronize()
    return T.to_numpy(out)


def oracle_trace(orc, a, cams, disk, solver, ray_ids=None, table=None):
    cams = cams if isinstance(cams, list) else [cams]
    m = orc.make_metric(a) if table is None else orc.make_metric(a, *table)
    return orc.trace(m, [orc.make_camera(c) for c in cams], orc.make_disk(disk), orc.make_solver(solver),
                     ray_ids=ray_ids)


def full_image_parity(T, orc, a, cam, disk, solver, precision=0, tol=FP64_TOL, htol=FP64_HTOL):
    g = gpu_trace(T, a, cam, disk, solver, precision)
    o = oracle_trace(orc, a, cam, disk, solver)
    band = edge_band(class_key(o).reshape(cam["ny"], cam["nx"])).ravel()
    res = compare(g, o, band, tol)
    say(res)
    assert_parity(res, tol, htol)
    return g, o


def sampled_parity(T, orc, a, cam, disk, solver, precision, nsample, seed, tol, htol=None, g=None):
    """Full image on the GPU; the oracle traces sampled pixels and their neighbours."""
    nx, ny = cam["nx"], cam["ny"]
    if g is None:
        g = gpu_trace(T, a, cam, disk, solver, precision)
    rng = np.random.default_rng(seed)
    ii = rng.integers(1, nx - 1, nsample)
    jj = rng.integers(1, ny - 1, nsample)
    offs = [(dj, di) for dj in (-1, 0, 1) for di in (-1, 0, 1)]
    ids = np.array([(j + dj) * nx + (i + di) for i, j in zip(ii, jj) for dj, di in offs], dtype=np.int64)
    uniq, inv = np.unique(ids, return_inverse=True)
    o_u = oracle_trace(orc, a, cam, disk, solver, ray_ids=uniq)
    key_u = class_key(o_u)
    key9 = key_u[inv].reshape(nsample, 9)
    band = np.any(key9 != key9[:, 4:5], axis=1)
    centre = inv.reshape(nsample, 9)[:, 4]
    o = {k: v[centre] for k, v in o_u.items()}
    gs = {k: v[uniq[centre]] for k, v in g.items()}
    res = compare(gs, o, band, tol)
    say(res)
    assert_parity(res, tol, htol)
    return g, res


# ------------------------------------------------------------------ FP64 images
def test_schwarzschild_64_full(T, orc):
    w = W.WORKLOADS["schwarzschild_64"]
    say("case schwarzschild_64 fp64")
    g, o = full_image_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"])
    assert np.array_equal(g["n_accept"], o["n_accept"]) or np.mean(g["n_accept"] == o["n_accept"]) > 0.99


def test_kerr_ragged_with_disk(T, orc):
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=37, ny=29)
    say("case kerr09 37x29 fp64")
    g, o = full_image_parity(T, orc, w["a"], cam, w["disk"], w["solver"])
    assert (o["n_hits"] > 0).sum() > 50


def test_narrow_disk_ring_edges(T, orc):
    """A ring r in [3, 4]: many equatorial crossings straddle an edge of the disk
    within one step, so the integrator locates those roots itself while the rest
    are left to the finishing pass; both must agree with the oracle."""
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=48, ny=40, alpha_min=-9.0, alpha_max=9.0, beta_min=-8.0, beta_max=8.0)
    for max_hits in (3, 1):
        disk = dict(w["disk"], r_in=3.0, r_out=4.0, max_hits=max_hits)
        say("case ring 3..4, max_hits", max_hits)
        g = gpu_trace(T, w["a"], cam, disk, w["solver"])
        o = oracle_trace(orc, w["a"], cam, disk, w["solver"])
        # a ring image has hit-count edges everywhere, so compare every ray whose
        # class and hit count agree (a disagreement needs a crossing within
        # rounding of r_in or r_out)
        same = (g["cls"] == o["cls"]) & (g["n_hits"] == o["n_hits"])
        say("rays", same.size, "class/hit-count disagreements", int((~same).sum()))
        assert (~same).sum() <= 2
        assert (o["n_hits"] > 0).sum() > 100
        for k in range(max_hits):
            m = same & (o["n_hits"] > k)
            if not m.any():
                continue
            er = np.abs(g["hit_r"][m, k] / o["hit_r"][m, k] - 1).max()
            eg = np.abs(g["hit_g"][m, k] / o["hit_g"][m, k] - 1).max()
            say("slot", k, "hits", int(m.sum()), "max rel err r", er, "g", eg)
            assert er <= FP64_TOL and eg <= FP64_TOL
            assert np.array_equal(g["hit_order"][m, k], o["hit_order"][m, k])


def test_more_cameras_than_the_lds_directory(T, orc):
    """1100 cameras in one launch (the job directory no longer fits in LDS):
    identical to the same cameras traced in launches of 550; a few cameras are
    checked against the oracle."""
    w = W.WORKLOADS["kerr09_512"]
    base = w["cameras"][0]
    cams = [dict(base, nx=3, ny=3, theta_obs=(5.0 + 80.0 * k / 1099) * math.pi / 180.0) for k in range(1100)]
    say("case 1100 cameras")
    g = gpu_trace(T, w["a"], cams, w["disk"], w["solver"])
    parts = [gpu_trace(T, w["a"], cams[i:i + 550], w["disk"], w["solver"]) for i in (0, 550)]
    for k in g:
        assert np.array_equal(g[k], np.concatenate([p[k] for p in parts])), k
    for c in (0, 549, 1099):
        o = oracle_trace(orc, w["a"], cams[c], w["disk"], w["solver"])
        gs = {k: v[9 * c:9 * c + 9] for k, v in g.items()}
        assert np.array_equal(gs["cls"], o["cls"]) and np.array_equal(gs["n_hits"], o["n_hits"])


def test_schwarzschild_disk_table1_scene(T, orc):
    """The scene of the paper's Table 1 (Sec. 4.3): Schwarzschild (a = 0) with the
    Novikov-Thorne disk, D = 100, 80 deg.  At a = 0 the root x_2 of Eq. (12)
    vanishes and its term of Eq. (11) is dropped; the redshift of Eq. (15) has
    no frame dragging.  Full 64^2 and ragged 45 x 37 images at the FP64 bar."""
    w = W.WORKLOADS["schwarzschild_disk_100"]
    for nx, ny in ((64, 64), (45, 37)):
        cam = dict(w["cameras"][0], nx=nx, ny=ny)
        say("case schwarzschild_disk_100", nx, ny, "fp64")
        g, o = full_image_parity(T, orc, w["a"], cam, w["disk"], w["solver"])
        assert (o["n_hits"] > 0).sum() > 0.1 * nx * ny
        assert (o["n_hits"] > 1).sum() > 0
        # the shading uses the a = 0 Page-Thorne form on every hit
        m = o["n_hits"] > 0
        assert np.all(g["hit_flux"][m, 0] > 0)


def test_schwarzschild_disk_table1_scene_mixed(T, orc):
    w = W.WORKLOADS["schwarzschild_disk_100"]
    cam = dict(w["cameras"][0], nx=64, ny=64)
    say("case schwarzschild_disk_100 64x64 mixed")
    g, o = full_image_parity(T, orc, w["a"], cam, w["disk"], w["solver"], precision=1, tol=MIXED_TOL, htol=None)
    assert g["n_fp32"].sum() > 0


@pytest.mark.parametrize("method", [1, 2], ids=["ck45", "rkf45"])
def test_six_stage_pairs_full_images(T, orc, method):
    """Cash-Karp and Fehlberg (Sec. 3.2) on the Schwarzschild shadow and a ragged
    Kerr image with the disk, against the oracle's same pair."""
    w = W.WORKLOADS["schwarzschild_64"]
    say("case schwarzschild_64 method", method)
    g, o = full_image_parity(T, orc, w["a"], w["cameras"][0], w["disk"], dict(w["solver"], method=method))
    assert np.mean(g["n_accept"] == o["n_accept"]) > 0.99
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=37, ny=29)
    say("case kerr09 37x29 method", method)
    g, o = full_image_parity(T, orc, w["a"], cam, w["disk"], dict(w["solver"], method=method))
    assert (o["n_hits"] > 0).sum() > 50
    # a different pair takes a different number of steps on the same image
    d = gpu_trace(T, w["a"], cam, w["disk"], w["solver"])
    assert not np.array_equal(d["n_accept"], g["n_accept"])


# ------------------------------------------------- Gragg-Bulirsch-Stoer
# The extrapolation's controller reading (Sec. 3.2 leaves it open): increments
# extrapolated, error components below their rounding floor taken as zero, the
# step factor rounded down to a power of two, so the step sequence does not
# depend on the rounding of the estimate; events are located on the method's
# own solution over the partial macro-step.  Parity is therefore held at the
# FP64 bar, with the step counts compared too.
GBS_NEAR_CAM = dict(r_obs=8.0, theta_obs=math.pi / 3, nx=24, ny=24, alpha_min=-5.0, alpha_max=5.0,
                    beta_min=-5.0, beta_max=5.0)


@pytest.mark.parametrize("h0_frac", [0.02, 0.1, 0.3, 1.0])
def test_extrapolation_first_macro_step(T, orc, h0_frac):
    """One macro-step (max_steps = 1) from a camera in the strong field (r = 8)
    and from the far camera: accept/reject and the state after it agree to
    1e-12 (the largest first step is rejected: the state stays put)."""
    disk = dict(r_in=0.0, r_out=20.0, max_hits=3)
    for cam in (GBS_NEAR_CAM, dict(W.WORKLOADS["kerr09_512"]["cameras"][0], nx=24, ny=24)):
        sv = dict(rtol=1e-8, atol=1e-10, h0_frac=h0_frac, horizon_factor=1.01, r_escape=1.1 * cam["r_obs"],
                  event_tol=1e-12, max_steps=1, method=3)
        say("case gbs one macro-step h0_frac", h0_frac, "r_obs", cam["r_obs"])
        g = gpu_trace(T, 0.9, cam, disk, sv)
        o = oracle_trace(orc, 0.9, cam, disk, sv)
        assert np.array_equal(g["n_accept"], o["n_accept"]) and np.array_equal(g["n_reject"], o["n_reject"])
        assert np.array_equal(g["cls"], o["cls"])
        d = np.abs(g["final_rtp"] - o["final_rtp"]) / np.maximum(1.0, np.abs(o["final_rtp"]))
        assert d.max() < 1e-12, d.max()
        # |H| after one step is at the rounding level of H itself (~1e-15)
        assert np.allclose(g["h_drift"], o["h_drift"], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("name,nx,ny,rtol", [("schwarzschild_64", 64, 64, 1e-8), ("kerr09_512", 37, 29, 1e-8),
                                             ("kerr09_512", 37, 29, 3e-10), ("schwarzschild_disk_100", 45, 37, 1e-8)])
def test_extrapolation_full_images(T, orc, name, nx, ny, rtol):
    """Gragg-Bulirsch-Stoer (Sec. 3.2) on the Schwarzschild shadow, a ragged
    Kerr image with the disk (config and gate tolerances) and the Table 1
    scene: the FP64 bar, and the same macro-steps as the oracle on every ray
    off the edge band."""
    w = W.WORKLOADS[name]
    cam = dict(w["cameras"][0], nx=nx, ny=ny)
    sv = dict(w["solver"], rtol=rtol, atol=rtol / 100, method=3)
    say("case gbs", name, nx, ny, rtol)
    g, o = full_image_parity(T, orc, w["a"], cam, w["disk"], sv)
    band = edge_band(class_key(o).reshape(ny, nx)).ravel()
    same = (g["n_accept"] == o["n_accept"]) & (g["n_reject"] == o["n_reject"])
    say("step counts identical on", same.mean(), "off band", same[~band].mean())
    # (an attempt whose estimate lies within rounding of 1 may still be
    # accepted on one side and rejected on the other: a rare extra attempt)
    assert same[~band].mean() >= 0.99
    # macro-steps: far fewer attempts per ray than the 5(4) pair needs
    d = gpu_trace(T, w["a"], cam, w["disk"], dict(sv, method=0))
    assert (g["n_accept"] + g["n_reject"]).mean() < 0.5 * (d["n_accept"] + d["n_reject"]).mean()


def test_extrapolation_kerr09_512_sampled(T, orc):
    """The 512^2 Kerr image with the disk at the gate tolerance, 200 sampled
    pixels and their neighbours, at the FP64 bar."""
    w = W.WORKLOADS["kerr09_512"]
    sv = dict(w["solver"], rtol=3e-10, atol=3e-12, method=3)
    say("case kerr09_512 gbs sampled")
    g, res = sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], sv, 0, 200, 5, FP64_TOL, FP64_HTOL)
    assert np.all(g["cls"] != 2)


# ---------------------------------------------------------- rendering variants
def test_opaque_disk_and_intrinsic_map(T, orc):
    """The optically thick disk (Sec. 2.3: the first crossing on the disk ends
    the ray, class ON_DISK) and the intrinsic map (Fig. KerrUHD b: flux F with
    the shift switched off), each on a ragged 61x47 spin-0.9 image, against
    the oracle at the FP64 bar."""
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=61, ny=47, theta_obs=75.0 * math.pi / 180)
    for extra in (dict(opaque=1), dict(shading=1), dict(opaque=1, shading=1)):
        disk = dict(w["disk"], **extra)
        say("case kerr09 61x47 disk", extra)
        g, o = full_image_parity(T, orc, w["a"], cam, disk, w["solver"])
        if extra.get("opaque"):
            on = o["cls"] == orc.ON_DISK
            assert on.sum() > 300 and np.array_equal(g["cls"] == 3, on)
            assert np.all(g["n_hits"][on] == 1)
            assert np.abs(np.cos(g["final_rtp"][on, 1])).max() < 1e-11
        if extra.get("shading"):
            m = g["n_hits"] > 0
            assert np.all(g["hit_flux"][m, 0] > 0) and np.all(g["hit_g"][m, 0] > 0)


# ------------------------------------------------------------------ Verlet
VERLET_CAM = dict(r_obs=100.0, theta_obs=math.pi / 3, nx=24, ny=24, alpha_min=-12.0, alpha_max=12.0,
                  beta_min=-12.0, beta_max=12.0)


def verlet_solver(h, horizon_factor):
    return dict(rtol=1e-8, atol=1e-10, h0_frac=h / VERLET_CAM["r_obs"], horizon_factor=horizon_factor,
                r_escape=1.1 * VERLET_CAM["r_obs"], event_tol=1e-12, max_steps=1000000, method=4)


def test_verlet_image_with_disk(T, orc):
    """Fixed-step Verlet (Sec. 3.2), h = 0.01, ~2e4 steps per ray, spin 0.9
    with the disk: no error control means no step decisions to disagree on,
    and the FP64 bar holds (the oracle's plain and FMA builds agree to 1e-12)."""
    disk = dict(r_in=0.0, r_out=20.0, max_hits=3)
    say("case verlet 24x24 h=0.01 stop 1.05 r+")
    g, o = full_image_parity(T, orc, 0.9, VERLET_CAM, disk, verlet_solver(0.01, 1.05))
    assert np.all(g["n_reject"] == 0) and np.array_equal(g["n_accept"], o["n_accept"])
    assert np.all(g["cls"] != 2) and (g["n_hits"] > 0).sum() > 100


def test_verlet_stage_without_solution_fails_the_ray(T, orc):
    """With the stop at 1.01 r_+ some captured rays reach radii where the
    implicit momentum stage has no solution near the current state for this
    step: they end FAILED on both sides, at the same state."""
    say("case verlet 24x24 h=0.01 stop 1.01 r+")
    sv = verlet_solver(0.01, 1.01)
    g = gpu_trace(T, 0.9, VERLET_CAM, None, sv)
    o = oracle_trace(orc, 0.9, VERLET_CAM, None, sv)
    assert (o["cls"] == 2).any()
    assert np.array_equal(g["cls"], o["cls"]) and np.array_equal(g["n_accept"], o["n_accept"])
    f = o["cls"] == 2
    assert np.abs(g["final_rtp"][f] / o["final_rtp"][f] - 1).max() < FP64_TOL


def test_single_pixel_and_single_row(T, orc):
    w = W.WORKLOADS["kerr09_512"]
    for nx, ny in ((1, 1), (17, 1), (1, 5)):
        cam = dict(w["cameras"][0], nx=nx, ny=ny)
        say("case kerr09", nx, ny)
        g = gpu_trace(T, w["a"], cam, w["disk"], w["solver"])
        o = oracle_trace(orc, w["a"], cam, w["disk"], w["solver"])
        assert np.array_equal(g["cls"], o["cls"]) and np.array_equal(g["n_hits"], o["n_hits"])
        m = o["n_hits"] > 0
        if m.any():
            assert np.abs(g["hit_r"][m, 0] / o["hit_r"][m, 0] - 1).max() < FP64_TOL


def test_max_steps_forces_failed(T, orc):
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=8, ny=8)
    sv = dict(w["solver"], max_steps=5)
    g = gpu_trace(T, w["a"], cam, w["disk"], sv)
    o = oracle_trace(orc, w["a"], cam, w["disk"], sv)
    assert np.all(g["cls"] == 2) and np.all(o["cls"] == 2)
    assert np.all(g["n_accept"] + g["n_reject"] == 5)
    assert np.array_equal(g["n_accept"], o["n_accept"])
    # After a fixed number of attempts the states sit at slightly different
    # affine parameters: the first error estimate (err ~ 1e-5) comes from a
    # ~1e9-fold cancellation in the phi component, so the step sizes of two
    # correct implementations differ at ~1e-7 relative.
    assert np.allclose(g["final_rtp"], o["final_rtp"], rtol=1e-5, atol=1e-9)


def test_kerr09_512_sampled_fp64(T, orc):
    w = W.WORKLOADS["kerr09_512"]
    say("case kerr09_512 fp64 sampled")
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"], 0, 300, 1, FP64_TOL, FP64_HTOL)


def test_launch_shape_invariance(T):
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=96, ny=80)
    ref = gpu_trace(T, w["a"], cam, w["disk"], w["solver"], launch=T.make_launch(order=T.ORDER_PIXEL))
    for bt, bpc, ch, rf, od in ((64, 1, 64, 1, T.ORDER_COST), (128, 0, 1024, 32, T.ORDER_PIXEL),
                                (256, 1, 96, 64, T.ORDER_COST), (256, 2, 4096, 8, T.ORDER_PIXEL),
                                (256, 0, 64, 4, T.ORDER_COST), (256, 0, 64, 4, T.ORDER_DEFAULT),
                                (256, 1, 1, 4, T.ORDER_TILE), (64, 2, 16, 1, T.ORDER_TILE)):
        say("launch", bt, bpc, ch, rf, od)
        g = gpu_trace(T, w["a"], cam, w["disk"], w["solver"], launch=T.make_launch(bt, bpc, ch, rf, od))
        for k in ref:
            assert np.array_equal(ref[k], g[k]), k


@pytest.mark.parametrize("method", [1, 2, 3, 4])
def test_launch_shape_invariance_other_methods(T, method):
    """Cash-Karp, Fehlberg, extrapolation and Verlet: the same bits for every
    launch shape and queue order (lanes share no arithmetic)."""
    w = W.WORKLOADS["kerr09_512"]
    if method == 4:
        cam, sv = VERLET_CAM, verlet_solver(0.05, 1.05)
    else:
        cam, sv = dict(w["cameras"][0], nx=72, ny=56), dict(w["solver"], method=method)
    ref = gpu_trace(T, w["a"], cam, w["disk"], sv, launch=T.make_launch(order=T.ORDER_PIXEL))
    for shape in ((64, 2, 16, 1, T.ORDER_COST), (256, 1, 1, 4, T.ORDER_TILE), (128, 0, 64, 8, T.ORDER_DEFAULT)):
        say("method", method, "launch", shape)
        g = gpu_trace(T, w["a"], cam, w["disk"], sv, launch=T.make_launch(*shape))
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (method, shape, k)


def test_launch_shape_invariance_mixed(T):
    """Mixed precision at rtol 1e-8, where most far-field attempts take FP32
    stages: the same bits for every launch shape and queue order (the regime
    is each ray's own decision, so a lane's neighbours never enter it)."""
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=72, ny=56)
    ref = gpu_trace(T, w["a"], cam, w["disk"], w["solver"], 1, launch=T.make_launch(order=T.ORDER_PIXEL))
    assert (ref["n_fp32"] > 0).mean() > 0.5
    for shape in ((64, 2, 16, 1, T.ORDER_COST), (256, 1, 1, 4, T.ORDER_TILE), (128, 0, 64, 8, T.ORDER_DEFAULT),
                  (256, 3, 1, 4, T.ORDER_COST)):
        say("mixed launch", shape)
        g = gpu_trace(T, w["a"], cam, w["disk"], w["solver"], 1, launch=T.make_launch(*shape))
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (shape, k)


def test_tile_order_ragged_cameras(T):
    """8 x 8 tile order on cameras whose sides are not multiples of 8 (edge
    tiles are smaller), three cameras in one trace: every pixel is traced once
    and gives the bits of pixel order."""
    w = W.WORKLOADS["kerr09_512"]
    cams = [dict(w["cameras"][0], nx=45, ny=29, theta_obs=t) for t in (0.6, 1.0, 1.4)]
    ref = gpu_trace(T, w["a"], cams, w["disk"], w["solver"], launch=T.make_launch(order=T.ORDER_PIXEL))
    for shape in ((256, 1, 1, 4, T.ORDER_TILE), (128, 0, 7, 2, T.ORDER_TILE)):
        g = gpu_trace(T, w["a"], cams, w["disk"], w["solver"], launch=T.make_launch(*shape))
        for k in ref:
            assert np.array_equal(ref[k], g[k]), k



def test_autotune_picks_a_valid_shape_with_identical_results(T):
    """The autotuner times candidate shapes; whatever it keeps must give the
    same bits as the default shape (results do not depend on the launch)."""
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=128, ny=112)
    ref = gpu_trace(T, w["a"], cam, w["disk"], w["solver"], launch=T.make_launch(256, 0, 64, 4, T.ORDER_PIXEL))
    out = T.alloc_outputs(cam["nx"] * cam["ny"])
    best = T.tartarus_autotune(T.make_metric(w["a"]), [T.make_camera(cam)], T.make_disk(w["disk"]),
                               T.make_solver(w["solver"]), out)
    say("tuned", best.block_threads, best.blocks_per_cu, best.chunk, best.refill_min, best.order)
    assert best.order in (T.ORDER_PIXEL, T.ORDER_COST, T.ORDER_TILE)
    assert best.block_threads in (64, 128, 256)
    assert best.blocks_per_cu >= 0 and best.chunk >= 1 and 1 <= best.refill_min <= 64
    tuned_out = T.to_numpy(out)
    again = gpu_trace(T, w["a"], cam, w["disk"], w["solver"])        # default launch = the tuned one
    for k in ref:
        assert np.array_equal(ref[k], tuned_out[k]), k
        assert np.array_equal(ref[k], again[k]), k

def test_integrator_timing_counts_the_integrator_launches(T):
    """Event timing of the integrator: one event pair per trace while enabled,
    none while disabled; the integrator launches take part of the time of the
    traces they belong to (ordering and finishing kernels are outside)."""
    import torch
    w = W.WORKLOADS["kerr09_512"]
    cam = dict(w["cameras"][0], nx=128, ny=96)
    args = (T.make_metric(w["a"]), [T.make_camera(cam)], T.make_disk(w["disk"]), T.make_solver(w["solver"]))
    out = T.alloc_outputs(cam["nx"] * cam["ny"])
    T.tartarus_trace(*args, out)
    torch.cuda.synchronize()
    T.tartarus_kernel_time()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    T.tartarus_kernel_timing(True)
    e0.record(st)
    for _ in range(3):
        T.tartarus_trace(*args, out)
    e1.record(st)
    torch.cuda.synchronize()
    T.tartarus_kernel_timing(False)
    ms, n = T.tartarus_kernel_time()
    say("integrator ms", ms, "launches", n, "traces ms", e0.elapsed_time(e1))
    assert n == 3
    assert 0.0 < ms <= e0.elapsed_time(e1) + 0.05
    T.tartarus_trace(*args, out)
    torch.cuda.synchronize()
    assert T.tartarus_kernel_time() == (0.0, 0)


# ------------------------------------------------------------------ tabulated metric
def test_table_build_matches_oracle(T, orc):
    import torch
    a = 0.7
    rp = orc.horizon(a)
    nr, nth, r_min, r_max = 64, 32, 1.1 * rp, 2000.0
    tab = torch.zeros(5 * nr * nth * 4, dtype=torch.float64, device="cuda")
    T.tartarus_build_kerr_table(a, nr, nth, r_min, r_max, tab)
    torch.cuda.synchronize()
    g = tab.cpu().numpy().reshape(5, nr, nth, 4)
    o = orc.build_kerr_table(a, nr, nth, r_min, r_max)
    big = np.abs(o).max(axis=(1, 2), keepdims=True)
    assert np.all(np.abs(g - o) <= 1e-13 * np.abs(o) + 1e-15 * big)


# ------------------------------------------------------------------ mixed precision
def test_mixed_small_full_image(T, orc):
    w = W.WORKLOADS["kerr0998_2048"]
    cam = dict(w["cameras"][0], nx=48, ny=41)
    say("case kerr0998 48x41 mixed")
    g, o = full_image_parity(T, orc, w["a"], cam, w["disk"], w["solver"], precision=1, tol=MIXED_TOL, htol=None)
    assert g["n_fp32"].sum() > 0.3 * (g["n_accept"] + g["n_reject"]).sum()


def test_kerr09_512_sampled_mixed(T, orc):
    w = W.WORKLOADS["kerr09_512"]
    say("case kerr09_512 mixed sampled")
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"], 1, 200, 2, MIXED_TOL)


def test_kerr0998_2048_sampled_fp64_and_mixed(T, orc):
    w = W.WORKLOADS["kerr0998_2048"]
    say("case kerr0998_2048 fp64 sampled")
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"], 0, 150, 3, FP64_TOL, FP64_HTOL)
    say("case kerr0998_2048 mixed sampled")
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"], 1, 150, 3, MIXED_TOL)


def test_gate_tolerance_fp64_sampled(T, orc):
    """The benchmark's tolerance (rtol 3e-10): parity and the |H| <= 1e-8 gate."""
    w = W.WORKLOADS["kerr09_512"]
    sv = dict(w["solver"], rtol=3e-10, atol=3e-12)
    say("case kerr09_512 fp64 rtol 3e-10 sampled")
    g, res = sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], sv, 0, 120, 4, FP64_TOL, FP64_HTOL)
    assert g["h_gate"][g["cls"] != 2].max() <= 1e-8


def test_headline_configuration_sampled(T, orc):
    """The benchmark's headline as it is timed: the 2048^2 a = 0.998 image at
    rtol 7e-11 (the loosest listed tolerance whose |H| <= 1e-8 gate holds) in
    the launch shape of the committed profile (256 threads x 3 blocks per CU,
    chunk 1, refill at 4 idle lanes, cost order); 120 sampled pixels with their
    neighbours at the FP64 bar, and the gate on every ray of the image."""
    w = W.WORKLOADS["kerr0998_2048"]
    sv = dict(w["solver"], rtol=7e-11, atol=7e-13)
    launch = T.make_launch(256, 3, 1, 4, T.ORDER_COST)
    say("case kerr0998_2048 fp64 rtol 7e-11 bench launch sampled")
    g = gpu_trace(T, w["a"], w["cameras"][0], w["disk"], sv, launch=launch)
    assert np.all(g["cls"] != 2)
    assert g["h_gate"].max() <= 1e-8
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], sv, 0, 120, 6, FP64_TOL, FP64_HTOL, g=g)


@pytest.mark.parametrize("method", [1, 2], ids=["ck45", "rkf45"])
def test_six_stage_pairs_kerr09_512_sampled(T, orc, method):
    """Cash-Karp and Fehlberg on the full 512^2 Kerr image with the disk, as the
    benchmark's legs trace it; 150 sampled pixels with their neighbours."""
    w = W.WORKLOADS["kerr09_512"]
    say("case kerr09_512 sampled method", method)
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], dict(w["solver"], method=method), 0, 150, 7 + method,
                   FP64_TOL, FP64_HTOL)


def test_osiris_and_table1_scenes_sampled(T, orc):
    """The paper's calibration scene (a = 0.98, edge-on, 1024^2, no disk) and its
    Table 1 scene (Schwarzschild with the disk, D = 100) at 2048^2, as the
    benchmark's legs trace them; sampled pixels with their neighbours."""
    w = W.WORKLOADS["osiris_1024"]
    say("case osiris_1024 sampled")
    sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"], 0, 150, 10, FP64_TOL, FP64_HTOL)
    w = W.scaled("schwarzschild_disk_100", 2048)
    say("case schwarzschild_disk_100 2048 sampled")
    g, res = sampled_parity(T, orc, w["a"], w["cameras"][0], w["disk"], w["solver"], 0, 150, 11, FP64_TOL, FP64_HTOL)
    assert res["hit_r"]["n"] >= 10   # the disk is seen in about one sample in seven


# ------------------------------------------------------------------ tabulated metric traces
def gpu_table(T, a, nr, nth, r_min, r_max):
    import torch
    tab = torch.zeros(5 * nr * nth * 4, dtype=torch.float64, device="cuda")
    T.tartarus_build_kerr_table(a, nr, nth, r_min, r_max, tab)
    torch.cuda.synchronize()
    return tab


def c5_setup(orc):
    w = W.WORKLOADS["tabulated07_64cams"]
    a, t = w["a"], w["table"]
    rp = orc.horizon(a)
    return w, a, t["nr"], t["nth"], t["r_min_over_rplus"] * rp, t["r_max"]


def test_tabulated_small_vs_oracle(T, orc):
    w, a, nr, nth, r_min, r_max = c5_setup(orc)
    tab_g = gpu_table(T, a, nr, nth, r_min, r_max)
    tab_o = orc.build_kerr_table(a, nr, nth, r_min, r_max)
    cam = dict(w["cameras"][20], nx=30, ny=23)
    say("case tabulated 30x23 fp64")
    g = gpu_trace(T, a, cam, w["disk"], w["solver"], table=(tab_g, nr, nth, r_min, r_max))
    o = oracle_trace(orc, a, cam, w["disk"], w["solver"], table=(tab_o, nr, nth, r_min, r_max))
    band = edge_band(class_key(o).reshape(cam["ny"], cam["nx"])).ravel()
    res = compare(g, o, band, TAB_TOL)
    say(res)
    assert_parity(res, TAB_TOL, TAB_HTOL)


def test_tabulated_vs_analytic_on_gpu(T, orc):
    """The tabulated path against the analytic path: identical classes off the
    band, emission radius and redshift within the interpolation error (~1e-6)."""
    w, a, nr, nth, r_min, r_max = c5_setup(orc)
    tab = gpu_table(T, a, nr, nth, r_min, r_max)
    cam = dict(w["cameras"][40], nx=64, ny=64)
    gt = gpu_trace(T, a, cam, w["disk"], w["solver"], table=(tab, nr, nth, r_min, r_max))
    ga = gpu_trace(T, a, cam, w["disk"], w["solver"])
    band = edge_band(class_key(ga).reshape(64, 64)).ravel()
    res = compare(gt, ga, band, 1e-5)
    say(res)
    assert res["class_mismatch_off_band"] == 0
    assert res["hit_r"]["max"] < 1e-5 and res["hit_g"]["max"] < 1e-5


def test_launch_shape_invariance_tabulated(T, orc):
    """The tabulated integrator on three ragged cameras: the same bits for every
    launch shape and queue order (each lane gathers its own table cells and
    shares no arithmetic with its neighbours)."""
    w, a, nr, nth, r_min, r_max = c5_setup(orc)
    tab = gpu_table(T, a, nr, nth, r_min, r_max)
    cams = [dict(w["cameras"][c], nx=53, ny=37) for c in (5, 31, 58)]
    say("case tabulated launch shapes, 3 cameras 53x37")
    ref = gpu_trace(T, a, cams, w["disk"], w["solver"], table=(tab, nr, nth, r_min, r_max),
                    launch=T.make_launch(order=T.ORDER_PIXEL))
    assert (ref["n_hits"] > 0).any() and (ref["cls"] == 1).any()
    for shape in ((64, 2, 16, 1, T.ORDER_COST), (256, 1, 1, 4, T.ORDER_TILE), (128, 0, 64, 8, T.ORDER_DEFAULT),
                  (256, 2, 1, 4, T.ORDER_PIXEL)):
        say("tabulated launch", shape)
        g = gpu_trace(T, a, cams, w["disk"], w["solver"], table=(tab, nr, nth, r_min, r_max),
                      launch=T.make_launch(*shape))
        for k in ref:
            assert np.array_equal(ref[k], g[k]), (shape, k)


def test_tabulated_64_cameras_sampled(T, orc):
    """All 64 cameras (512^2 each) in one launch, in the launch shape the
    benchmark times (256 threads x 2 blocks per CU, pixel order); 400 sampled
    pixels and their 8 neighbours traced by the oracle.  Classes must be
    identical off the edge band (a sample with a neighbour of another oracle
    class); every class difference must lie in that band; values on matching
    off-band samples within the tabulated bar."""
    w, a, nr, nth, r_min, r_max = c5_setup(orc)
    tab_g = gpu_table(T, a, nr, nth, r_min, r_max)
    tab_o = orc.build_kerr_table(a, nr, nth, r_min, r_max)
    cams = w["cameras"]
    say("case tabulated 64 cameras x 512^2 fp64")
    g = gpu_trace(T, a, cams, w["disk"], w["solver"], table=(tab_g, nr, nth, r_min, r_max),
                  launch=T.make_launch(256, 2, 1, 4, T.ORDER_PIXEL))
    nx = ny = 512
    per = nx * ny
    nsample = 400
    rng = np.random.default_rng(5)
    cc = rng.integers(0, len(cams), nsample)
    ii, jj = rng.integers(1, nx - 1, nsample), rng.integers(1, ny - 1, nsample)
    ids = np.array([c * per + (j + dj) * nx + (i + di) for c, i, j in zip(cc, ii, jj)
                    for dj in (-1, 0, 1) for di in (-1, 0, 1)], dtype=np.int64)
    uniq, inv = np.unique(ids, return_inverse=True)
    o_u = orc.trace(orc.make_metric(a, tab_o, nr, nth, r_min, r_max), [orc.make_camera(c) for c in cams],
                    orc.make_disk(w["disk"]), orc.make_solver(w["solver"]), ray_ids=uniq)
    key9 = class_key(o_u)[inv].reshape(nsample, 9)
    band = np.any(key9 != key9[:, 4:5], axis=1)
    centre = inv.reshape(nsample, 9)[:, 4]
    o = {k: v[centre] for k, v in o_u.items()}
    gs = {k: v[uniq[centre]] for k, v in g.items()}
    res = compare(gs, o, band, TAB_TOL)
    say(res)
    mism = class_key(gs) != class_key(o)
    say("band", int(band.sum()), "class differences", int(mism.sum()), "of which in the band", int((mism & band).sum()))
    assert not np.any(mism & ~band), np.flatnonzero(mism & ~band)
    assert_parity(res, TAB_TOL, TAB_HTOL)
    assert np.all(g["cls"] != 2)
