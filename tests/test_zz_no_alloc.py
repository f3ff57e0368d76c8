"""The allocation-free trace (tartarus_trace_noalloc) through the C ABI, against
tartarus_trace_launch with the same arguments and launch shape: two calls in a
row, the second on a smaller input (three ragged cameras), each bit-identical
(same kernels; the working memory is the library's fixed per-device array
instead of allocated buffers).  Requests beyond the array are refused."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_08989_amd import tartarus as T
    T.tartarus_init(0, 0)
    return T


def test_noalloc_matches_trace_on_two_calls(T):
    import torch
    w = W.WORKLOADS["kerr09_512"]
    for nx, ny, thetas in ((300, 200, (1.0,)), (97, 61, (1.0, 0.7, 1.3))):
        cams = [dict(w["cameras"][0], nx=nx, ny=ny, theta_obs=t) for t in thetas]
        args = (T.make_metric(w["a"]), [T.make_camera(c) for c in cams], T.make_disk(w["disk"]),
                T.make_solver(w["solver"]))
        launch = T.make_launch(256, 1, 1, 4, T.ORDER_COST)
        n = nx * ny * len(cams)
        print("case noalloc", nx, ny, len(cams), flush=True)
        ref, out = T.alloc_outputs(n), T.alloc_outputs(n)
        T.tartarus_trace(*args, ref, launch=launch)
        T.tartarus_trace_noalloc(*args, out, launch=launch)
        torch.cuda.synchronize()
        a, b = T.to_numpy(ref), T.to_numpy(out)
        assert (a["n_hits"] > 0).sum() > 100
        for k in a:
            assert np.array_equal(a[k], b[k]), k


def test_noalloc_refuses_what_does_not_fit(T):
    w = W.WORKLOADS["kerr09_512"]
    big = dict(w["cameras"][0], nx=513, ny=512)
    with pytest.raises(T.TartarusError) as e:
        T.tartarus_trace_noalloc(T.make_metric(w["a"]), [T.make_camera(big)], T.make_disk(w["disk"]),
                                 T.make_solver(w["solver"]), T.alloc_outputs(1))
    assert e.value.code == T.E_TOO_LARGE
