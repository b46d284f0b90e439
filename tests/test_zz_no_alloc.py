"""upper_hull_noalloc: the upper hood in the library's fixed per-device
scratch, for callers that cannot allocate (needs an MI355X).

Its results are compared index for index with the existing entry point
upper_hull (which uses a workspace) and with the CPU oracle, on two calls in
a row, the second with a smaller input; at the maximum size; above it (a
clear error, nothing enqueued); with free device memory unchanged over the
calls; and replayed from a captured graph.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1203_5004_amd as uh  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uh.load_library()


def _both(xy):
    """(noalloc result, upper_hull result) for the same points, as numpy."""
    n = len(xy)
    pts = torch.from_numpy(np.ascontiguousarray(xy)).cuda()
    a_idx = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    a_cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    b_idx = torch.full((max(n, 1),), -9, dtype=torch.int32, device="cuda")
    b_cnt = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    uh.upper_hull_noalloc(pts, a_idx, a_cnt)
    uh.upper_hull(pts, b_idx, b_cnt)
    torch.cuda.synchronize()
    ca, cb = int(a_cnt.item()), int(b_cnt.item())
    return (ca, a_idx[:max(ca, 0)].cpu().numpy()), (cb, b_idx[:max(cb, 0)].cpu().numpy())


def _check(xy, what):
    (ca, ia), (cb, ib) = _both(xy)
    ref = oracle.upper_hull(xy)
    assert ca == cb == len(ref), (what, ca, cb, len(ref))
    assert np.array_equal(ia, ib), what
    assert np.array_equal(ia, ref), what


def test_two_calls_in_a_row_second_smaller():
    # a large hull first (several merge passes), then a smaller uniform set:
    # the second call must not see anything the first left in the scratch
    _check(synth.arc(1_500_001, 24, 4, seed=31), "arc 1.5M")
    _check(synth.uniform(70_001, 20, seed=32), "uniform 70001")
    _check(synth.parabola(5_000, 20, 1, seed=33), "parabola 5000")


def test_maximum_size_and_edge_sizes():
    n = uh.UH_NOALLOC_MAX_N
    _check(synth.uniform_iid(n, 27, seed=34), "uniform_iid max n")  # equal-x runs
    _check(synth.arc(n, 24, 4, seed=35), "arc max n")
    for n in (0, 1, 2, 1023, 1024, 1025):
        xy = synth.uniform(n, 20, seed=36 + n) if n else np.zeros((0, 2), np.float32)
        _check(xy, f"n={n}")


def test_data_error_then_clean_data():
    xy = synth.uniform(50_000, 20, seed=40)
    bad = xy.copy()
    bad[30_000, 0] = bad[29_990, 0]  # x decreases
    (ca, _), (cb, _) = _both(bad)
    assert ca == cb == uh.UH_ERR_UNSORTED
    _check(xy, "clean after an error")


def test_above_the_maximum_is_refused_and_enqueues_nothing():
    lib = uh.load_library()
    n = uh.UH_NOALLOC_MAX_N + 1
    pts = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.upper_hull_noalloc(ctypes.c_void_p(pts.data_ptr()), n,
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), s)
    assert rc == uh.UH_ERR_TOO_LARGE
    assert uh.upper_hull_status_string(rc) != "unknown status"
    torch.cuda.synchronize()
    assert int(cnt.item()) == -7
    rc = lib.upper_hull_noalloc(ctypes.c_void_p(pts.data_ptr()), -1,
                                ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(cnt.data_ptr()), s)
    assert rc == uh.UH_ERR_ARG


def test_free_memory_unchanged_over_calls():
    sizes = [2_000_000, 1, 0, 777_777, 4096, 1_048_577, 65_536]
    nmax = max(sizes)
    pts = torch.empty((nmax, 2), dtype=torch.float32, device="cuda")
    out = torch.empty(nmax, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    inputs = {n: synth.arc(n, 24, 4, seed=n) if n > 1 else np.full((n, 2), 0.5, np.float32)
              for n in sizes}
    uh.upper_hull_noalloc(pts[:1], out, cnt)  # the device's first call looks the scratch up
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for n in sizes:
        pts[:n].copy_(torch.from_numpy(inputs[n]))
        uh.upper_hull_noalloc(pts[:n], out, cnt)
        torch.cuda.synchronize()
        ref = oracle.upper_hull(inputs[n])
        c = int(cnt.item())
        assert c == len(ref), (n, c, len(ref))
        assert np.array_equal(out[:c].cpu().numpy(), ref), n
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0


def test_graph_replay():
    n = 600_001
    pts = torch.from_numpy(synth.arc(n, 24, 4, seed=50)).cuda()
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    uh.upper_hull_noalloc(pts, out, cnt)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        uh.upper_hull_noalloc(pts, out, cnt)
    for rep, seed in enumerate([51, 52, 51, 53]):
        xy = synth.arc(n, 24, 4, seed=seed) if seed % 2 else synth.uniform(n, 24, seed=seed)
        pts.copy_(torch.from_numpy(xy))
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        del junk
        ref = oracle.upper_hull(xy)
        c = int(cnt.item())
        assert c == len(ref), (rep, c, len(ref))
        assert np.array_equal(out[:c].cpu().numpy(), ref), rep
