"""The boundary's workspace, capture, status and cache behaviour (needs an
MI355X).  Every result is compared index for index with the CPU oracle.

* With a caller workspace set, the single-set calls allocate nothing: a call
  for a size never seen before is captured into a graph in a fresh process and
  replayed, and free device memory stays the same over 100 calls of 100
  distinct sizes.
* A plan (single set and batched) run on data with an error and then on clean
  data of the same layout gives the oracle's result the second time.
* Stats report rounds and status; x just below 0 is a range error.
* The plan-less batched call's cache of layouts is used from two threads with
  more layouts than it holds.
"""
import os
import subprocess
import sys
import threading

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1203_5004_amd as uh  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uh.load_library()


@pytest.fixture
def no_user_workspace():
    yield
    uh.upper_hull_set_workspace(None)
    torch.cuda.synchronize()


def _dev(xy):
    return torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)).cuda()


def _points(n, seed):
    G = 20 if n <= (1 << 19) else 24  # room for n distinct x
    kind = seed % 3
    if kind == 0:
        return synth.uniform(n, G, seed=seed)
    if kind == 1:
        return synth.arc(n, G, 4, seed=seed)
    return synth.parabola(n, G, 1, seed=seed)


CAPTURE_SCRIPT = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import oracle, synth
import paper_1203_5004_amd as uh

n = int(sys.argv[2])
ws = torch.empty(uh.upper_hull_workspace_bytes(n, 1), dtype=torch.uint8, device="cuda")
uh.upper_hull_set_workspace(ws)
xy0 = synth.arc(n, 20, 4, seed=77)
pts = torch.from_numpy(xy0).cuda()
out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
g = torch.cuda.CUDAGraph()
with torch.cuda.graph(g):       # this process has never run the library before
    uh.upper_hull(pts, out, cnt)
torch.cuda.synchronize()
for rep, seed in enumerate([77, 5, 77, 9]):
    xy = synth.arc(n, 20, 4, seed=seed) if seed % 2 else synth.uniform(n, 20, seed=seed)
    pts.copy_(torch.from_numpy(xy))           # new input, same buffer
    junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
    g.replay()
    torch.cuda.synchronize()
    c = int(cnt.item())
    ref = oracle.upper_hull(xy)
    assert c == len(ref), (rep, c, len(ref))
    assert np.array_equal(out[:c].cpu().numpy(), ref), rep
print("captured replays ok", n, flush=True)
"""


def test_capture_of_a_never_seen_size_in_a_fresh_process():
    n = 300_007  # not a power of two, several merge passes
    r = subprocess.run([sys.executable, "-c", CAPTURE_SCRIPT, ROOT, str(n)],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "captured replays ok" in r.stdout


def test_no_allocation_over_100_distinct_sizes(no_user_workspace):
    rng = np.random.default_rng(2024)
    sizes = sorted(set(int(v) for v in rng.integers(0, 1 << 20, 120)))[:100]
    sizes[0], sizes[1], sizes[2] = 0, 1, 1025  # empty, one point, just over a tile
    nmax = max(sizes)
    ws = torch.empty(uh.upper_hull_workspace_bytes(nmax, 1), dtype=torch.uint8, device="cuda")
    uh.upper_hull_set_workspace(ws)
    pts_all = torch.empty((nmax, 2), dtype=torch.float32, device="cuda")
    out = torch.empty(max(nmax, 1), dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    inputs = {n: _points(n, n) if n else np.zeros((0, 2), np.float32) for n in sizes}
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for n in sizes:
        xy = inputs[n]
        if n:
            pts_all[:n].copy_(torch.from_numpy(xy))
        uh.upper_hull(pts_all[:n], out, cnt)
        torch.cuda.synchronize()
        c = int(cnt.item())
        ref = oracle.upper_hull(xy)
        assert c == len(ref), (n, c, len(ref))
        assert np.array_equal(out[:c].cpu().numpy(), ref), n
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)


def test_workspace_sized_for_each_call_is_enough(no_user_workspace):
    # the bound holds at the fan-in thresholds and for the convex hull's two hoods
    for n in (1024, 1025, 65536, 2047 * 1024 + 1, 2048 * 1024, 2 * 1024 * 1024 + 5):
        xy = _points(n, n)
        ws = torch.empty(uh.upper_hull_workspace_bytes(n, 1), dtype=torch.uint8, device="cuda")
        uh.upper_hull_set_workspace(ws)
        idx, cnt = uh.upper_hull(_dev(xy))
        torch.cuda.synchronize()
        assert np.array_equal(idx[:int(cnt.item())].cpu().numpy(), oracle.upper_hull(xy)), n
        ws2 = torch.empty(uh.upper_hull_workspace_bytes(2 * n, 2), dtype=torch.uint8,
                          device="cuda")
        uh.upper_hull_set_workspace(ws2)
        idx, cnt = uh.convex_hull(_dev(xy))
        torch.cuda.synchronize()
        assert np.array_equal(idx[:int(cnt.item())].cpu().numpy(), oracle.convex_hull(xy)), n
        uh.upper_hull_set_workspace(None)
        del ws, ws2


def test_workspace_too_small_enqueues_nothing(no_user_workspace):
    n = 100_000
    ws = torch.empty(uh.upper_hull_workspace_bytes(n // 4, 1), dtype=torch.uint8, device="cuda")
    uh.upper_hull_set_workspace(ws)
    pts = _dev(_points(n, 3))
    out = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="workspace"):
        uh.upper_hull(pts, out, cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == -7
    # convex_hull counts two sets of n points
    ws2 = torch.empty(uh.upper_hull_workspace_bytes(n, 1), dtype=torch.uint8, device="cuda")
    uh.upper_hull_set_workspace(ws2)
    with pytest.raises(RuntimeError, match="workspace"):
        uh.convex_hull(pts, out, cnt)


def test_set_workspace_argument_errors(no_user_workspace):
    lib = uh.load_library()
    import ctypes
    assert lib.upper_hull_set_workspace(ctypes.c_void_p(0), 64) == uh.UH_ERR_ARG
    buf = torch.empty(4096, dtype=torch.uint8, device="cuda")
    assert lib.upper_hull_set_workspace(ctypes.c_void_p(buf.data_ptr() + 8), 1024) == uh.UH_ERR_ARG


def test_library_workspace_is_not_grown_during_capture(no_user_workspace):
    s = torch.cuda.Stream()
    n_big = 3_000_001  # larger than anything this stream's workspace has held
    pts = _dev(_points(n_big, 1))
    out = torch.empty(n_big, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    g = torch.cuda.CUDAGraph()
    raised = []
    try:
        with torch.cuda.graph(g, stream=s):
            try:
                uh.upper_hull(pts, out, cnt)
            except RuntimeError as e:
                raised.append(str(e))
    except Exception:
        pass  # an empty capture may be rejected by torch; the refusal is what is tested
    torch.cuda.synchronize()
    assert raised and "capturing" in raised[0]


# ---------------------------------------------------------------- statuses
def test_error_then_clean_data_on_the_same_plans():
    for n, S in ((50_000, 1), (30_000, 5)):
        rng = np.random.default_rng(n)
        sizes = [n // S + (7 * k) for k in range(S)]
        sets = [_points(m, 40 + k) for k, m in enumerate(sizes)]
        pts, off = synth.concat_sets(sets)
        bad = pts.copy()
        for s in range(S):  # an error in the middle of a multi-tile set
            a, b = int(off[s]), int(off[s + 1])
            bad[int(rng.integers(a + 2000, b - 2000)), 0] = np.float32(1.5)
        plan = uh.upper_hull_plan_create(off)
        batched_off = off
        out = torch.full((len(pts),), -7, dtype=torch.int32, device="cuda")
        cnt = torch.full((S,), -7, dtype=torch.int32, device="cuda")
        for data, expect_error in ((bad, True), (pts, False), (bad, True), (pts, False)):
            for run in ("plan", "batched"):
                out.fill_(-7)
                cnt.fill_(-7)
                if run == "plan":
                    plan.run(_dev(data), out, cnt)
                else:
                    uh.upper_hull_batched(_dev(data), batched_off, out, cnt)
                torch.cuda.synchronize()
                c = cnt.cpu().numpy()
                if expect_error:
                    assert np.all(c == uh.UH_ERR_RANGE), (run, c)
                    continue
                ref_out, ref_cnt = oracle.upper_hull_batched(data, off)
                assert np.array_equal(c, ref_cnt.astype(np.int32)), (run, c)
                o = out.cpu().numpy()
                for s in range(S):
                    a = int(off[s])
                    assert np.array_equal(o[a:a + c[s]], ref_out[a:a + c[s]]), (run, s)
        plan.close()


def test_single_set_call_error_then_clean():
    xy = _points(70_000, 2)
    bad = xy.copy()
    bad[33_333, 1] = np.float32(3 * 2 ** -31)  # off the grid
    for data in (bad, xy, bad, xy):
        idx, cnt = uh.upper_hull(_dev(data))
        torch.cuda.synchronize()
        rc, ref = oracle.upper_hull_status(data)
        c = int(cnt.item())
        if rc:
            assert c == rc
        else:
            assert c == len(ref) and np.array_equal(idx[:c].cpu().numpy(), ref)


@pytest.mark.parametrize("xbad", [-2.0 ** -30, -2.0 ** -25, -0.25, 1.0 + 2.0 ** -23])
@pytest.mark.parametrize("where", [0, 1, 700, 4096, 9999])
def test_x_just_outside_the_range(xbad, where):
    n = 10_000
    xy = synth.uniform(n, 20, seed=where + 1)
    xy = xy.copy()
    xy[where if xbad < 0 else n - 1, 0] = np.float32(xbad)
    rc, _ = oracle.upper_hull_status(xy)
    assert rc < 0
    idx, cnt = uh.upper_hull(_dev(xy))
    torch.cuda.synchronize()
    # a point below 0 after a valid one is also a decrease of x; the range
    # error takes precedence, as in the oracle's check of that point
    assert int(cnt.item()) == rc == uh.UH_ERR_RANGE
    # in any order: the device sort puts it first or last; always a range error
    plan = uh.upper_hull_plan_create([0, n], flags=uh.UH_FLAG_UNSORTED)
    perm = np.random.default_rng(where).permutation(n)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    cnt2 = torch.empty(1, dtype=torch.int32, device="cuda")
    plan.run(_dev(xy[perm]), out, cnt2)
    torch.cuda.synchronize()
    urc, _ = oracle.unsorted_hull(xy[perm])
    assert int(cnt2.item()) == urc == uh.UH_ERR_RANGE
    plan.close()


def test_stats_rounds_and_status():
    sizes = [0, 1, 16, 17, 1024, 1025, 5000, 70_001]
    sets = [_points(m, 10 + k) if m else np.zeros((0, 2), np.float32)
            for k, m in enumerate(sizes)]
    pts, off = synth.concat_sets(sets)
    pts = pts.copy()
    pts[int(off[6]) + 77, 1] = np.float32(1.5)  # set 6: a range error
    S = len(sizes)
    for strip in (8, 16):
        plan = uh.upper_hull_plan_create(off, strip=strip)
        out = torch.empty(len(pts), dtype=torch.int32, device="cuda")
        cnt = torch.empty(S, dtype=torch.int32, device="cuda")
        st = uh.new_stats(S)
        plan.run(_dev(pts), out, cnt, st)
        torch.cuda.synchronize()
        d = uh.decode_stats(st.cpu().numpy())
        c = cnt.cpu().numpy()
        for s, m in enumerate(sizes):
            strips = -(-m // strip)
            want = int(np.ceil(np.log2(strips))) if strips > 1 else 0
            assert d["rounds"][s] == want, (strip, s, m, d["rounds"][s])
            assert d["status"][s] == (uh.UH_ERR_RANGE if s == 6 else 0), s
            assert c[s] == (uh.UH_ERR_RANGE if s == 6 else len(oracle.upper_hull(sets[s])))
        plan.close()


# ---------------------------------------------------------------- plan cache
def test_batched_layout_cache_from_two_threads():
    # more layouts than the cache holds (8), used from two threads at once,
    # each thread on its own stream, so layouts are dropped while the other
    # thread's runs may be in flight; every result must match the oracle
    layouts = []
    for k in range(12):
        sizes = [3000 + 997 * k, 5 + k, 20_000 + 13 * k]
        sets = [_points(m, 100 * k + j) for j, m in enumerate(sizes)]
        layouts.append(synth.concat_sets(sets))
    errors = []

    def worker(order, seed):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for rep in range(3):
                    for k in order:
                        pts, off = layouts[k]
                        out = torch.empty(len(pts), dtype=torch.int32, device="cuda")
                        cnt = torch.empty(len(off) - 1, dtype=torch.int32, device="cuda")
                        uh.upper_hull_batched(_dev(pts), off, out, cnt, stream=s)
                        s.synchronize()
                        ref_out, ref_cnt = oracle.upper_hull_batched(pts, off)
                        c = cnt.cpu().numpy()
                        if not np.array_equal(c, ref_cnt.astype(np.int32)):
                            errors.append(("counts", k, rep))
                            continue
                        o = out.cpu().numpy()
                        for j in range(len(off) - 1):
                            a = int(off[j])
                            if not np.array_equal(o[a:a + c[j]], ref_out[a:a + c[j]]):
                                errors.append(("idx", k, j, rep))
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    # disjoint layouts: calls with one layout share its plan's workspace
    t1 = threading.Thread(target=worker, args=(list(range(6)), 1))
    t2 = threading.Thread(target=worker, args=(list(range(6, 12)), 2))
    t1.start()
    t2.start()
    t1.join(timeout=240)
    t2.join(timeout=240)
    assert not t1.is_alive() and not t2.is_alive()
    assert not errors, errors[:5]
