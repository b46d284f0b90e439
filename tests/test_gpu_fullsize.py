"""Parity at the workloads' full sizes, in the configuration bench.py times
(needs an MI355X); also both hoods at full size, and shuffled input.

Each of the five workloads is drawn at its full size (2^16 to 4.4e8 points)
and solved through the C ABI with the default plan (the one bench.py uses);
the result is compared index for index with the CPU oracle on every set --
the oracle is linear-time, so no sampling is needed -- and the invariants
of the strict hood are checked on a sample of sets.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import invariants

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1203_5004_amd as uh  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    uh.load_library()


@pytest.mark.parametrize("name", list(synth.WORKLOADS))
def test_full_size_workload(name):
    pts, off = synth.WORKLOADS[name][0]()
    S, N = len(off) - 1, int(off[-1])
    print(f"[fullsize] {name}: {N} points, {S} sets", flush=True)
    plan = uh.upper_hull_plan_create(off)
    d = torch.from_numpy(pts).cuda()
    out = torch.empty(N, dtype=torch.int32, device="cuda")
    cnt = torch.empty(S, dtype=torch.int32, device="cuda")
    stats = uh.new_stats(S)
    plan.run(d, out, cnt, stats)
    torch.cuda.synchronize()
    got_cnt = cnt.cpu().numpy()
    got = out.cpu().numpy()
    st = stats.cpu().numpy()
    plan.close()
    del d, out
    ref_out, ref_cnt = oracle.upper_hull_batched(pts, off)
    assert np.array_equal(got_cnt, ref_cnt.astype(np.int32))
    for s in range(S):
        a, c = int(off[s]), int(got_cnt[s])
        assert np.array_equal(got[a:a + c], ref_out[a:a + c]), f"set {s}"
    for s in np.linspace(0, S - 1, min(S, 8)).astype(int):
        a, b = int(off[s]), int(off[s + 1])
        if b - a <= (1 << 24):
            assert invariants.check(pts[a:b], got[a:a + got_cnt[s]]) == []
    assert np.all(st[:, 1] <= st[:, 0])
    print(f"[fullsize] {name}: corners {int(got_cnt.sum())}, orient tests "
          f"{int(st[:, 0].sum())}, fallbacks {int(st[:, 1].sum())}", flush=True)


@pytest.mark.parametrize("name", list(synth.WORKLOADS))
def test_full_size_both_hoods(name):
    pts, off = synth.WORKLOADS[name][0]()
    S, N = len(off) - 1, int(off[-1])
    print(f"[fullsize] {name}, both hoods: {N} points, {S} sets", flush=True)
    plan = uh.upper_hull_plan_create(off, flags=uh.UH_FLAG_BOTH_HOODS)
    d = torch.from_numpy(pts).cuda()
    out = torch.empty(2 * N, dtype=torch.int32, device="cuda")
    cnt = torch.empty(2 * S, dtype=torch.int32, device="cuda")
    plan.run(d, out, cnt)
    torch.cuda.synchronize()
    got_cnt = cnt.cpu().numpy()
    got = out.cpu().numpy()
    plan.close()
    del d, out
    for half, fn in ((0, oracle.upper_hull_batched), (1, oracle.lower_hull_batched)):
        ref_out, ref_cnt = fn(pts, off)
        assert np.array_equal(got_cnt[half * S:(half + 1) * S], ref_cnt.astype(np.int32)), half
        for s in range(S):
            a, c = int(off[s]), int(got_cnt[half * S + s])
            assert np.array_equal(got[half * N + a:half * N + a + c], ref_out[a:a + c]), (half, s)
        del ref_out


# shuffled input at full size: the arc (the oracle's host sort of 2^27 points
# alone takes most of a minute; bench.py --unsorted checks that size)
@pytest.mark.parametrize("name", ["arc_2^24"])
def test_full_size_unsorted(name):
    pts, off = synth.WORKLOADS[name][0]()
    N = int(off[-1])
    pts = pts[np.random.default_rng(20350).permutation(N)]
    print(f"[fullsize] {name}, shuffled: {N} points", flush=True)
    plan = uh.upper_hull_plan_create(off, flags=uh.UH_FLAG_UNSORTED)
    d = torch.from_numpy(pts).cuda()
    out = torch.empty(N, dtype=torch.int32, device="cuda")
    cnt = torch.empty(1, dtype=torch.int32, device="cuda")
    plan.run(d, out, cnt)
    torch.cuda.synchronize()
    c = int(cnt.item())
    got = out[:max(c, 0)].cpu().numpy()
    plan.close()
    del d, out
    rc, ref = oracle.unsorted_hull(pts, "upper")
    assert rc == 0 and c == len(ref) and np.array_equal(got, ref)
