"""Per-level parity of the merge tree with the oracle (needs an MI355X), the
paper's per-stage state: after every round, each block holds the hood of its
own points (the stage loop's invariant that show_current_hoods printed).

* With UH_FLAG_NO_ELIMINATION every block of every level -- tiles, then the
  blocks of each merge pass -- must be exactly the oracle's hood of the
  block's points, for single sets and batches, upper and lower hoods.
* With elimination on, a block holds only what survived: every corner of the
  final hood that lies in the block's range must still be there, in order.
* The soundness check (UH_FLAG_CHECK_SIGNS) finds no orientation whose sign
  differs from a 128-bit integer evaluation, and the results do not change.
"""
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


def _dev(xy):
    return torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float32).reshape(-1, 2)).cuda()


def _set_of(off, start):
    return int(np.searchsorted(off, start, side="right") - 1)


def check_levels(pts, off, strip, fan_in, both=False):
    flags = uh.UH_FLAG_NO_ELIMINATION | (uh.UH_FLAG_BOTH_HOODS if both else 0)
    plan = uh.upper_hull_plan_create(off, strip=strip, fan_in=fan_in, flags=flags)
    N = int(off[-1])
    d = _dev(pts)
    levels = plan.passes + 1
    for level in range(levels):
        rng = plan.blocks(level)
        res = plan.trace(d, level)
        assert len(res) == len(rng)
        for b, ((start, length), (cnt, idx)) in enumerate(zip(rng, res)):
            lower = start >= N  # the mirrored half: input points start - N ...
            a = start - N if lower else start
            s = _set_of(off, a)
            sl = pts[a:a + length]
            ref = (oracle.lower_hull(sl) if lower else oracle.upper_hull(sl)) + (a - off[s])
            assert cnt == len(ref), (level, b, start, length, cnt, len(ref))
            assert np.array_equal(idx, ref), (level, b)
    plan.close()
    return levels


@pytest.mark.parametrize("case", [
    ("uniform", 300_001, 16, 16), ("arc", 262_147, 16, 8), ("parabola", 200_003, 8, 4),
    ("uniform_iid", 150_000, 16, 4), ("arc", 70_000, 4, 2), ("uniform", 1024 * 256 * 3 + 5, 16, 256),
])
def test_every_block_of_every_level_is_its_hood(case):
    kind, n, strip, fan = case
    if kind == "uniform":
        xy = synth.uniform(n, 20, seed=n)
    elif kind == "arc":
        xy = synth.arc(n, 20, 4, seed=n)
    elif kind == "parabola":
        xy = synth.parabola(n, 20, 1, seed=n)
    else:
        xy = synth.uniform_iid(n, 27, seed=n)  # equal-x runs cut by tiles
    levels = check_levels(xy, np.array([0, n], np.int64), strip, fan)
    assert levels >= 2


def test_levels_of_a_batch_and_of_both_hoods():
    rng = np.random.default_rng(5)
    sizes = [0, 1, 3, 1024, 1025, 5000, 20_011, 70_001]
    sets = []
    for k, m in enumerate(sizes):
        if m == 0:
            sets.append(np.zeros((0, 2), np.float32))
        elif k % 2:
            sets.append(synth.arc(m, 20, 4, seed=int(rng.integers(1 << 30))))
        else:
            sets.append(synth.uniform(m, 20, seed=int(rng.integers(1 << 30))))
    pts, off = synth.concat_sets(sets)
    check_levels(pts, off, 16, 4)
    check_levels(pts, off, 8, 16, both=True)
    xy = synth.parabola(90_000, 20, 1, seed=3)
    check_levels(xy, np.array([0, len(xy)], np.int64), 16, 8, both=True)


@pytest.mark.parametrize("kind", ["uniform_iid", "arc", "parabola"])
def test_elimination_keeps_every_final_corner_at_every_level(kind):
    n = 400_000
    xy = {"uniform_iid": lambda: synth.uniform_iid(n, 27, seed=9),
          "arc": lambda: synth.arc(n, 20, 4, seed=9),
          "parabola": lambda: synth.parabola(n, 20, 1, seed=9)}[kind]()
    final = oracle.upper_hull(xy)
    plan = uh.upper_hull_plan_create([0, n], fan_in=8)
    d = _dev(xy)
    for level in range(plan.passes + 1):
        for (start, length), (cnt, idx) in zip(plan.blocks(level), plan.trace(d, level)):
            assert cnt >= 0 or (cnt & 0x7fffffff) == len(idx)
            assert np.all(np.diff(idx) > 0)  # left to right
            want = final[(final >= start) & (final < start + length)]
            assert np.all(np.isin(want, idx)), (level, start)
    plan.close()


def test_no_elimination_gives_the_same_hoods():
    for pts, off in (synth.batched_mixed(64), synth.WORKLOADS["uniform_2^27"][0](1 << 21)):
        for flags in (0, uh.UH_FLAG_NO_ELIMINATION):
            plan = uh.upper_hull_plan_create(off, flags=flags)
            out = torch.empty(len(pts), dtype=torch.int32, device="cuda")
            cnt = torch.empty(len(off) - 1, dtype=torch.int32, device="cuda")
            plan.run(_dev(pts), out, cnt)
            torch.cuda.synchronize()
            ref_out, ref_cnt = oracle.upper_hull_batched(pts, off)
            c = cnt.cpu().numpy()
            assert np.array_equal(c, ref_cnt.astype(np.int32))
            o = out.cpu().numpy()
            for s in range(len(off) - 1):
                a = int(off[s])
                assert np.array_equal(o[a:a + c[s]], ref_out[a:a + c[s]]), (flags, s)
            plan.close()


@pytest.mark.parametrize("flags", [0, uh.UH_FLAG_FORCE_FALLBACK, uh.UH_FLAG_NO_ELIMINATION,
                                   uh.UH_FLAG_BOTH_HOODS])
def test_sign_check_finds_no_error(flags):
    sets = [synth.parabola(60_000, 20, 1, seed=1), synth.arc(50_000, 20, 4, seed=2),
            synth.uniform_iid(80_000, 27, seed=3), synth.parabola(3000, 20, 0, seed=4)]
    pts, off = synth.concat_sets(sets)
    S, H = len(sets), 2 if flags & uh.UH_FLAG_BOTH_HOODS else 1
    res = []
    for check in (0, uh.UH_FLAG_CHECK_SIGNS):
        plan = uh.upper_hull_plan_create(off, flags=flags | check)
        out = torch.empty(H * len(pts), dtype=torch.int32, device="cuda")
        cnt = torch.empty(H * S, dtype=torch.int32, device="cuda")
        st = uh.new_stats(H * S)
        plan.run(_dev(pts), out, cnt, st)
        torch.cuda.synchronize()
        d = uh.decode_stats(st.cpu().numpy())
        assert np.all(d["orient_evals"] > 0)
        assert np.all(d["sign_errors"] == 0), d["sign_errors"]
        c = cnt.cpu().numpy()
        o = out.cpu().numpy()
        res.append((c, [o[int(off[s]) + h * len(pts):int(off[s]) + h * len(pts) + c[h * S + s]]
                        for h in range(H) for s in range(S)]))
        plan.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert all(np.array_equal(a, b) for a, b in zip(res[0][1], res[1][1]))
    ref_out, ref_cnt = oracle.upper_hull_batched(pts, off)
    assert np.array_equal(res[0][0][:S], ref_cnt.astype(np.int32))
