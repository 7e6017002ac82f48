"""Host-only plan of the matrix-core Kerr contraction (mmnlse_kerr_plan, CPU).

The contraction multiplies only the (32-slot row tile, k-step) blocks listed
for each pass.  These tests check the plan against the packed tensor computed
here from its definition, Sp[(p,n)][(l,m)] = w S[p,l,m,n] (w = 2 for l < m):
every row appears in exactly one slot, every nonzero entry must fall in a
listed block of the pass that holds its row, passes must cover every row
tile once, and the reported counts must match.  A planted mistake (one
nonzero block dropped from the lists) must be caught by the same check.
"""

import os

import numpy as np
import pytest

import workloads as W

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1901_01895_amd", "libmmnlse.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def packed(S):
    M = S.shape[0]
    pairs = [(i, j) for i in range(M) for j in range(i, M)]
    a = np.array([x[0] for x in pairs])
    b = np.array([x[1] for x in pairs])
    w = np.where(a < b, 2.0, 1.0)
    return w[None, :] * S.astype(np.float64)[a[:, None], a[None, :], b[None, :], b[:, None]]


def uncovered(plan, Sp):
    """Nonzero entries of the packed matrix (rows in their slots, columns in
    the plan's order) outside every listed block."""
    perm, kw, rows = plan["perm"], plan["kw"], plan["rows"]
    slots = np.nonzero(rows >= 0)[0]
    pos = np.nonzero(perm >= 0)[0]
    X = Sp[np.ix_(rows[slots], perm[pos])]
    listed = np.zeros((plan["nrt"], plan["Ppad"] // kw), bool)
    for rt0, nt, off, n in plan["passes"]:
        for k in plan["klist"][off:off + n]:
            listed[rt0:rt0 + nt, k] = True
    r, c = np.nonzero(X)
    return int(np.count_nonzero(~listed[slots[r] // 32, pos[c] // kw]))


def check(plan, Sp):
    P, kw = plan["P"], plan["kw"]
    perm = plan["perm"]
    assert len(perm) == plan["Ppad"] and plan["Ppad"] % 32 == 0
    assert sorted(perm[perm >= 0].tolist()) == list(range(P))
    assert np.all(perm[perm < 0] == -1)
    rows = plan["rows"]
    assert len(rows) == 32 * plan["nrt"]
    assert sorted(rows[rows >= 0].tolist()) == list(range(P))
    assert np.all(rows[rows < 0] == -1)
    assert np.all((rows.reshape(-1, 32) >= 0).any(axis=1))       # no empty tile
    tiles = np.zeros(plan["nrt"], int)
    for rt0, nt, off, n in plan["passes"]:
        tiles[rt0:rt0 + nt] += 1
        ks = plan["klist"][off:off + n]
        assert np.all(np.diff(ks) > 0) and (n == 0 or (ks[0] >= 0 and ks[-1] < plan["Ppad"] // kw))
        assert nt in (1, 2, 4) and nt <= plan["rtm"]
    assert np.all(tiles == 1)
    assert uncovered(plan, Sp) == 0
    e = plan["entries"]
    assert e["dense"] == P * P
    assert e["nonzero"] == np.count_nonzero(Sp)
    assert e["multiplied"] == sum(nt * 32 * kw * n for _, nt, _, n in plan["passes"])
    assert e["nonzero"] <= e["multiplied"] <= 32 * plan["nrt"] * plan["Ppad"]


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_tensor_keeps_natural_order_and_full_lists(precision):
    import paper_1901_01895_amd as mm
    S = W.symmetric_gaussian_tensor(6, np.random.default_rng(41)).astype(np.float32)
    plan = mm.kerr_plan(S, precision)
    Sp = packed(S)
    check(plan, Sp)
    assert np.array_equal(plan["perm"][:plan["P"]], np.arange(plan["P"]))
    assert np.all(plan["perm"][plan["P"]:] == -1) and plan["Ppad"] == -(-plan["P"] // 32) * 32
    # a dense tensor keeps the fixed tiles: tile t holds rows 32t .. 32t + 31 (in
    # the slot order that lets both lane halves scatter at once), padding only in
    # the last tile
    assert plan["nrt"] == -(-plan["P"] // 32)
    rows = np.asarray(plan["rows"]).reshape(-1, 32)
    for t in range(plan["nrt"]):
        real = sorted(r for r in rows[t] if r >= 0)
        assert real == list(range(32 * t, min(32 * t + 32, plan["P"])))
    # every k-step holding a real column is listed; all-padding k-steps are not
    nk_real = -(-plan["P"] // plan["kw"])
    assert all(n == nk_real for _, _, _, n in plan["passes"])


@pytest.mark.parametrize("precision", [0, 1])
def test_mode_group_masked_tensor_skips_only_zero_blocks(precision):
    import paper_1901_01895_amd as mm
    p = W.make_problem("wdm36", T=2 ** 10, n_steps=1)
    plan = mm.kerr_plan(p.S, precision)
    Sp = packed(p.S)
    check(plan, Sp)
    e = plan["entries"]
    # the 70 % masked tensor leaves well under the dense block count multiplied;
    # cutting the row tiles and k-steps at the zero-pattern groups takes FP32 from
    # 0.56 to 0.48 (the split path keeps fixed tiles and k-steps)
    assert e["nonzero"] / e["dense"] < 0.35
    assert e["multiplied"] / e["dense"] < (0.50 if precision == 0 else 0.80)
    if precision == 1:
        assert plan["nrt"] == -(-plan["P"] // 32)


def test_planted_dropped_block_is_caught():
    import paper_1901_01895_amd as mm
    p = W.make_problem("wdm36", T=2 ** 10, n_steps=1)
    plan = mm.kerr_plan(p.S, 0)
    Sp = packed(p.S)
    # mistake: remove the first listed k-step of the first non-empty pass
    i = next(j for j, ps in enumerate(plan["passes"]) if ps[3] > 0)
    rt0, nt, off, n = plan["passes"][i]
    klist = np.delete(plan["klist"], off)
    passes = plan["passes"].copy()
    passes[i, 3] -= 1
    passes[i + 1:, 2] -= 1
    assert uncovered(dict(plan, passes=passes, klist=klist), Sp) > 0


def test_sparse_random_pattern_covered():
    """A symmetric tensor with random whole-class zeros (not by mode group)."""
    import paper_1901_01895_amd as mm
    rng = np.random.default_rng(43)
    M = 12
    S = W.symmetric_gaussian_tensor(M, rng)
    keep = rng.random((M,) * 4) < 0.4
    keep = keep | keep.transpose(0, 2, 1, 3)
    keep = keep & keep.transpose(3, 1, 2, 0)   # zero set symmetric in (l,m) and (p,n)
    S = np.where(keep, S, 0.0).astype(np.float32)
    for precision in (0, 1):
        plan = mm.kerr_plan(S, precision)
        check(plan, packed(S))


def test_plan_rejects_bad_arguments():
    import paper_1901_01895_amd as mm
    with pytest.raises(mm.MMNLSEError):
        mm.kerr_plan(np.ones((1, 1, 1, 1), np.float32), precision=5)


@pytest.mark.parametrize("precision", [0, 1])
def test_masked_tensor_tiles_let_both_lane_halves_scatter(precision):
    """In the 32 x 32 accumulator lane half h holds rows 8g + 4h + j, so the
    scatter of both halves at once updates the modes of slots 8g + j and
    8g + 4 + j in the same instructions.  On the mode-group masked 36-mode
    tensor the plan places every tile's rows so that those two rows differ in
    p and in n (or one is padding), which the simultaneous scatter needs."""
    import paper_1901_01895_amd as mm
    p = W.make_problem("wdm36", T=2 ** 10, n_steps=1)
    plan = mm.kerr_plan(p.S, precision)
    na, nb = [], []
    for i in range(p.M):
        for j in range(i, p.M):
            na.append(i)
            nb.append(j)
    rows = np.asarray(plan["rows"]).reshape(-1, 32)
    for t in range(rows.shape[0]):
        for g in range(4):
            for j in range(4):
                x, y = rows[t, 8 * g + j], rows[t, 8 * g + 4 + j]
                if x >= 0 and y >= 0:
                    assert na[x] != na[y] and nb[x] != nb[y], (t, g, j)
