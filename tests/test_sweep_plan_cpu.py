"""CPU emulation of the balanced Bellman sweep's work split and LDS indexing, driven by the
library's own plan (dp_sweep_plan, host only; no GPU).

For each block (part p of a row) the emulation follows the kernel: the group geometry, the
staged W segment and reward row, each lane's group and run of chunks (slot-major), the chunk maxima with the first raising chunk, the merge of the
lanes of a group (largest value, then smallest chunk) and the rescan of the winning chunk.
Checked: every (group, chunk) unit is covered by exactly one lane, every LDS read lies in
the staged segment and reward row and reaches every feasible move, the LDS bytes fit the
plan, and the merged result is the brute-force maximum with its smallest maximising next
state, on integer-valued inputs with many exact ties."""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.fixture(scope="module")
def dp():
    import paper_2511_15629_amd as m
    m.lib()
    return m


class St:
    def __init__(self, S, wu, wd):
        self.S, self.w_up, self.w_down = S, wu, wd
        self.delta, self.eta_c, self.eta_d, self.c_deg, self.c_start = 0.01, 0.95, 0.95, 0.0, 0.0


def group(g, R, D, S, wu, wd):
    s0 = R * g
    s_last = min(s0 + R, S) - 1
    dlo = max(-wd, -s_last)
    dhi = min(wu, S - 1 - s0)
    dlo4 = dlo & ~3
    return dlo4, (dhi - dlo4 + D) // D


def layout(R, D, g0, g1, S, wu, wd):
    dlo0, _ = group(g0, R, D, S, wu, wd)
    dloL, _ = group(g1 - 1, R, D, S, wu, wd)
    j_org = R * g0 + dlo0
    r_org = dloL
    nW = (R * (g1 - 1) + R + wu + D - j_org + 4 + 3) & ~3
    nRw = (wu + D - r_org + 3) & ~3
    return j_org, r_org, nW, nRw


def lanes_of_part(R, D, S, wu, wd, g0, g1, Lg, NT):
    """[(local group, first chunk, chunk count)] per lane, in lane order (slot-major)."""
    ngr = g1 - g0
    geo = [group(g, R, D, S, wu, wd) for g in range(g0, g1)]
    assert Lg >= 1 and Lg * ngr <= NT, "more lanes than threads"
    lanes = []
    for t in range(NT):
        gi, slot = t % ngr, t // ngr
        if slot >= Lg:
            lanes.append((gi, 0, 0))
            continue
        n = geo[gi][1]
        c_lo, rem = n // Lg, n % Lg
        lanes.append((gi, slot * c_lo + min(slot, rem), c_lo + (slot < rem)))
    return geo, lanes


def emulate_row(plan, S, wu, wd, W, r_of_d, check_values=True):
    R, D, NT = plan["R"], plan["D"], plan["threads"]
    G = -(-S // R)
    parts = plan["parts"]
    assert parts[0][0] == 0 and parts[-1][1] == G
    assert all(a[1] == b[0] and a[0] < a[1] for a, b in zip(parts, parts[1:] + [(G, G + 1)]))
    V = np.full(S, -np.inf)
    J = np.full(S, -1, dtype=np.int64)
    for (g0, g1, Lg) in parts:
        j_org, r_org, nW, nRw = layout(R, D, g0, g1, S, wu, wd)
        ngr = g1 - g0
        lds = 4 * (nW + nRw) + 8 * ngr * R
        assert lds <= plan["lds"] <= 160 * 1024
        j = j_org + np.arange(nW)
        Wl = np.where((j >= 0) & (j < S), W[np.clip(j, 0, S - 1)], -np.inf)
        d = r_org + np.arange(nRw)
        rl = np.where((d >= -wd) & (d <= wu), r_of_d(np.clip(d, -wd, wu)), -np.inf)
        geo, lanes = lanes_of_part(R, D, S, wu, wd, g0, g1, Lg, NT)
        covered = [np.zeros(n, dtype=np.int64) for (_, n) in geo]
        best = {}
        for (gi, c0, cnt) in lanes:
            if cnt == 0:
                continue
            dlo4, n = geo[gi]
            covered[gi][c0:c0 + cnt] += 1
            wb = R * (g0 + gi) + dlo4 - j_org
            rb = dlo4 - r_org
            assert wb >= 0 and rb >= 0
            assert wb + (c0 + cnt - 1) * D + R + D - 1 < nW, "W segment read past its end"
            assert rb + (c0 + cnt - 1) * D + D - 1 < nRw, "reward row read past its end"
            if not check_values:
                continue
            c = np.arange(c0, c0 + cnt)
            wi = wb + c[:, None, None] * D + np.arange(R)[None, :, None] + np.arange(D)[None, None, :]
            ri = rb + c[:, None] * D + np.arange(D)[None, :]
            cand = Wl[wi] + rl[ri][:, None, :]                 # [chunk, output, move]
            m = cand.max(axis=2)                                # chunk maxima
            bv = m.max(axis=0)
            first = np.argmax(m == bv[None, :], axis=0)         # first chunk reaching it
            for i in range(R):
                if bv[i] == -np.inf:
                    continue
                key = (bv[i], -(c0 + first[i]))
                o = (gi, i)
                if o not in best or key > best[o]:
                    best[o] = key
        for gi, cov in enumerate(covered):
            assert np.all(cov == 1), f"group {g0 + gi}: chunks covered {cov.tolist()}"
            dlo4, n = geo[gi]
            s_first = R * (g0 + gi)
            # the chunks reach every feasible move of the group's outputs
            for s in range(s_first, min(s_first + R, S)):
                assert dlo4 <= max(-wd, -s) and dlo4 + D * n - 1 >= min(wu, S - 1 - s)
        if not check_values:
            continue
        for (gi, i), (v, negc) in best.items():
            s = R * (g0 + gi) + i
            if s >= S:
                continue
            dlo4, _ = geo[gi]
            bc = -negc
            base = s + dlo4 + bc * D
            xs = Wl[base + np.arange(D) - j_org] + rl[dlo4 + bc * D + np.arange(D) - r_org]
            arg = int(np.argmax(xs == v))
            assert xs[arg] == v
            V[s], J[s] = v, base + arg
    if check_values:
        for s in range(S):
            jj = np.arange(max(0, s - wd), min(S - 1, s + wu) + 1)
            q_ = W[jj] + r_of_d(jj - s)
            assert V[s] == q_.max(), f"s={s}: {V[s]} vs {q_.max()}"
            assert J[s] == jj[np.argmax(q_ == q_.max())], f"s={s}: j {J[s]}"


CASES = [
    (50, 2001, 500, 500), (100, 1001, 250, 250), (10, 101, 25, 25), (3, 7, 2, 3),
    (17, 600, 40, 70), (33, 1300, 300, 5), (1, 2, 1, 1), (5, 40, 0, 0), (4, 257, 256, 256),
    (64, 512, 64, 64), (20, 2001, 160, 190), (2, 129, 1, 100), (6, 300, 20, 35),
    (1024, 64, 8, 8), (1, 5000, 3, 2000), (7, 333, 333, 1),
]


@pytest.mark.parametrize("K,S,wu,wd", CASES)
def test_balanced_plan_covers_every_unit_and_finds_the_smallest_argmax(dp, K, S, wu, wd):
    # the balanced kernel forced with R = 8, D = 16 and 8 waves; the library's cost model
    # picks the split of the row into parts and the lanes per group
    dp.set_sweep_shape(8, 16, 8, 0)
    try:
        plan = dp.sweep_plan(3, K, St(S, wu, wd))
    finally:
        dp.set_sweep_shape()
    assert plan["kernel"] == "balanced"
    rng = np.random.default_rng(S * 7 + wu)
    W = rng.integers(-6, 7, size=S).astype(np.float64)
    rtab = rng.integers(-3, 4, size=wu + wd + 1).astype(np.float64)
    rtab[wd] = 0.0
    emulate_row(plan, S, wu, wd, W, lambda d: rtab[np.asarray(d) + wd])


@pytest.mark.parametrize("shape", [(8, 16, 8), (8, 16, 4), (4, 16, 8), (4, 16, 4), (8, 8, 8), (4, 8, 4)])
@pytest.mark.parametrize("K,S,wu,wd", [(50, 2001, 500, 500), (17, 600, 40, 70), (3, 7, 2, 3), (2, 129, 1, 100)])
def test_every_forced_balanced_shape(dp, shape, K, S, wu, wd):
    R, D, NW = shape
    dp.set_sweep_shape(R, D, NW, 0)
    try:
        plan = dp.sweep_plan(3, K, St(S, wu, wd))
    finally:
        dp.set_sweep_shape()
    assert plan["kernel"] == "balanced" and (plan["R"], plan["D"], plan["threads"]) == (R, D, 64 * NW)
    rng = np.random.default_rng(S + R + D)
    W = rng.integers(-4, 5, size=S).astype(np.float64)
    rtab = rng.integers(-2, 3, size=wu + wd + 1).astype(np.float64)
    rtab[wd] = 0.0
    emulate_row(plan, S, wu, wd, W, lambda d: rtab[np.asarray(d) + wd])


@pytest.mark.parametrize("K,S,wu,wd", [(2, 32767, 7000, 7000), (2, 32767, 9000, 9000), (1, 32767, 1, 1)])
def test_largest_grids_stay_in_bounds(dp, K, S, wu, wd):
    dp.set_sweep_shape(4, 16, 4, 0)
    try:
        plan = dp.sweep_plan(3, K, St(S, wu, wd))
    finally:
        dp.set_sweep_shape()
    assert plan["kernel"] == "balanced"
    emulate_row(plan, S, wu, wd, np.zeros(S), lambda d: np.zeros(np.shape(d)), check_values=False)


def test_forced_row_tile_shape_is_reported(dp):
    dp.set_sweep_shape(8, 16, 8, 8)
    try:
        plan = dp.sweep_plan(3, 50, St(2001, 500, 500))
    finally:
        dp.set_sweep_shape()
    assert plan["kernel"] == "row_tile" and (plan["R"], plan["NW"], plan["NSPLIT"]) == (8, 8, 8)
