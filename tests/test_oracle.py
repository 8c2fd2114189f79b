"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: published
known-answer values, closed forms, invariants of the method, exact rational
arithmetic, or brute force on tiny inputs.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# T1: Philox4x32-10 against its published known-answer vectors
# ---------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_philox_known_answers(ctr, key, expect):
    assert [int(x) for x in O.philox(ctr, key)] == expect


def test_philox_bit_balance():
    # every output bit of a good generator is set half the time
    words = np.array([O.philox([k, 0, 3, 0], [24301, 0]) for k in range(4096)], dtype=np.uint64)
    bits = np.unpackbits(words.astype(">u4").view(np.uint8)).reshape(-1, 128).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 5 * 0.5 / math.sqrt(4096))


# ---------------------------------------------------------------------------
# T3: Zipf table and sampler
# ---------------------------------------------------------------------------
def test_zipf_table_matches_generalized_harmonic_numbers():
    theta, W = 0.99, 1000
    C = O.zipf_table(theta, W).astype(np.float64)
    # exactly-rounded partial sums (math.fsum) as the closed form F[k]/F[W]
    terms = [k ** -theta for k in range(1, W + 1)]
    FW = math.fsum(terms)
    F = np.array([math.fsum(terms[:k]) for k in range(1, W + 1)])
    assert C[0] == 0 and C[W] == 2 ** 32 - 1
    assert np.all(np.diff(C) > 0), "table must be strictly increasing"
    assert np.max(np.abs(C[1:] / C[W] - F / FW)) < 2 ** -31


def test_zipf_table_theta1_exact_rational():
    # theta = 1: F[k] is the harmonic number H_k; compare with exact Fractions
    W = 60
    C = O.zipf_table(1.0, W)
    H = [Fraction(0)]
    for k in range(1, W + 1):
        H.append(H[-1] + Fraction(1, k))
    for k in range(1, W + 1):
        exact = math.floor(H[k] / H[W] * (2 ** 32 - 1))
        assert abs(int(C[k]) - exact) <= 1


def test_zipf_table_theta0_is_uniform():
    W = 37
    C = O.zipf_table(0.0, W)
    for k in range(W + 1):
        assert abs(int(C[k]) - (k * (2 ** 32 - 1)) // W) <= 1


def test_zipf_draw_equals_linear_scan_and_stays_in_range():
    C = O.zipf_table(0.99, 1000)
    rng = np.random.default_rng(3)
    for n in [1, 2, 3, 7, 64, 999, 1000]:
        for r in rng.integers(0, 2 ** 32, size=300, dtype=np.uint64):
            z = O.zipf_draw(C, n, int(r))
            u = (int(r) * int(C[n])) >> 32
            brute = next(k for k in range(1, n + 1) if C[k] > u)
            assert z == brute and 1 <= z <= n
    assert O.zipf_draw(C, 5, 0) == 1
    assert O.zipf_draw(C, 5, 2 ** 32 - 1) == 5


@pytest.mark.parametrize("n", [1, 2, 7, 1000])
def test_zipf_draw_histogram_chi_square(n):
    C = O.zipf_table(0.99, 1000)
    # a fine uniform grid over the 32-bit input (deterministic, ~uniform)
    N = 1 << 18
    rs = (np.arange(N, dtype=np.uint64) * (2 ** 32 // N) + 12345) % (2 ** 32)
    counts = np.zeros(n + 1)
    for r in rs:
        counts[O.zipf_draw(C, n, int(r))] += 1
    pmf = np.diff(C[: n + 1].astype(np.float64)) / float(C[n])
    expected = pmf * N
    if n == 1:
        assert counts[1] == N
        return
    chi2 = float(np.sum((counts[1:] - expected) ** 2 / expected))
    # a grid is far more even than random sampling; bound by the chi-square 99.9% point
    dof = n - 1
    assert chi2 < dof + 4.5 * math.sqrt(2 * dof) + 10
    # the table pmf is the truncated Zipf law z^-theta / H_{n,theta}
    true = np.array([k ** -0.99 for k in range(1, n + 1)])
    true /= true.sum()
    assert np.max(np.abs(pmf - true)) < 1e-6


# ---------------------------------------------------------------------------
# T4: positions are node-length prefix sums; endpoint coordinates
# ---------------------------------------------------------------------------
def test_positions_are_prefix_sums(tiny_synth, tiny_oracle):
    g, sg = tiny_oracle, tiny_synth
    pos = g.pos
    for p in range(g.n_paths):
        acc = 0
        for s in range(int(sg.path_off[p]), int(sg.path_off[p + 1])):
            assert pos[s] == acc
            acc += int(sg.node_len[int(sg.step_node[s]) & 0x7FFFFFFF])
        assert g.path_nt[p] == acc
    assert g.d_max == max(g.path_nt)


def test_endpoint_positions_forward_and_reverse():
    # node 0 (len 3) forward, node 1 (len 2) reverse, node 2 (len 4) forward
    g = O.Graph(np.array([3, 2, 4], np.uint32), np.array([0, 3], np.uint64),
                np.array([0, 1 | synth.REV_BIT, 2], np.uint32))
    assert [g.endpoint_pos(0, 0), g.endpoint_pos(0, 1)] == [0, 3]
    assert [g.endpoint_pos(1, 0), g.endpoint_pos(1, 1)] == [5, 3]   # reverse: start is met last
    assert [g.endpoint_pos(2, 0), g.endpoint_pos(2, 1)] == [5, 9]
    for s, L in [(0, 3), (1, 2), (2, 4)]:
        assert abs(g.endpoint_pos(s, 0) - g.endpoint_pos(s, 1)) == L


# ---------------------------------------------------------------------------
# T5: schedule
# ---------------------------------------------------------------------------
def test_schedule_closed_form():
    dmax = 8973
    eta = O.schedule(30, float(dmax) ** 2, 0.01)
    assert eta[0] == float(dmax) ** 2
    assert abs(eta[-1] - 0.01) <= 1e-15
    ratio = eta[1:] / eta[:-1]
    assert np.allclose(ratio, ratio[0], rtol=1e-12, atol=0)
    assert abs(ratio[0] - (0.01 / dmax ** 2) ** (1 / 29)) < 1e-12
    assert list(O.schedule(1, 5.0, 0.01)) == [5.0]


# ---------------------------------------------------------------------------
# T2: sampling invariants and uniformity
# ---------------------------------------------------------------------------
def _path_of(path_off, s):
    return np.searchsorted(path_off, s, side="right") - 1


def test_sampling_invariants(tiny_synth, tiny_oracle):
    g, sg = tiny_oracle, tiny_synth
    for it in [0, 14, 15, 29]:
        i, j, f = O.sample_terms(g, it, 0, 20000)
        assert np.all(i < g.S) and np.all(j < g.S)
        pi, pj = _path_of(sg.path_off, i), _path_of(sg.path_off, j)
        assert np.all(pi == pj), "partner must lie on the same path"
        cool = (f >> 2) & 1
        if it >= 15:
            assert np.all(cool == 1)
        else:
            assert 0.3 < cool.mean() < 0.7
            # the coin is shared by each aligned group of 64 terms
            assert np.all(cool.reshape(-1, 64)[:, :-1] == cool.reshape(-1, 64)[:, 1:]) if len(cool) % 64 == 0 \
                else True
        hop = np.abs(i.astype(np.int64) - j.astype(np.int64))
        c = cool == 1
        skip = ((f >> 3) & 1) == 1
        assert np.all(hop[c & ~skip] >= 1) and np.all(hop[c] <= 1000)
        # endpoint coins are fair
        assert abs((f & 1).mean() - 0.5) < 0.02 and abs(((f >> 1) & 1).mean() - 0.5) < 0.02


def test_sampling_group_coin_is_group_leader_bit(tiny_oracle):
    g = tiny_oracle
    i, j, f = O.sample_terms(g, 3, 64 * 10 + 5, 64 * 3)
    for k in range(len(f)):
        t = 64 * 10 + 5 + k
        lead = O.philox([(t - t % 64) & 0xFFFFFFFF, t >> 32, 3, 0], [24301, 0])
        assert ((f[k] >> 2) & 1) == ((lead[3] >> 3) & 1)


def test_step_selection_uniform_chi_square(tiny_oracle):
    g = tiny_oracle
    N = 400_000
    i, _, _ = O.sample_terms(g, 0, 0, N)
    counts = np.bincount(i.astype(np.int64), minlength=g.S)
    e = N / g.S
    chi2 = float(np.sum((counts - e) ** 2 / e))
    dof = g.S - 1
    assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof)


def test_sampling_counter_carry_into_high_word(tiny_oracle):
    # terms around t = 2^32 use counter words (t mod 2^32, t >> 32)
    g = tiny_oracle
    t0 = 2 ** 32 - 3
    i, j, f = O.sample_terms(g, 7, t0, 6)
    for k in range(6):
        t = t0 + k
        r = O.philox([t & 0xFFFFFFFF, t >> 32, 7, 0], [24301, 0])
        u64 = int(r[0]) | (int(r[1]) << 32)
        assert int(i[k]) == (u64 * g.S) >> 64


def test_uniform_partner_is_uniform_within_path():
    # one path of 5 steps: the uniform partner of any i covers all 5 steps evenly
    g = O.Graph(np.full(5, 2, np.uint32), np.array([0, 5], np.uint64), np.arange(5, dtype=np.uint32))
    i, j, f = O.sample_terms(g, 0, 0, 64 * 2000)
    cool = ((f >> 2) & 1) == 1
    cnt = np.bincount(j[~cool].astype(np.int64), minlength=5)
    assert cnt.min() > 0.9 * cnt.mean() and cnt.max() < 1.1 * cnt.mean()


def test_power_law_partner_boundaries():
    # a single-step path is always skipped in cooling; at the path ends the hop turns inwards
    g = O.Graph(np.array([4, 3, 3, 3], np.uint32), np.array([0, 1, 4], np.uint64), np.arange(4, dtype=np.uint32))
    i, j, f = O.sample_terms(g, 20, 0, 20000)
    cool_skip = ((f >> 3) & 1) == 1
    assert np.all(cool_skip[i == 0]), "len-1 path must be skipped"
    assert np.all(j[i == 1] > 1) and np.all(j[i == 3] < 3)
    assert np.all((j[(i >= 1)] >= 1) & (j[(i >= 1)] <= 3))


# ---------------------------------------------------------------------------
# T5b: the window-major enumeration (reading R18) against the plain definition
# and the uniform law it must reproduce
# ---------------------------------------------------------------------------
def _windows(S):
    sh = O.window_shift(S)
    return sh, (S + (1 << sh) - 1) >> sh


@pytest.mark.parametrize("S", [0, 1, 63, 64, 1000, 14416, 64 << 14, (64 << 14) - 1, 10 ** 8, 408037251, 10 ** 12])
def test_window_shift_bounds(S):
    sh, n = _windows(S)
    assert 6 <= sh
    assert n <= 32768
    assert n >= 16 or sh == 6           # at least 16 windows unless they are at their 64-step minimum
    assert sh <= 14 or _windows(S)[1] > 16384  # longer than 2^14 only when 2^14 would exceed the window cap


def test_window_counts_are_the_histogram_of_plain_draws(tiny_oracle):
    g = tiny_oracle
    sh = O.window_shift(g.S)
    T = 10 * g.S
    for it in (0, 17):
        i, _, _ = O.sample_terms(g, it, 0, T)
        brute = np.bincount((i >> np.uint64(sh)).astype(np.int64), minlength=_windows(g.S)[1])
        assert np.array_equal(O.window_counts(g, it).astype(np.int64), brute)
        assert np.array_equal(O.window_counts(g, it, threads=3), O.window_counts(g, it))


def test_windowed_slots_follow_their_window(tiny_synth, tiny_oracle):
    g, sg = tiny_oracle, tiny_synth
    sh = O.window_shift(g.S)
    T = 10 * g.S
    for it in (0, 15):
        counts = O.window_counts(g, it).astype(np.int64)
        i, j, f = O.sample_terms_windowed(g, it, 0, T)
        w_of_slot = np.repeat(np.arange(len(counts)), counts)
        assert np.array_equal(i.astype(np.int64) >> sh, w_of_slot), "slot step outside its window"
        assert np.all(j < g.S)
        assert np.all(_path_of(sg.path_off, i) == _path_of(sg.path_off, j)), "partner must lie on the same path"
        cool = (f >> 2) & 1
        hop = np.abs(i.astype(np.int64) - j.astype(np.int64))
        assert np.all(hop[cool == 1] <= 1000)
        if it >= 15:
            assert np.all(cool == 1)
        else:
            assert 0.3 < cool.mean() < 0.7
            off = np.concatenate([[0], np.cumsum(counts)])
            for w in range(len(counts)):  # one coin per aligned 64-slot group of a window
                cw = cool[off[w]:off[w + 1]]
                for b in range(0, len(cw), 64):
                    assert np.all(cw[b:b + 64] == cw[b])
        assert abs((f & 1).mean() - 0.5) < 0.02 and abs(((f >> 1) & 1).mean() - 0.5) < 0.02


def test_windowed_steps_are_uniform_chi_square(tiny_oracle):
    # pooled over three iterations: 3 * 10 * S slots over S steps
    g = tiny_oracle
    T = 10 * g.S
    i = np.concatenate([O.sample_terms_windowed(g, it, 0, T)[0] for it in (0, 1, 2)])
    counts = np.bincount(i.astype(np.int64), minlength=g.S)
    e = len(i) / g.S
    chi2 = float(np.sum((counts - e) ** 2 / e))
    dof = g.S - 1
    assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof)
    # and uniform inside the windows (offsets in the full-length windows)
    sh = O.window_shift(g.S)
    full = i < ((g.S >> sh) << sh)
    pos = (i[full] & np.uint64((1 << sh) - 1)).astype(np.int64)
    c2 = np.bincount(pos, minlength=1 << sh)
    e2 = len(pos) / (1 << sh)
    chi2b = float(np.sum((c2 - e2) ** 2 / e2))
    assert abs(chi2b - ((1 << sh) - 1)) < 5 * math.sqrt(2 * ((1 << sh) - 1))


def test_windowed_slot_draw_and_counter(tiny_oracle):
    # slot s draws Philox stream 5 at counter (s mod 2^32, s >> 32, iteration, 5 << 24 | graph_id)
    g = tiny_oracle
    sh = O.window_shift(g.S)
    counts = O.window_counts(g, 4, graph_id=3).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(counts)])
    s0 = int(off[7]) + 60
    i, j, f = O.sample_terms_windowed(g, 4, s0, 10, graph_id=3)
    for k in range(10):
        s = s0 + k
        w = int(np.searchsorted(off, s, side="right") - 1)
        r = O.philox([s & 0xFFFFFFFF, s >> 32, 4, (5 << 24) | 3], [24301, 0])
        start = w << sh
        ln = min(1 << sh, g.S - start)
        assert int(i[k]) == start + ((int(r[0]) | (int(r[1]) << 32)) * ln >> 64)
        lead_slot = int(off[w]) + ((s - int(off[w])) // 64) * 64
        lead = O.philox([lead_slot & 0xFFFFFFFF, lead_slot >> 32, 4, (5 << 24) | 3], [24301, 0])
        assert ((int(f[k]) >> 2) & 1) == ((int(lead[3]) >> 3) & 1)


def test_windowed_layout_quality_equals_plain_on_tiny(tiny_oracle):
    # same term distribution, another sequential order: the exact expectation of the
    # sampled path stress after full layouts agrees within 3% (mean of 3 seeds each)
    g = tiny_oracle
    c0 = O.init_coords(g)
    plain, win = [], []
    for seed in (0, 1, 2):
        a = c0.copy()
        O.layout(g, a, seed=seed)
        plain.append(O.sps_expectation(g, a)[0])
        b = c0.copy()
        O.layout_windowed(g, b, seed=seed)
        win.append(O.sps_expectation(g, b)[0])
    assert abs(np.mean(win) / np.mean(plain) - 1) < 0.03


def test_windowed_layout_converges_on_a_linear_path():
    n = 400
    g = O.Graph(np.full(n, 5, np.uint32), np.array([0, n], np.uint64), np.arange(n, dtype=np.uint32))
    c = O.init_coords(g)
    O.layout_windowed(g, c)
    assert O.sps_expectation(g, c)[0] < 1e-3


# ---------------------------------------------------------------------------
# T5c: layout loops (plain, windowed, data reuse on both) against a fixed point
# ---------------------------------------------------------------------------
def _disjoint_paths_fixed_point():
    """Three paths over disjoint nodes (some visited on the reverse strand), each laid out on
    its own horizontal line at its path coordinates: every same-path pair has |v_a - v_b| = d,
    so every update of a correct loop is zero and the layout must not move at all."""
    rng = np.random.default_rng(5)
    sizes = [700, 1, 450]
    node_len, step_node, off = [], [], [0]
    nid = 0
    for n in sizes:
        for _ in range(n):
            node_len.append(int(rng.integers(1, 9)))
            step_node.append(nid | (synth.REV_BIT if rng.random() < 0.2 else 0))
            nid += 1
        off.append(off[-1] + n)
    g = O.Graph(np.array(node_len, np.uint32), np.array(off, np.uint64), np.array(step_node, np.uint32))
    c = np.zeros(4 * nid, np.float32)
    X, Y = c[:2 * nid], c[2 * nid:]
    for p_, (b, e) in enumerate(zip(off[:-1], off[1:])):
        for s_ in range(b, e):
            node = step_node[s_] & 0x7FFFFFFF
            for end in (0, 1):
                X[2 * node + end] = g.endpoint_pos(s_, end)
                Y[2 * node + end] = 1000.0 * p_
    return g, c


@pytest.mark.parametrize("loop", ["plain", "windowed", "reuse_plain", "reuse_windowed"])
def test_layout_loops_keep_a_fixed_point(loop):
    # pins d_ref (step positions, endpoint orientation), the same-path condition of reuse pairs
    # and the update arithmetic of every loop: any wrong distance moves some point
    g, c = _disjoint_paths_fixed_point()
    before = c.copy()
    if loop == "plain":
        n = O.layout(g, c, n_iters=6)
    elif loop == "windowed":
        n = O.layout_windowed(g, c, n_iters=6)
    elif loop == "reuse_plain":
        n = O.layout_reuse(g, c, 4, 2, n_iters=6)
    else:
        n = O.layout_windowed(g, c, n_iters=6, reuse_factor=4, step_reduction=2)
    assert n > 0
    assert np.array_equal(c, before)


def test_windowed_slot_count_with_step_reduction(tiny_oracle):
    g = tiny_oracle
    sh = O.window_shift(g.S)
    for srf in (2, 3, 7):
        T = O.window_slots(g, 10, srf)
        assert T == -(-10 * g.S // srf)
        i, _, _ = O.sample_terms(g, 5, 0, T)
        brute = np.bincount((i >> np.uint64(sh)).astype(np.int64), minlength=(g.S + (1 << sh) - 1) >> sh)
        assert np.array_equal(O.window_counts(g, 5, step_reduction=srf).astype(np.int64), brute)


def test_reuse_offsets_follow_the_stated_draw():
    # o_k = 1 + (byte k-1 of the words of Philox stream 4 at counter (group, 0, iter)) mod 63
    for group, it, drf in ((0, 0, 16), (12345, 7, 5), ((1 << 33) + 9, 29, 9)):
        o = O.reuse_offsets(it, group, drf, seed=24301, graph_id=2)
        r = O.philox([group & 0xFFFFFFFF, group >> 32, it, (4 << 24) | 2], [24301, 0])
        expect = [1 + ((int(r[(k - 1) // 4]) >> (8 * ((k - 1) % 4))) & 0xFF) % 63 for k in range(1, drf)]
        assert o == expect and all(1 <= x <= 63 for x in o)


def test_reuse_rounds_add_updates(tiny_oracle):
    g = tiny_oracle
    c0 = O.init_coords(g)
    a, b = c0.copy(), c0.copy()
    n1 = O.layout_windowed(g, a, n_iters=2, step_reduction=2)
    n4 = O.layout_windowed(g, b, n_iters=2, reuse_factor=4, step_reduction=2)
    assert 2.5 * n1 < n4 <= 4 * n1 + 10


# ---------------------------------------------------------------------------
# T6: one update against the closed form (two-node example) and the gradient
# ---------------------------------------------------------------------------
def _two_node():
    # node A (len 3) then node B (len 2), one forward path: A.start at 0, B.end at 5 -> d = 5
    return O.Graph(np.array([3, 2], np.uint32), np.array([0, 2], np.uint64), np.array([0, 1], np.uint32))


def _coords_two_node(xa, xb):
    c = np.zeros(8, np.float64)   # X plane [A.s, A.e, B.s, B.e], then Y plane
    c[0], c[3] = xa, xb
    return c


@pytest.mark.parametrize("eta,expect", [(25.0, (2.5, 7.5)), (1000.0, (2.5, 7.5)), (5.0, (0.5, 9.5))])
def test_two_node_update_closed_form(eta, expect):
    g = _two_node()
    c = _coords_two_node(0.0, 10.0)
    i, j, fl = np.array([0], np.uint64), np.array([1], np.uint64), np.array([0 | (1 << 1)], np.uint8)
    assert O.apply_terms_f64(g, eta, i, j, fl, c) == 1
    assert c[0] == expect[0] and c[3] == expect[1]
    assert c[4] == 0 and c[7] == 0
    c32 = _coords_two_node(0.0, 10.0).astype(np.float32)
    O.apply_terms_f32(g, eta, i, j, fl, c32)
    assert c32[0] == expect[0] and c32[3] == expect[1]


def test_update_is_quarter_eta_gradient_step_and_keeps_midpoint():
    g = _two_node()
    rng = np.random.default_rng(5)
    i, j, fl = np.array([0], np.uint64), np.array([1], np.uint64), np.array([0 | (1 << 1)], np.uint8)
    d = 5.0
    for _ in range(20):
        c = np.zeros(8)
        c[[0, 3, 4, 7]] = rng.normal(scale=20, size=4)
        va, vb = np.array([c[0], c[4]]), np.array([c[3], c[7]])
        mag = np.linalg.norm(va - vb)
        eta = float(rng.uniform(0.1, 20))          # mu = eta/d^2 < 1
        mu = min(eta / d ** 2, 1.0)

        def stress(a):
            return ((np.linalg.norm(a - vb) - d) / d) ** 2

        h = 1e-6
        grad = np.array([(stress(va + h * e) - stress(va - h * e)) / (2 * h) for e in np.eye(2)])
        O.apply_terms_f64(g, eta, i, j, fl, c)
        na, nb = np.array([c[0], c[4]]), np.array([c[3], c[7]])
        assert np.allclose(na, va - eta / 4 * grad, rtol=1e-6, atol=1e-6)
        assert np.allclose((na + nb) / 2, (va + vb) / 2, atol=1e-9)
        assert abs(np.linalg.norm(na - nb) - abs(mag - mu * (mag - d))) < 1e-9


def test_update_skips_degenerate_terms():
    # same slot (a == b) and zero distance are skipped at sampling; mag == 0 at update
    g = _two_node()
    c = np.zeros(8)
    assert O.apply_terms_f64(g, 10.0, np.array([0], np.uint64), np.array([1], np.uint64),
                             np.array([2], np.uint8), c) == 0   # coincident points: mag == 0
    i, j, f = O.sample_terms(g, 0, 0, 4096)
    a = i * 2 + (f & 1)
    b = j * 2 + ((f >> 1) & 1)
    pa = np.where((f & 1) == 1, np.array([3, 5])[i.astype(int)], np.array([0, 3])[i.astype(int)])
    pb = np.where(((f >> 1) & 1) == 1, np.array([3, 5])[j.astype(int)], np.array([0, 3])[j.astype(int)])
    should_skip = (a == b) | (pa == pb)
    assert np.array_equal(((f >> 3) & 1) == 1, should_skip)


# ---------------------------------------------------------------------------
# T7: a single linear path converges to near-zero stress
# ---------------------------------------------------------------------------
def test_linear_path_converges():
    sg = synth.linear_path(2000)
    g = O.Graph.from_synth(sg)
    c = O.init_coords(g)
    O.layout(g, c)
    assert O.sampled_path_stress(g, c)["mean"] < 1e-4
    # from a scrambled start (initial stress ~4e3) the stress falls by more than 1e6
    rng = np.random.default_rng(0)
    c1 = O.init_coords(g)
    c1[: 2 * g.n_nodes] = (rng.random(2 * g.n_nodes) * g.d_max).astype(np.float32)
    s0 = O.sampled_path_stress(g, c1)["mean"]
    c2 = c1.copy()
    O.layout(g, c2)
    assert O.sampled_path_stress(g, c2)["mean"] < s0 * 1e-6
    c3 = c1.copy()
    O.layout(g, c3, n_iters=60)
    assert O.sampled_path_stress(g, c3)["mean"] < 1e-4


def test_layout_reduces_stress_on_tiny(tiny_oracle):
    g = tiny_oracle
    c = O.init_coords(g)
    s0 = O.sps_expectation(g, c)[0]
    O.layout(g, c)
    s1 = O.sps_expectation(g, c)[0]
    assert s1 < 0.05 * s0


def test_layout_split_run_equals_full_run(tiny_oracle):
    g = tiny_oracle
    c_full = O.init_coords(g)
    O.layout(g, c_full)
    c_split = O.init_coords(g)
    O.layout(g, c_split, first_iter=0, last_iter=11)
    O.layout(g, c_split, first_iter=11, last_iter=30)
    assert np.array_equal(c_full, c_split)


def test_threaded_mode_with_one_thread_equals_sequential(tiny_oracle):
    g = tiny_oracle
    a = O.init_coords(g)
    b = a.copy()
    O.layout(g, a, first_iter=0, last_iter=3)
    O.layout(g, b, first_iter=0, last_iter=3, threads=1, term_limit=10 * g.S)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# T8: sampled path stress (Eq. 2) and path stress (Eq. 1)
# ---------------------------------------------------------------------------
def _scaled_line(g, lam):
    # a single forward path drawn on a line scaled by lam: every pair has mag = lam * d
    c = np.zeros(4 * g.n_nodes, np.float32)
    pos = g.pos
    for s in range(g.S):
        n = s
        c[2 * n] = lam * pos[s]
        c[2 * n + 1] = lam * (pos[s] + int(g.node_len[n]))
    return c


@pytest.mark.parametrize("lam", [1.0, 0.5, 2.0, 3.0])
def test_stress_of_scaled_line_is_closed_form(lam):
    sg = synth.linear_path(300, seed=4)
    g = O.Graph.from_synth(sg)
    c = _scaled_line(g, lam)
    s = O.sampled_path_stress(g, c, m=20)
    assert s["n_valid"] + s["n_skipped"] == 20 * g.S
    assert abs(s["mean"] - (lam - 1) ** 2) < 1e-9
    assert s["stddev"] < 1e-6
    ps, pairs = O.path_stress_exact(g, c)
    assert pairs == g.S * (g.S - 1) // 2
    assert abs(ps - (lam - 1) ** 2) < 1e-9
    assert abs(O.sps_expectation(g, c)[0] - (lam - 1) ** 2) < 1e-9


@pytest.mark.parametrize("lam", [0.5, 2.0])
def test_power_law_pair_stress_of_scaled_line_is_closed_form(lam):
    # every pair of a scaled straight line has stress (lam - 1)^2, whichever partner is drawn
    n = 3000
    lens = (np.arange(n) % 5 + 1).astype(np.uint32)
    g = O.Graph(lens, np.array([0, n], np.uint64), np.arange(n, dtype=np.uint32))
    pos = np.concatenate([[0], np.cumsum(lens.astype(np.int64))])
    c = np.zeros(4 * n, np.float32)
    c[0:2 * n:2] = lam * pos[:-1]
    c[1:2 * n:2] = lam * pos[1:]
    r = O.sampled_path_stress(g, c, m=3, seed=9, pairs="power_law")
    assert r["n_valid"] + r["n_skipped"] == 3 * n
    assert abs(r["mean"] - (lam - 1) ** 2) <= 1e-6 * (lam - 1) ** 2


def test_power_law_pairs_on_a_doubled_line():
    # one long path of unit nodes laid out at twice the path distance: every valid pair has
    # stress exactly 1; skipped pairs are exactly those whose two endpoints touch (d = 0), which
    # needs hop 1 with the facing endpoint coins, so they stay a small fraction (the partner rule
    # itself is pinned with the layout's sampling tests)
    n = 20000
    g = O.Graph(np.ones(n, np.uint32), np.array([0, n], np.uint64), np.arange(n, dtype=np.uint32))
    pos = np.arange(n + 1, dtype=np.int64)
    c = np.zeros(4 * n, np.float32)
    c[0:2 * n:2] = 2 * pos[:-1]
    c[1:2 * n:2] = 2 * pos[1:]
    r = O.sampled_path_stress(g, c, m=1, seed=3, pairs="power_law")
    assert r["n_valid"] + r["n_skipped"] == n
    # P(hop = 1) = 1 / H_1000(0.99) ~ 0.13, then a quarter of the coin pairs face each other
    assert 0.02 * n < r["n_skipped"] < 0.05 * n
    assert abs(r["mean"] - 1.0) < 1e-9
    # single-step paths have no power-law partner: every such pair is skipped
    g1 = O.Graph(np.array([4, 3], np.uint32), np.array([0, 1, 2], np.uint64), np.array([0, 1], np.uint32))
    r1 = O.sampled_path_stress(g1, np.zeros(8, np.float32), m=5, seed=1, pairs="power_law")
    assert r1["n_valid"] == 0 and r1["n_skipped"] == 10


def test_power_law_pairs_are_local_on_a_collapsed_layout(tiny_oracle):
    # all points at the origin: every valid pair has stress exactly 1 in both modes, and the power-law
    # pairs (hop <= 1000 steps) skip no more pairs than there are single-step paths allow
    g = tiny_oracle
    c = np.zeros(4 * g.n_nodes, np.float32)
    for mode in ("uniform", "power_law"):
        r = O.sampled_path_stress(g, c, m=2, seed=4, pairs=mode)
        assert r["n_valid"] + r["n_skipped"] == 2 * g.S
        assert abs(r["mean"] - 1.0) < 1e-12


def test_two_node_path_stress_by_hand():
    # A (len 3) then B (len 2); layout: A.s=(0,0) A.e=(3,0) B.s=(3,4) B.e=(6,4)
    g = _two_node()
    c = np.zeros(8, np.float32)
    c[0:4] = [0, 3, 3, 6]
    c[4:8] = [0, 0, 4, 4]
    # pair (A,B): combos (A.s,B.s): d=3, mag=5 -> (2/3)^2; (A.s,B.e): d=5, mag=sqrt(52);
    # (A.e,B.s): d=0 -> excluded; (A.e,B.e): d=2, mag=5 -> (3/2)^2
    v = [(2 / 3) ** 2, ((math.sqrt(52) - 5) / 5) ** 2, 1.5 ** 2]
    ps, pairs = O.path_stress_exact(g, c)
    assert pairs == 1 and abs(ps - sum(v) / 3) < 1e-6
    # the SPS estimator's expectation: all (i, j, e_i, e_j) over 2 steps with equal weight;
    # same-node pairs: (A.s,A.e) d=3 mag=3 -> 0, (B.s,B.e) d=2 mag=3 -> 1/4; same endpoints d=0
    vals = [0, 0, 0.25, 0.25] + v + v
    assert abs(O.sps_expectation(g, c)[0] - sum(vals) / len(vals)) < 1e-6


def test_sps_matches_its_expectation_within_ci(tiny_oracle):
    g = tiny_oracle
    c = O.init_coords(g)
    O.layout(g, c, first_iter=0, last_iter=20)
    exp_mean, frac_valid = O.sps_expectation(g, c)
    s = O.sampled_path_stress(g, c, m=100, seed=7)
    n = s["n_valid"]
    assert abs(s["mean"] - exp_mean) < 3.29 * s["stddev"] / math.sqrt(n)
    assert abs(n / (100 * g.S) - frac_valid) < 5 * math.sqrt(frac_valid * (1 - frac_valid) / (100 * g.S)) + 1e-9
    assert s["ci_lo"] < s["mean"] < s["ci_hi"]
    assert abs((s["ci_hi"] - s["ci_lo"]) / 2 - 1.96 * s["stddev"] / math.sqrt(n)) < 1e-12
    # a second seed gives a consistent value (the metric is stable across seeds)
    s2 = O.sampled_path_stress(g, c, m=100, seed=8)
    assert abs(s2["mean"] - s["mean"]) < 4.0 * s["stddev"] / math.sqrt(n)


def test_sps_pair_count_is_m_times_path_length(tiny_oracle):
    g = tiny_oracle
    c = O.init_coords(g)
    for m in [1, 3, 10]:
        s = O.sampled_path_stress(g, c, m=m)
        assert s["n_valid"] + s["n_skipped"] == m * g.S


# ---------------------------------------------------------------------------
# T8b: Eq. 2's pairs in window-major order (reading R21): the same law
# ---------------------------------------------------------------------------
def _small_graph_with_empty_path():
    # paths of 5, 0 and 3 steps over 8 nodes of length 3
    return O.Graph(np.full(8, 3, np.uint32), np.array([0, 5, 5, 8], np.uint64), np.arange(8, dtype=np.uint32))


def test_sps_segments_tile_the_paths_along_window_boundaries(tiny_oracle):
    graphs = [tiny_oracle, _disjoint_paths_fixed_point()[0], _small_graph_with_empty_path(),
              O.Graph.from_synth(synth.linear_path(300, seed=4))]
    for g in graphs:
        start, path = O.sps_segments(g)
        sh = O.window_shift(g.S)
        off = g.path_off.astype(np.int64)
        assert start[0] == 0 and int(start[-1]) == g.S and np.all(np.diff(start.astype(np.int64)) > 0)
        for k in range(len(path)):
            a, b, p = int(start[k]), int(start[k + 1]), int(path[k])
            assert off[p] <= a < b <= off[p + 1], "a segment lies inside one path"
            assert a >> sh == (b - 1) >> sh, "a segment lies inside one window"
            assert a % (1 << sh) == 0 or a == off[p], "segments are maximal"
            assert b % (1 << sh) == 0 or b == off[p + 1], "segments are maximal"


def test_sps_segment_counts_are_the_histogram_of_the_plain_pair_draws():
    # brute force over the plain pair enumeration of Eq. 2 (Philox stream 1 at counter q)
    g, _ = _disjoint_paths_fixed_point()
    m, seed, gid = 3, 7, 2
    start, path = O.sps_segments(g)
    off = g.path_off.astype(np.int64)
    brute = np.zeros(len(path), np.int64)
    for p in range(len(off) - 1):
        length = int(off[p + 1] - off[p])
        for q in range(m * int(off[p]), m * int(off[p + 1])):
            r = O.philox([q & 0xFFFFFFFF, q >> 32, 0, (1 << 24) | gid], [seed, 0])
            i = int(off[p]) + (((int(r[0]) | (int(r[1]) << 32)) * length) >> 64)
            brute[np.searchsorted(start, i, side="right") - 1] += 1
    counts = O.sps_segment_counts(g, m, seed, gid).astype(np.int64)
    assert np.array_equal(counts, brute)
    per_path = np.bincount(path.astype(np.int64), weights=counts, minlength=len(off) - 1)
    assert np.array_equal(per_path.astype(np.int64), m * np.diff(off))


def test_sps_windowed_pairs_follow_the_uniform_law(tiny_synth, tiny_oracle):
    g, sg = tiny_oracle, tiny_synth
    m = 30
    i, j, e = O.sps_windowed_pairs(g, m, 7)
    assert len(i) == m * g.S
    start, path = O.sps_segments(g)
    counts = O.sps_segment_counts(g, m, 7).astype(np.int64)
    seg_of_slot = np.repeat(np.arange(len(counts)), counts)
    assert np.all((i >= start[seg_of_slot]) & (i < start[seg_of_slot + 1])), "slot step outside its segment"
    pi, pj = _path_of(sg.path_off, i), _path_of(sg.path_off, j)
    assert np.array_equal(pi, pj), "the partner lies on the same path"
    assert np.array_equal(np.bincount(pi, minlength=sg.n_paths), m * np.diff(sg.path_off.astype(np.int64)))
    dof = g.S - 1
    for x in (i, j):  # both ends uniform over the steps: every step has density m
        c = np.bincount(x.astype(np.int64), minlength=g.S)
        chi2 = float(np.sum((c - m) ** 2 / m))
        assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof)
    # i and j independent: relative positions in the longest path, 8 x 8 table
    lens = np.diff(sg.path_off.astype(np.int64))
    p0 = int(np.argmax(lens))
    sel = pi == p0
    bi = ((i[sel].astype(np.int64) - int(sg.path_off[p0])) * 8) // int(lens[p0])
    bj = ((j[sel].astype(np.int64) - int(sg.path_off[p0])) * 8) // int(lens[p0])
    tab = np.bincount(bi * 8 + bj, minlength=64).reshape(8, 8).astype(np.float64)
    exp = np.outer(tab.sum(1), tab.sum(0)) / tab.sum()
    chi2 = float(np.sum((tab - exp) ** 2 / exp))
    assert chi2 < 49 + 5 * math.sqrt(2 * 49)
    for b in (0, 1):
        assert abs(((e >> b) & 1).mean() - 0.5) < 0.01


@pytest.mark.parametrize("lam", [1.0, 0.5, 2.0])
def test_sps_on_lines_per_path_is_closed_form(lam):
    # each path on its own line at its path coordinates, scaled by lam: a same-path pair has
    # mag = lam * d, a pair across paths would not (the lines lie 1000 * lam apart)
    g, c = _disjoint_paths_fixed_point()
    c = c * np.float32(lam)
    for pairs in ("uniform", "uniform_windowed"):
        s = O.sampled_path_stress(g, c, m=7, pairs=pairs)
        assert s["n_valid"] + s["n_skipped"] == 7 * g.S
        assert abs(s["mean"] - (lam - 1) ** 2) < 1e-12
        assert s["stddev"] < 1e-9


def test_sps_windowed_matches_its_expectation_within_ci(tiny_oracle):
    g = tiny_oracle
    c = O.init_coords(g)
    O.layout(g, c, first_iter=0, last_iter=20)
    exp_mean, frac_valid = O.sps_expectation(g, c)
    s = O.sampled_path_stress(g, c, m=100, seed=7, pairs="uniform_windowed")
    n = s["n_valid"]
    assert n + s["n_skipped"] == 100 * g.S
    assert abs(s["mean"] - exp_mean) < 3.29 * s["stddev"] / math.sqrt(n)
    assert abs(n / (100 * g.S) - frac_valid) < 5 * math.sqrt(frac_valid * (1 - frac_valid) / (100 * g.S)) + 1e-9
    assert abs((s["ci_hi"] - s["ci_lo"]) / 2 - 1.96 * s["stddev"] / math.sqrt(n)) < 1e-12


# ---------------------------------------------------------------------------
# Differentiable form: loss and gradient
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [0.5, 2.0])
def test_loss_of_scaled_line_is_closed_form(lam):
    sg = synth.linear_path(500, seed=2)
    g = O.Graph.from_synth(sg)
    c = _scaled_line(g, lam)
    L, n, grad = O.stress_loss_grad(g, c, 20000, seed=11)
    assert n > 0.9 * 20000 and abs(L - (lam - 1) ** 2) < 1e-9


def test_gradient_matches_finite_differences():
    sg = synth.generate(60, 0.2, 3, 9)
    g = O.Graph.from_synth(sg)
    rng = np.random.default_rng(1)
    c = (O.init_coords(g) + rng.normal(scale=3.0, size=4 * g.n_nodes)).astype(np.float32)
    L, n, grad = O.stress_loss_grad(g, c, 3000, seed=11, step=2)
    # the loss as a function of FP64 coordinates: perturb through float32-exact steps
    idx = rng.choice(4 * g.n_nodes, size=40, replace=False)
    for k in idx:
        h = np.float32(2.0 ** (np.floor(np.log2(max(1.0, abs(float(c[k]))))) - 14))
        cp, cm = c.copy(), c.copy()
        cp[k] += h
        cm[k] -= h
        Lp = O.stress_loss_grad(g, cp, 3000, seed=11, step=2, want_grad=False)[0]
        Lm = O.stress_loss_grad(g, cm, 3000, seed=11, step=2, want_grad=False)[0]
        fd = (Lp - Lm) / (float(cp[k]) - float(cm[k]))
        assert abs(fd - grad[k]) <= 1e-4 * max(abs(grad[k]), 1e-3 * np.abs(grad).max()), (k, fd, grad[k])


# ---------------------------------------------------------------------------
# The loss pairs in window-major order (reading R22): the law of the plain
# loss pairs listed segment by segment
# ---------------------------------------------------------------------------
def test_loss_shift_rule():
    # 2^10-step windows, halved (down to 2^6) while fewer than 16, doubled while more than 32768
    cases = {0: 6, 1: 6, 1000: 6, 16 * 64: 6, 16 * 64 + 1: 6, 16 * 128: 7, 14416: 9, 16 * 1024: 10, 10**6: 10,
             32768 * 1024: 10, 32768 * 1024 + 1: 11, 29_016_220: 10, 408_037_251: 14}
    for S, sh in cases.items():
        assert O.loss_shift(S) == sh, (S, O.loss_shift(S), sh)
        n = -(-S // (1 << sh))
        assert n <= 32768
        assert sh == 6 or n >= 16 or sh > 10


def test_loss_segments_tile_the_paths_along_their_window_boundaries(tiny_oracle):
    graphs = [tiny_oracle, _disjoint_paths_fixed_point()[0], _small_graph_with_empty_path(),
              O.Graph.from_synth(synth.linear_path(3000, seed=4))]
    for g in graphs:
        start, path = O.loss_segments(g)
        sh = O.loss_shift(g.S)
        off = g.path_off.astype(np.int64)
        assert start[0] == 0 and int(start[-1]) == g.S and np.all(np.diff(start.astype(np.int64)) > 0)
        for k in range(len(path)):
            a, b, p = int(start[k]), int(start[k + 1]), int(path[k])
            assert off[p] <= a < b <= off[p + 1], "a segment lies inside one path"
            assert a >> sh == (b - 1) >> sh, "a segment lies inside one window"
            assert a % (1 << sh) == 0 or a == off[p], "segments are maximal"
            assert b % (1 << sh) == 0 or b == off[p + 1], "segments are maximal"


def test_loss_segment_counts_are_the_histogram_of_the_loss_draws():
    # brute force over the plain loss pairs (Philox stream 2 at counter q, word 2 = step)
    g, _ = _disjoint_paths_fixed_point()
    n_pairs, seed, gid, step = 3000, 11, 3, 5
    start, path = O.loss_segments(g)
    brute = np.zeros(len(path), np.int64)
    for q in range(n_pairs):
        r = O.philox([q & 0xFFFFFFFF, q >> 32, step, (2 << 24) | gid], [seed, 0])
        i = ((int(r[0]) | (int(r[1]) << 32)) * g.S) >> 64
        brute[np.searchsorted(start, i, side="right") - 1] += 1
    counts = O.loss_segment_counts(g, n_pairs, seed=seed, step=step, graph_id=gid).astype(np.int64)
    assert np.array_equal(counts, brute) and counts.sum() == n_pairs


def test_loss_windowed_pairs_follow_the_power_law(tiny_synth, tiny_oracle):
    from scipy.stats import chi2 as chi2_dist
    g, sg = tiny_oracle, tiny_synth
    n_pairs, W = 400_000, 200  # paths of ~1,800 steps: room for hops up to W both ways in the middle
    i, j, f = O.loss_windowed_pairs(g, n_pairs, 0, n_pairs, seed=11, step=3, window=W)
    i, j = i.astype(np.int64), j.astype(np.int64)
    start, path = O.loss_segments(g)
    counts = O.loss_segment_counts(g, n_pairs, seed=11, step=3).astype(np.int64)
    seg_of_slot = np.repeat(np.arange(len(counts)), counts)
    assert np.all((i >= start[seg_of_slot]) & (i < start[seg_of_slot + 1])), "slot step outside its segment"
    # i uniform over all steps
    c = np.bincount(i, minlength=g.S)
    exp = n_pairs / g.S
    chi2 = float(np.sum((c - exp) ** 2 / exp))
    assert chi2 < chi2_dist.ppf(1 - 1e-4, g.S - 1)
    # j on the path of i, at most W steps away, never i itself
    pi, pj = _path_of(sg.path_off, i), _path_of(sg.path_off, j)
    assert np.array_equal(pi, pj) and np.all(np.abs(j - i) <= W) and np.all(j != i)
    # direction and endpoint coins fair; hop ~ Zipf(0.99) on [1, W] where both directions have room
    off = sg.path_off.astype(np.int64)
    room = np.minimum(i - off[pi], off[pi + 1] - 1 - i)
    inner = room >= W
    z = np.abs(j - i)[inner]
    pmf = 1.0 / np.arange(1, W + 1) ** 0.99
    pmf /= pmf.sum()
    obs = np.bincount(z, minlength=W + 1)[1:]
    bins = np.concatenate([np.arange(0, 20), np.unique(np.geomspace(20, W - 1, 12).astype(int))])
    ob = np.add.reduceat(obs, bins)
    ex = np.add.reduceat(pmf * inner.sum(), bins)
    assert float(np.sum((ob - ex) ** 2 / ex)) < chi2_dist.ppf(1 - 1e-4, len(bins) - 1)
    assert abs((j < i)[inner].mean() - 0.5) < 0.01
    for b in (0, 1):
        assert abs(((f >> b) & 1).mean() - 0.5) < 0.01


@pytest.mark.parametrize("lam", [0.5, 2.0])
def test_windowed_loss_on_lines_per_path_is_closed_form(lam):
    # each path on its own line at its path coordinates scaled by lam: every same-path pair has
    # mag = lam * d, so the loss is (lam - 1)^2; a pair across paths would not give it
    g, c = _disjoint_paths_fixed_point()
    c = c * np.float32(lam)
    L, n, grad = O.stress_loss_grad_windowed(g, c, 20000, seed=11, step=1)
    assert n > 0.9 * 20000 and abs(L - (lam - 1) ** 2) < 1e-12
    Lp, n_p, _ = O.stress_loss_grad(g, c, 20000, seed=11, step=1, want_grad=False)
    assert abs(Lp - L) < 1e-12


def test_windowed_gradient_matches_finite_differences():
    sg = synth.generate(60, 0.2, 3, 9)
    g = O.Graph.from_synth(sg)
    rng = np.random.default_rng(2)
    c = (O.init_coords(g) + rng.normal(scale=3.0, size=4 * g.n_nodes)).astype(np.float32)
    L, n, grad = O.stress_loss_grad_windowed(g, c, 3000, seed=11, step=4)
    idx = rng.choice(4 * g.n_nodes, size=40, replace=False)
    for k in idx:
        h = np.float32(2.0 ** (np.floor(np.log2(max(1.0, abs(float(c[k]))))) - 14))
        cp, cm = c.copy(), c.copy()
        cp[k] += h
        cm[k] -= h
        Lp = O.stress_loss_grad_windowed(g, cp, 3000, seed=11, step=4, want_grad=False)[0]
        Lm = O.stress_loss_grad_windowed(g, cm, 3000, seed=11, step=4, want_grad=False)[0]
        fd = (Lp - Lm) / (float(cp[k]) - float(cm[k]))
        assert abs(fd - grad[k]) <= 1e-4 * max(abs(grad[k]), 1e-3 * np.abs(grad).max()), (k, fd, grad[k])


def test_windowed_and_plain_loss_estimate_the_same_expectation(tiny_oracle):
    g = tiny_oracle
    c = O.init_coords(g)
    O.layout(g, c, first_iter=0, last_iter=6)
    plain = [O.stress_loss_grad(g, c, 50_000, seed=11, step=s, want_grad=False)[0] for s in range(1, 9)]
    wind = [O.stress_loss_grad_windowed(g, c, 50_000, seed=11, step=s, want_grad=False)[0] for s in range(1, 9)]
    mp, mw = float(np.mean(plain)), float(np.mean(wind))
    se = math.sqrt(np.var(plain, ddof=1) / 8 + np.var(wind, ddof=1) / 8)
    assert abs(mp - mw) < 4 * se


def test_init_coords_follow_first_visits(tiny_synth, tiny_oracle):
    g, sg = tiny_oracle, tiny_synth
    c = O.init_coords(g, seed=5, jitter=10.0)
    X, Y = c[: 2 * g.n_nodes], c[2 * g.n_nodes:]
    pos = g.pos
    seen = set()
    for s in range(g.S):
        n = int(int(sg.step_node[s]) & 0x7FFFFFFF)
        if n in seen:
            continue
        seen.add(n)
        assert X[2 * n] == np.float32(pos[s]) and X[2 * n + 1] == np.float32(pos[s] + int(sg.node_len[n]))
    assert np.all(np.abs(Y) <= 5.0) and abs(float(Y.mean())) < 0.5


# ---------------------------------------------------------------------------
# The power-law direction coin (Alg. 1's power-law partner, reading R4): bit 2
# of word 3 of the term's own draw, fair, independent of the group's cooling
# coin and of both endpoint coins, and flipped only where the path has no room
# in the drawn direction
# ---------------------------------------------------------------------------
def test_power_law_direction_coin_is_bit2_fair_and_independent():
    from scipy.stats import chi2 as chi2_dist
    from scipy.stats import chi2_contingency
    L = 3000
    g = O.Graph(np.full(L, 3, np.uint32), np.array([0, L], np.uint64), np.arange(L, dtype=np.uint32))
    N = 64 * 4096
    it = 21  # a cooling iteration: every term takes the power-law partner
    i, j, f = O.sample_terms(g, it, 0, N)
    i, j = i.astype(np.int64), j.astype(np.int64)
    down = (j < i).astype(np.int64)
    assert np.all(j != i)
    inner = (i > 0) & (i < L - 1)
    # the definition: bit 2 of r3 of the term's own draw (counter (t, 0, iter, stream 0 | graph 0))
    bit2 = np.array([(int(O.philox([t, 0, it, 0], [24301, 0])[3]) >> 2) & 1 for t in range(N)])
    lead3 = np.array([(int(O.philox([t - t % 64, 0, it, 0], [24301, 0])[3]) >> 3) & 1 for t in range(0, N, 64)])
    group = np.repeat(lead3, 64)
    assert np.array_equal(down[inner], bit2[inner])
    # flips only at the path ends, towards the inside
    assert np.all(down[i == 0] == 0) and np.all(down[i == L - 1] == 1)
    # fair and independent of both endpoint coins: chi-square over the 8 cells (down, e_i, e_j)
    ei, ej, gi = f[inner] & 1, (f[inner] >> 1) & 1, group[inner]

    def fair_p(dirn):
        counts = np.bincount(dirn * 4 + ei * 2 + ej, minlength=8)
        e = counts.sum() / 8
        return chi2_dist.sf(float(np.sum((counts - e) ** 2 / e)), 7)

    def indep_p(dirn):  # 2 x 2 contingency with the group coin (shared by 64 terms, so not a uniform cell)
        return chi2_contingency(np.array([[np.sum((dirn == x) & (gi == y)) for y in (0, 1)] for x in (0, 1)]))[1]

    assert fair_p(down[inner]) > 1e-4 and indep_p(down[inner]) > 1e-4
    # a direction taken from the group coin or an endpoint coin fails one of the two
    for wrong in (gi, ei, ej):
        assert min(fair_p(wrong), indep_p(wrong)) < 1e-12


# ---------------------------------------------------------------------------
# The initial layout's jitter (reading R11): Y[k] = jitter * (u - 1/2) with
# u = (r0 >> 8) / 2^24 from Philox stream 3 at counter k, in FP32
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,graph_id,jitter", [(5, 0, 10.0), ((7 << 32) | 3, 9, 2.5)])
def test_init_jitter_follows_the_stream3_draw(tiny_oracle, seed, graph_id, jitter):
    g = tiny_oracle
    c = O.init_coords(g, seed=seed, jitter=jitter, graph_id=graph_id)
    Y = c[2 * g.n_nodes:]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in list(range(0, 2 * g.n_nodes, 97)) + [2 * g.n_nodes - 1]:
        r0 = int(O.philox([k, 0, 0, (3 << 24) | graph_id], key)[0])
        u = np.float32(r0 >> 8) * np.float32(1.0 / 16777216.0)
        assert Y[k] == np.float32(jitter) * (u - np.float32(0.5)), k


def test_init_jitter_is_uniform_and_independent_between_endpoints(tiny_oracle):
    from scipy.stats import chi2 as chi2_dist
    g = tiny_oracle
    Y = O.init_coords(g, seed=5, jitter=10.0)[2 * g.n_nodes:].astype(np.float64)
    u = Y / 10.0 + 0.5
    assert np.all((u >= 0) & (u < 1))
    counts = np.bincount(np.floor(u * 16).astype(np.int64), minlength=16)
    e = u.size / 16
    assert chi2_dist.sf(float(np.sum((counts - e) ** 2 / e)), 15) > 1e-4
    # the two endpoints of a node draw independently
    assert abs(np.corrcoef(u[0::2], u[1::2])[0, 1]) < 4 / np.sqrt(g.n_nodes)


# ---------------------------------------------------------------------------
# The threaded evaluation of Eq. 2 (stored results of large layouts) against
# the one-thread evaluation: the same pairs, so equal counts and sums up to
# the rounding of the summation order
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("pairs", ["uniform", "uniform_windowed"])
@pytest.mark.parametrize("threads", [2, 3, 7])
def test_threaded_sps_equals_one_thread(tiny_oracle, pairs, threads):
    g = tiny_oracle
    rng = np.random.default_rng(3)
    c = (O.init_coords(g) + rng.normal(scale=40.0, size=4 * g.n_nodes)).astype(np.float32)
    a = O.sampled_path_stress(g, c, m=20, seed=7, pairs=pairs)
    b = O.sampled_path_stress(g, c, m=20, seed=7, pairs=pairs, threads=threads)
    assert a["n_valid"] == b["n_valid"] and a["n_skipped"] == b["n_skipped"]
    for k in ("sum", "sumsq_dev", "mean", "stddev"):
        assert b[k] == pytest.approx(a[k], rel=1e-12), k


def test_threaded_sps_on_a_graph_with_empty_paths():
    node_len = np.array([2, 3, 1, 4, 5], np.uint32)
    off = np.array([0, 0, 3, 3, 5, 5], np.uint64)
    steps = np.array([0, 1, 2, 3 | 0x80000000, 4], np.uint32)
    g = O.Graph(node_len, off, steps)
    c = np.linspace(-5, 5, 4 * 5).astype(np.float32)
    for pairs in ("uniform", "uniform_windowed"):
        a = O.sampled_path_stress(g, c, m=7, seed=1, pairs=pairs)
        b = O.sampled_path_stress(g, c, m=7, seed=1, pairs=pairs, threads=4)
        assert (a["n_valid"], a["n_skipped"]) == (b["n_valid"], b["n_skipped"])
        assert b["sum"] == pytest.approx(a["sum"], rel=1e-12)


@pytest.mark.parametrize("pairs", ["uniform", "power_law", "uniform_windowed"])
def test_sps_outliers_list_the_pairs_of_eq2(tiny_oracle, pairs):
    # with a threshold below every stress the listing is every valid pair of Eq. 2: its count and its sum are
    # the estimator's; a threshold keeps exactly the pairs above it
    g = tiny_oracle
    c = O.init_coords(g)
    O.layout(g, c, first_iter=0, last_iter=8)
    s = O.sampled_path_stress(g, c, m=5, seed=7, pairs=pairs)
    n, i, j, e, st = O.sps_outliers(g, c, 5, -1.0, max_out=5 * g.S + 1, seed=7, pairs=pairs)
    assert n == s["n_valid"] == len(st)
    assert abs(float(np.sum(st)) - s["sum"]) <= 1e-9 * abs(s["sum"])
    thr = float(np.quantile(st, 0.99))
    n2, i2, j2, e2, st2 = O.sps_outliers(g, c, 5, thr, seed=7, pairs=pairs)
    keep = st > thr
    assert n2 == int(keep.sum()) and np.array_equal(st2, st[keep]) and np.array_equal(i2, i[keep])
    n3, *_ = O.sps_outliers(g, c, 5, thr, max_out=3, seed=7, pairs=pairs)
    assert n3 == n2


@pytest.mark.parametrize("pairs", ["uniform", "power_law", "uniform_windowed"])
def test_sps_compare_pins(tiny_oracle, pairs):
    # a layout against itself: ratio exactly 1 with a zero-width interval, both means the estimator's
    g = tiny_oracle
    c = O.init_coords(g)
    O.layout(g, c, first_iter=0, last_iter=8)
    s = O.sampled_path_stress(g, c, m=5, seed=7, pairs=pairs)
    r = O.sps_compare(g, c, c, m=5, seed=7, pairs=pairs)
    assert r["n_valid"] == s["n_valid"] and r["n_skipped"] == s["n_skipped"]
    assert r["mean_a"] == r["mean_b"] and abs(r["mean_a"] - s["mean"]) <= 1e-12 * s["mean"]
    assert r["ratio"] == 1.0 and r["ratio_ci_lo"] == 1.0 and r["ratio_ci_hi"] == 1.0
    assert abs(r["sd_a"] - s["stddev"]) <= 1e-9 * s["stddev"]


@pytest.mark.parametrize("pairs", ["uniform", "uniform_windowed"])
def test_sps_compare_on_scaled_lines_is_closed_form(pairs):
    # per-path lines scaled by lam and by mu: every pair's stress is (lam - 1)^2 and (mu - 1)^2
    g, c = _disjoint_paths_fixed_point()
    lam, mu = 2.0, 0.5
    r = O.sps_compare(g, c * np.float32(lam), c * np.float32(mu), m=7, pairs=pairs)
    assert abs(r["mean_a"] - (lam - 1) ** 2) < 1e-12 and abs(r["mean_b"] - (mu - 1) ** 2) < 1e-12
    assert abs(r["ratio"] - (lam - 1) ** 2 / (mu - 1) ** 2) < 1e-12
    assert r["sd_diff"] < 1e-9 and r["ratio_ci_hi"] - r["ratio_ci_lo"] < 1e-9
