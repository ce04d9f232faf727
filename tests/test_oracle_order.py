"""Pins of the oracle's ordering (Alg. 1 with Eq. 3) against independent facts."""
import itertools

import numpy as np
import pytest

import synth
from oracle import varlingam as O


def _order_violations(order, B0):
    pos = {int(v): k for k, v in enumerate(order)}
    eff, cau = np.nonzero(B0)
    return int(sum(pos[int(i)] < pos[int(j)] for i, j in zip(eff, cau)))


def test_hand_built_total_order_is_recovered():
    rng = np.random.default_rng(0)
    for m in (1, 2, 3, 7, 20):
        true = rng.permutation(m)
        pos = np.empty(m, int)
        pos[true] = np.arange(m)
        S = np.where(pos[:, None] < pos[None, :], 1.0, -1.0) * rng.uniform(0.1, 1, (m, m))
        S = np.triu(S, 1) - np.triu(S, 1).T          # antisymmetric, sign from the order
        S[np.tril_indices(m, -1)] = -S.T[np.tril_indices(m, -1)]
        order, margin = O.approx_order(S)
        assert list(order) == list(true)
        assert margin[-1] == np.inf and np.all(margin[:-1] > 0)


def test_ties_go_to_lowest_index_and_margin_zero():
    order, margin = O.approx_order(np.zeros((4, 4)))
    assert list(order) == [0, 1, 2, 3]
    assert np.all(margin[:-1] == 0.0)


def test_duplicated_variables_tie_at_every_pair():
    """Variables 2i and 2i+1 with identical rows and columns of S (their pair scores 0) keep equal
    M at every step while both are candidates, so the lowest-index rule takes 2i first and the
    step that takes it has margin exactly 0."""
    h = 30
    rng = np.random.default_rng(7)
    A = rng.normal(size=(h, h))
    A = A - A.T
    S = np.kron(A, np.ones((2, 2)))
    for i in range(h):
        S[2 * i, 2 * i + 1] = S[2 * i + 1, 2 * i] = 0.0
    order, margin = O.approx_order(S)
    pos = np.empty(2 * h, int)
    pos[order] = np.arange(2 * h)
    assert np.all(pos[0::2] < pos[1::2])
    assert np.all(margin[pos[0::2]] == 0.0)


def test_pure_python_loop_form_small():
    """Alg. 1 written as explicit loops over U (tiny m), compared element by element."""
    rng = np.random.default_rng(4)
    for m in (2, 3, 5, 8):
        A = rng.normal(size=(m, m))
        S = A - A.T
        U = list(range(m))
        ref = []
        for _ in range(m):
            best, best_val = None, None
            for i in U:
                tot = 0.0
                for j in U:
                    if j != i and S[i, j] < 0:
                        tot += S[i, j] * S[i, j]
                if best_val is None or tot < best_val:
                    best, best_val = i, tot
            ref.append(best)
            U.remove(best)
        order, _ = O.approx_order(S)
        assert list(order) == ref


def test_m2_heuristic_equals_iterative_and_first_pick_equal():
    for seed in range(5):
        inst = synth.make_custom(2, 2000, 1, "uniform", seed)
        _, _, E = O.fit_var(inst.X_parity, 1)
        _, _, S = O.pairwise_stats(E)
        order, _ = O.approx_order(S)
        assert list(order) == list(O.directlingam_iterative(E))
    for seed in range(3):
        inst = synth.make_custom(6, 2000, 1, "laplace", seed)
        _, _, E = O.fit_var(inst.X_parity, 1)
        _, _, S = O.pairwise_stats(E)
        order, _ = O.approx_order(S)
        assert order[0] == O.directlingam_iterative(E)[0]


@pytest.mark.slow
def test_tiny_m_agreement_with_iterative():
    """Brute force on tiny inputs: for strongly non-Gaussian (uniform) data with m <= 5 the
    heuristic and the full iterative DirectLiNGAM recover orders that are both consistent with
    the true DAG in most seeds (statistical; the heuristic has no guarantee)."""
    agree = 0
    seeds = range(30)
    for seed in seeds:
        m = 3 + seed % 3
        inst = synth.make_custom(m, 5000, 1, "uniform", seed, edge_prob=0.5, w_lo=0.4, w_hi=0.9)
        _, _, E = O.fit_var(inst.X_parity, 1)
        _, _, S = O.pairwise_stats(E)
        h, _ = O.approx_order(S)
        it = O.directlingam_iterative(E)
        if _order_violations(h, inst.B0) == _order_violations(it, inst.B0) == 0:
            agree += 1
    assert agree >= 0.9 * len(seeds)


@pytest.mark.slow
def test_recovery_of_generating_order_small_workload():
    viol = []
    for seed in range(10):
        inst = synth.make_instance(synth.SMALL, seed)
        res = O.fit(inst.X_parity, 1)
        viol.append(_order_violations(res["order"], inst.B0))
    assert np.median(viol) == 0


def test_aggregate_scores_over_current_set():
    S = np.array([[0.0, -1.0, 2.0], [1.0, 0.0, -3.0], [-2.0, 3.0, 0.0]])
    np.testing.assert_array_equal(O.aggregate_scores(S, [0, 1, 2]), [1.0, 9.0, 4.0])
    np.testing.assert_array_equal(O.aggregate_scores(S, [0, 2]), [0.0, 4.0])


def test_order_is_a_permutation():
    A = np.random.default_rng(1).normal(size=(30, 30))
    order, _ = O.approx_order(A - A.T)
    assert sorted(order) == list(range(30))


def test_incremental_update_equals_recompute():
    """Removing c from U lowers every M_i by min(0, S[i, c])^2 (the O(m^2) form a GPU pass can
    use) -- checked against the oracle's from-scratch O(m^3) recompute."""
    rng = np.random.default_rng(8)
    A = rng.normal(size=(25, 25))
    S = A - A.T
    order, _ = O.approx_order(S)
    U = list(range(25))
    M = O.aggregate_scores(S, U)
    Md = dict(zip(U, M))
    for c in order[:-1]:
        U.remove(int(c))
        for i in U:
            Md[i] -= min(0.0, S[i, c]) ** 2
        ref = O.aggregate_scores(S, U)
        np.testing.assert_allclose([Md[i] for i in U], ref, atol=1e-12)


def test_exhaustive_tiny_permutations():
    """For m = 4, every relabelling of the variables relabels the order (equivariance)."""
    A = np.random.default_rng(2).normal(size=(4, 4))
    S = A - A.T
    order, _ = O.approx_order(S)
    for P in itertools.permutations(range(4)):
        P = np.array(P)
        oP, _ = O.approx_order(S[np.ix_(P, P)])
        # variable k of the permuted problem is variable P[k] of the original one
        assert list(P[oP]) == list(order)


def test_hybrid_reduces_to_the_two_searches():
    """k exact steps then the heuristic on the refined data: k = 0 is Alg. 1 on E, k >= m - 1
    the original search, and any k keeps the original search's first k picks."""
    for seed in range(3):
        inst = synth.make_custom(6, 1500, 1, "laplace", 40 + seed, edge_prob=0.4)
        _, _, E = O.fit_var(inst.X_parity, 1)
        _, _, S = O.pairwise_stats(E)
        heur, _ = O.approx_order(S)
        full = O.directlingam_iterative(E)
        assert list(O.directlingam_iterative(E, k_exact=0)) == list(heur)
        assert list(O.directlingam_iterative(E, k_exact=5)) == list(full)
        assert list(O.directlingam_iterative(E, k_exact=6)) == list(full)
        for k in (1, 2, 3):
            hyb = O.directlingam_iterative(E, k_exact=k)
            assert sorted(hyb.tolist()) == list(range(6))
            assert list(hyb[:k]) == list(full[:k])


def test_hybrid_recovers_the_generating_order():
    """Strongly non-Gaussian data with a known DAG: every split point gives an order consistent
    with the generating B0."""
    inst = synth.make_custom(5, 6000, 1, "uniform", 3, edge_prob=0.6, w_lo=0.5, w_hi=0.9)
    _, _, E = O.fit_var(inst.X_parity, 1)
    for k in range(6):
        assert _order_violations(O.directlingam_iterative(E, k_exact=k), inst.B0) == 0, k


def test_hybrid_walker_accepts_the_oracle_and_rejects_a_swap():
    """The GPU tests' hybrid walker: the oracle's own hybrid order passes it; the same order
    with two clearly separated picks of the heuristic tail swapped does not."""
    import parity as PA
    inst = synth.make_custom(6, 1500, 1, "laplace", 41, edge_prob=0.4)
    _, _, E = O.fit_var(inst.X_parity, 1)
    for k in (1, 2, 3):
        hyb = O.directlingam_iterative(E, k_exact=k)
        assert PA.hybrid_order_violations(hyb, E, k) == []
        bad = hyb.copy()
        bad[k], bad[-1] = bad[-1], bad[k]
        v = PA.hybrid_order_violations(bad, E, k)
        assert v and v[0][0] == k
        early = hyb.copy()
        early[0], early[-1] = early[-1], early[0]
        assert PA.hybrid_order_violations(early, E, k)[0][0] == 0


def test_margins_by_hand():
    """Margins of Alg. 1 on a small integer score matrix, worked out by hand:
    S01 = 1, S02 = -2, S03 = 3, S12 = 1, S13 = -1, S23 = 2 (S = -S^T).
      U = {0,1,2,3}: M = (4, 1 + 1, 1, 9 + 4) = (4, 2, 1, 13)  -> pick 2, margin 2 - 1 = 1
      U = {0,1,3}:   M = (0, 1 + 1, 9)                         -> pick 0, margin 2 - 0 = 2
      U = {1,3}:     M = (1, 0)                                -> pick 3, margin 1 - 0 = 1
      U = {1}:                                                  -> pick 1, margin +inf
    At the first step the runner-up (variable 1) is not the next pick (variable 0), so a
    margin taken against the next pick, the largest M or a removed variable fails here, as
    does the sign of the difference."""
    S = np.zeros((4, 4))
    for (i, j), v in {(0, 1): 1.0, (0, 2): -2.0, (0, 3): 3.0, (1, 2): 1.0, (1, 3): -1.0,
                      (2, 3): 2.0}.items():
        S[i, j], S[j, i] = v, -v
    order, margin = O.approx_order(S)
    assert list(order) == [2, 0, 3, 1]
    assert list(margin) == [1.0, 2.0, 1.0, np.inf]
    # a relabelling moves the same margins with the variables
    P = np.array([3, 1, 0, 2])
    oP, mP = O.approx_order(S[np.ix_(P, P)])
    assert list(P[oP]) == [2, 0, 3, 1] and list(mP) == [1.0, 2.0, 1.0, np.inf]


def test_margin_is_exact_second_minus_first_with_fractional_scores():
    """Scores that are exact binary fractions, so every M is exact: U = {0,1,2},
    S01 = -0.5, S02 = 0.25, S12 = -0.75: M = (0.25, 0.5625, 0.0625) -> pick 2, margin
    0.25 - 0.0625 = 0.1875; then U = {0,1}: M = (0.25, 0) -> pick 1, margin 0.25."""
    S = np.zeros((3, 3))
    for (i, j), v in {(0, 1): -0.5, (0, 2): 0.25, (1, 2): -0.75}.items():
        S[i, j], S[j, i] = v, -v
    order, margin = O.approx_order(S)
    assert list(order) == [2, 1, 0]
    assert list(margin) == [0.1875, 0.25, np.inf]
