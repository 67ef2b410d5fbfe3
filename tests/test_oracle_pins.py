"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

Each test ties one oracle function to something other than itself: a value the
paper prints, a closed form, a library routine used as an independent check, an
exact rational computation, brute force, or an invariant.  Chosen so that a
dropped term, a wrong sign or index, or a transposed operand fails one of them.
"""
import itertools
import math
import os
import statistics
from fractions import Fraction

import numpy as np
import pytest
import scipy.special
import scipy.stats

from paper_2501_03381_amd import synth

HALF_LOG_2PIE = 0.5 * math.log(2 * math.pi * math.e)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, value, _cite = (s.strip() for s in line.split("|", 2))
            vals[name] = float(value)
    return vals


# --------------------------------------------------------------------------- inverse normal CDF
def test_ndtri_matches_two_libraries(orc):
    ps = np.concatenate([np.logspace(-300, -1, 400), np.linspace(0.001, 0.999, 999),
                         1 - np.logspace(-16, -1, 100)])
    nd = statistics.NormalDist()
    for p in ps:
        x = orc.ndtri(p)
        ref = scipy.special.ndtri(p)
        assert abs(x - ref) <= 2e-14 * max(1.0, abs(ref)), (p, x, ref)
        if 1e-300 < p < 1 - 1e-16:
            assert abs(x - nd.inv_cdf(p)) <= 1e-13 * max(1.0, abs(ref)), p


def test_normal_scores_symmetric_and_match_scipy(orc):
    for T in (2, 3, 10, 1000, 10001):
        for r in sorted({1, 2, T // 2, (T + 1) // 2, T - 1, T}):
            if r < 1:
                continue
            s = orc.normal_score(r, T)
            assert s == -orc.normal_score(T + 1 - r, T)
            ref = scipy.special.ndtri(r / (T + 1))
            assert abs(s - ref) <= 1e-13 * max(1.0, abs(ref))


# --------------------------------------------------------------------------- digamma and bias corrector
def test_digamma_closed_forms_and_scipy(orc):
    gamma = 0.57721566490153286061
    for n in range(1, 60):
        exact = -gamma + sum(1.0 / k for k in range(1, n))
        assert abs(orc.digamma(n) - exact) <= 1e-14 * max(1, abs(exact))
        half = -gamma - 2 * math.log(2) + sum(2.0 / (2 * k - 1) for k in range(1, n + 1))
        assert abs(orc.digamma(n + 0.5) - half) <= 1e-14 * max(1, abs(half))
    for x in np.linspace(0.05, 5000, 777):
        assert abs(orc.digamma(x) - scipy.special.digamma(x)) <= 2e-14 * max(1, abs(scipy.special.digamma(x)))


def test_bias_eta_matches_library_digamma(orc):
    for n in (1, 2, 5, 20):
        for T in (50, 1000, 10000):
            ref = 0.5 * (n * math.log(2.0 / (T - 1)) + sum(scipy.special.digamma((T - j) / 2.0) for j in range(1, n + 1)))
            assert abs(orc.bias_eta(n, T) - ref) <= 1e-12 * max(1, abs(ref))
    # large T: E[log det S] -> log det Sigma, so eta -> 0
    assert abs(orc.bias_eta(3, 10 ** 8)) < 1e-6


# --------------------------------------------------------------------------- linear algebra
def _exact_det(M):
    """Determinant by fraction-exact Gaussian elimination."""
    A = [[Fraction(int(v)) for v in row] for row in M]
    n, det = len(A), Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if A[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            A[c], A[p] = A[p], A[c]
            det = -det
        det *= A[c][c]
        for r in range(c + 1, n):
            m = A[r][c] / A[c][c]
            for j in range(c, n):
                A[r][j] -= m * A[c][j]
    return det


def test_lu_logdet_exact_rationals(orc):
    rng = np.random.default_rng(11)
    for n in range(1, 8):
        for _ in range(20):
            M = rng.integers(-5, 6, (n, n))
            d = _exact_det(M)
            sign, ld = orc.lu_logdet(M.astype(float))
            if d == 0:
                assert sign == 0 or ld < -25
                continue
            assert sign == (1 if d > 0 else -1)
            assert abs(ld - math.log(abs(d))) < 1e-12 * max(1.0, abs(math.log(abs(d))))


def test_lu_logdet_vs_numpy_and_inverse(orc):
    rng = np.random.default_rng(12)
    for n in (1, 3, 10, 30):
        A = synth.random_spd(rng, n, cond=1e4)
        sign, ld = orc.lu_logdet(A)
        s2, ld2 = np.linalg.slogdet(A)
        assert sign == 1 and s2 == 1 and abs(ld - ld2) < 1e-10
        assert np.allclose(orc.inverse(A), np.linalg.inv(A), rtol=1e-9, atol=1e-12)
    assert orc.lu_logdet(np.zeros((0, 0)))[1] == 0.0


def test_is_pd_matches_eigenvalues(orc):
    rng = np.random.default_rng(13)
    for _ in range(200):
        n = int(rng.integers(1, 7))
        M = rng.standard_normal((n, n))
        A = M + M.T + rng.uniform(-2, 4) * np.eye(n)
        ev = np.linalg.eigvalsh(A)
        if abs(ev).min() < 1e-9:
            continue
        assert orc.is_pd(A) == bool(ev.min() > 0)


# --------------------------------------------------------------------------- copula and covariance
def test_copula_matches_library_ranks_and_quantiles(orc):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((257, 6)) * rng.uniform(0.1, 10, 6)
    Z = orc.copula(X)
    for c in range(6):
        r = scipy.stats.rankdata(X[:, c], method="ordinal")
        assert np.allclose(Z[:, c], scipy.special.ndtri(r / 258.0), rtol=1e-13, atol=1e-15)


def test_copula_invariant_to_monotone_transforms(orc):
    X = synth.planted_10(T=500)
    Z = orc.copula(X)
    assert np.array_equal(Z, orc.copula(np.exp(X)))
    assert np.array_equal(Z, orc.copula(X ** 3 - 7.0))
    assert not np.array_equal(Z, orc.copula(-X))


def test_copula_ties_ordinal_by_sample_index(orc):
    X = np.array([[1.0], [0.0], [1.0], [-0.0], [1.0], [2.0]])
    Z = orc.copula(X)
    # values: 1, 0, 1, -0 (== 0), 1, 2 -> ranks 3, 1, 4, 2, 5, 6
    ranks = [3, 1, 4, 2, 5, 6]
    assert np.allclose(Z[:, 0], scipy.special.ndtri(np.array(ranks) / 7.0), rtol=1e-13)
    with pytest.raises(ValueError):
        orc.copula(np.array([[1.0], [np.nan], [0.0]]))


def test_copula_diagonal_and_zero_mean(orc):
    for T in (1000, 1200, 10000):
        rng = np.random.default_rng(T)
        X = rng.standard_normal((T, 3))
        S = orc.covariance(orc.copula(X))
        v = float(np.sum(scipy.special.ndtri(np.arange(1, T + 1) / (T + 1.0)) ** 2) / (T - 1))
        assert np.allclose(np.diag(S), v, rtol=1e-12)
        assert abs(orc.copula(X).sum(axis=0)).max() < 1e-10


def test_covariance_matches_numpy(orc):
    rng = np.random.default_rng(6)
    Z = rng.standard_normal((300, 7)) + 3.0
    assert np.allclose(orc.covariance(Z), np.cov(Z, rowvar=False), rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------- enumeration
def _comb_count(n):
    return 2 ** n - 1 - n - n * (n - 1) // 2


def test_enumeration_brute_force(orc):
    for N in (1, 5, 10):
        for kmin, kmax in ((0, N), (3, N), (2, 3)):
            idx = orc.enumerate_nplets(N, kmin, kmax)
            ref = [c for k in range(kmin, kmax + 1) for c in itertools.combinations(range(N), k)]
            assert len(idx) == len(ref)
            for row, c in zip(idx, ref):
                assert tuple(int(v) for v in row[: len(c)]) == c
                assert all(v == -1 for v in row[len(c):])


def test_enumeration_n20_full(orc):
    idx = orc.enumerate_nplets(20, 3, 20)
    assert len(idx) == _comb_count(20) == 1048365
    k = (idx >= 0).sum(axis=1)
    assert np.all(np.diff(k) >= 0)
    ref = np.full((len(idx), 20), -1, dtype=np.int32)
    o = 0
    for kk in range(3, 21):
        combs = np.array(list(itertools.combinations(range(20), kk)), dtype=np.int32)
        ref[o:o + len(combs), :kk] = combs
        o += len(combs)
    assert np.array_equal(idx, ref)


def test_counts_eq_comb_and_paper(orc):
    g = _golden()
    assert orc.count_nplets(10, 3, 10) == _comb_count(10) == 968
    assert orc.count_nplets(20, 3, 20) == 1048365
    assert _comb_count(30) == 1073741358
    assert sum(math.comb(30, k) for k in range(3, 31)) == _comb_count(30)
    # Introduction: about 2^30 interactions for 30 elements
    assert abs(_comb_count(30) - g["nplets_n30_approx"]) / g["nplets_n30_approx"] < 1e-6
    assert g["nplets_formula_offset"] == 1


# --------------------------------------------------------------------------- Gaussian entropy and measures
def test_printed_normal_entropy_and_padding_identity(orc):
    g = _golden()
    assert abs(HALF_LOG_2PIE - g["normal_entropy_unit_variance"]) < 5e-5
    _, H1, _ = orc.measures(np.eye(1), [0])
    assert abs(H1 - HALF_LOG_2PIE) < 1e-15
    # padded batches: H(Sigma^k) = H(Sigma^k (+) I^{n-k}) - (n-k) * H(N(0,1))
    rng = np.random.default_rng(7)
    A = synth.random_spd(rng, 5, 50.0)
    padded = synth.block_diag(A, np.eye(4))
    _, Hk, _ = orc.measures(A, range(5))
    _, Hn, _ = orc.measures(padded, range(9))
    assert abs(Hk - (Hn - 4 * HALF_LOG_2PIE)) < 1e-12
    # padding leaves TC, DTC and S unchanged and adds no O-information
    out_k, _, _ = orc.measures(A, range(5))
    out_n, _, _ = orc.measures(padded, range(9))
    assert np.allclose(out_k, out_n, atol=1e-12)


def test_entropy_closed_form_diagonal(orc):
    sig2 = np.array([0.3, 1.0, 2.5, 7.0])
    out, H, _ = orc.measures(np.diag(sig2), range(4))
    assert abs(H - sum(0.5 * math.log(2 * math.pi * math.e * s) for s in sig2)) < 1e-13
    assert np.all(np.abs(out) < 1e-14)
    # the literal entropy form cancels the 1/2 log(2 pi e) terms only up to rounding
    out, _, _ = orc.measures(np.eye(6), range(6))
    assert np.all(np.abs(out) < 1e-13)


def test_pairs_have_zero_o_information(orc):
    for r in (-0.9, -0.3, 0.0, 0.6, 0.99):
        S = np.array([[2.0, r * math.sqrt(2 * 3)], [r * math.sqrt(2 * 3), 3.0]])
        out, _, _ = orc.measures(S, [0, 1])
        mi = -0.5 * math.log(1 - r * r)
        assert abs(out[0] - mi) < 1e-13 and abs(out[1] - mi) < 1e-13
        assert abs(out[2]) < 1e-13 and abs(out[3] - 2 * mi) < 1e-13
    out, _, _ = orc.measures(np.array([[1.0, 0.6], [0.6, 1.0]]), [0, 1])
    assert abs(out[0] - 0.223143551314) < 1e-12


def test_triplets_equal_co_information(orc):
    rng = np.random.default_rng(8)
    for _ in range(50):
        A = synth.random_spd(rng, 3, 30.0)
        d = np.sqrt(np.diag(A))
        R = A / np.outer(d, d)
        co = 0.5 * (math.log(np.linalg.det(R)) - sum(math.log(1 - R[i, j] ** 2) for i, j in ((0, 1), (0, 2), (1, 2))))
        out, _, _ = orc.measures(A, [0, 1, 2])
        assert abs(out[2] - co) < 1e-12
    out, _, _ = orc.measures(np.array([[2.0, 1, 1], [1, 2, 1], [1, 1, 2]]), [0, 1, 2])
    assert abs(out[2] - 0.5 * (math.log(0.5) - 3 * math.log(0.75))) < 1e-13
    assert abs(out[2] - 0.084949518398) < 1e-11 and abs(out[3] - 0.608197662162) < 1e-11


def _s_closed(n, c, m=None):
    """S-system (n X's + Y): TC, DTC of the sub-system of m X's plus Y (m = n: whole system)."""
    m = n if m is None else m
    sig = (n - m) * c * c + 1.0
    tc = 0.5 * (math.log(n * c * c + 1) - math.log(sig))
    dtc = 0.5 * m * math.log(1 + c * c / sig)
    return tc, dtc


@pytest.mark.parametrize("n,c", [(2, 1.0), (5, 0.5), (19, 0.5), (19, 1.0), (20, 1.0), (3, 3.0)])
def test_pgm_closed_forms(orc, n, c):
    tc, dtc = _s_closed(n, c)
    out, H, _ = orc.measures(synth.s_system(n, c), range(n + 1))
    assert np.allclose(out, [tc, dtc, tc - dtc, tc + dtc], atol=1e-11, rtol=1e-11)
    # det Sigma_S = 1, so H is (n+1) times the unit-normal entropy
    assert abs(H - (n + 1) * HALF_LOG_2PIE) < 1e-11
    # R-system: TC and DTC swap, Omega changes sign
    out_r, H_r, _ = orc.measures(synth.r_system(n, c), range(n + 1))
    assert np.allclose(out_r, [dtc, tc, dtc - tc, tc + dtc], atol=1e-11, rtol=1e-11)
    assert abs(H_r - (n + 1) * HALF_LOG_2PIE) < 1e-11
    assert out[2] < 0 < out_r[2]        # synergy-dominated vs redundancy-dominated
    # sub-systems: m X's with Y (S-system) and k X's without Y (R-system)
    for m in range(1, n + 1):
        tcm, dtcm = _s_closed(n, c, m)
        o, _, _ = orc.measures(synth.s_system(n, c), list(range(m)) + [n])
        assert np.allclose(o[:2], [tcm, dtcm], atol=1e-11, rtol=1e-11)
    for k in range(2, n + 1):
        omk = 0.5 * (k * math.log(1 + c * c) + (k - 2) * math.log(1 + k * c * c) - k * math.log(1 + (k - 1) * c * c))
        o, _, _ = orc.measures(synth.r_system(n, c), range(k))
        assert abs(o[2] - omk) < 1e-11


def test_pgm_printed_values(orc):
    for (n, c, om) in ((2, 1.0, -0.1438410362), (19, 0.5, -1.2452638101), (19, 1.0, -5.0870320785),
                       (20, 1.0, -5.4092105867)):
        out, _, _ = orc.measures(synth.s_system(n, c), range(n + 1))
        assert abs(out[2] - om) < 1e-9


def test_additivity_over_independent_blocks(orc):
    rng = np.random.default_rng(9)
    A = synth.random_spd(rng, 4, 20.0)
    B = synth.random_spd(rng, 5, 20.0)
    AB = synth.block_diag(A, B)
    oa, _, _ = orc.measures(A, range(4))
    ob, _, _ = orc.measures(B, range(5))
    oab, _, _ = orc.measures(AB, range(9))
    assert np.allclose(oab, oa + ob, atol=1e-11)
    # the 100-variable concatenated system: the four R/S blocks cancel pairwise
    C = synth.concatenated_100()
    out, _, _ = orc.measures(C, range(100))
    assert abs(out[2]) < 1e-8


def test_invariances(orc):
    rng = np.random.default_rng(10)
    A = synth.random_spd(rng, 8, 100.0)
    D = np.diag(rng.uniform(0.1, 10.0, 8))
    o1, H1, _ = orc.measures(A, [0, 2, 3, 5, 7])
    o2, H2, _ = orc.measures(D @ A @ D, [0, 2, 3, 5, 7])
    o3, _, _ = orc.measures(A, [7, 3, 0, 5, 2])
    assert np.allclose(o1, o2, atol=1e-12) and np.allclose(o1, o3, atol=1e-12)
    assert abs((H2 - H1) - sum(math.log(D[i, i]) for i in (0, 2, 3, 5, 7))) < 1e-12
    assert o1[0] >= 0 and o1[1] >= 0


def test_not_pd_gives_nan_and_flag(orc):
    S = np.array([[1.0, 1.5, 0.0], [1.5, 1.0, 0.0], [0.0, 0.0, 1.0]])
    out, H, flag = orc.measures(S, [0, 1, 2])
    assert flag == orc.FLAG_NOT_PD and np.all(np.isnan(out)) and math.isnan(H)
    out, _, flag = orc.measures(S, [0, 2])
    assert flag == 0 and np.all(np.isfinite(out))


def test_bias_offsets(orc):
    """The corrected measures differ from the plain ones by per-(k, T) constants."""
    rng = np.random.default_rng(14)
    A = synth.random_spd(rng, 6, 30.0)
    T = 1000
    psi = lambda j: scipy.special.digamma((T - j) / 2.0)
    for k in (1, 2, 3, 6):
        o0, H0, _ = orc.measures(A, range(k))
        o1, H1, _ = orc.measures(A, range(k), bias=True, T=T)
        P = lambda m: sum(psi(j) for j in range(1, m + 1))
        dtc_off = 0.5 * (P(k) - k * psi(1))
        ddtc_off = 0.5 * ((k - 1) * psi(k) - P(k - 1))
        assert abs((o1[0] - o0[0]) - dtc_off) < 1e-10
        assert abs((o1[1] - o0[1]) - ddtc_off) < 1e-10
        assert abs((H0 - H1) - orc.bias_eta(k, T)) < 1e-12


# --------------------------------------------------------------------------- gradient
def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(15)
    N = 7
    S = synth.random_spd(rng, N, 20.0)
    idx = orc.pad_list([(0, 1, 2), (1, 3, 4, 6), (0, 2, 3, 4, 5, 6), (2, 5)], kmax=6)
    w = rng.standard_normal((4, len(idx)))
    G = orc.grad_list(S, idx, w)
    assert np.allclose(G, G.T, atol=1e-12)

    def loss(M):
        out, _, _ = orc.eval_list(M, idx)
        return float((w * out).sum())

    h = 1e-6
    FD = np.zeros_like(S)
    for a in range(N):
        for b in range(a, N):
            E = np.zeros_like(S)
            E[a, b] = E[b, a] = h
            d = (loss(S + E) - loss(S - E)) / (2 * h)
            FD[a, b] = FD[b, a] = d / (1.0 if a == b else 2.0)
    err = np.linalg.norm(G - FD) / np.linalg.norm(FD)
    assert err < 1e-6, err


def test_gradient_fd_on_latent100_nplets(orc):
    """The first 100 n-plets of the N=100 differentiation workload (orders 8..20, planted groups of
    four): the oracle's explicit-inverse gradient of a random combination of the four measures
    against central differences (h = 1e-6) of the literal measures, entry by entry.  The bound,
    1e-6 of the n-plet's largest gradient entry, is 16x the largest discrepancy observed."""
    from _checks import fd_nplet_grad
    X, idx = synth.latent_100()
    S = orc.gc_covariance(X)
    W = np.random.default_rng(40).uniform(-1.0, 1.0, (4, 100))
    worst = 0.0
    for b in range(100):
        r, G_fd = fd_nplet_grad(orc, S, idx[b], W[:, b])
        G = orc.grad_list(S, idx[b:b + 1], W[:, b:b + 1])
        # the gradient lives on the n-plet's block only
        mask = np.zeros(S.shape, dtype=bool)
        mask[np.ix_(r, r)] = True
        assert np.all(G[~mask] == 0.0)
        scale = max(1.0, np.abs(G_fd).max())
        err = np.abs(G[np.ix_(r, r)] - G_fd).max() / scale
        worst = max(worst, err)
    assert worst < 1e-6, worst


# --------------------------------------------------------------------------- planted data
def test_planted_10_population_values(orc):
    c = 1.0 / 0.3
    red = 0.5 * (3 * math.log(1 + c * c) + math.log(1 + 3 * c * c) - 3 * math.log(1 + 2 * c * c))
    syn = 0.5 * (math.log(1 + 2 * c * c) - 2 * math.log(1 + c * c))
    assert abs(red - 0.7915787952) < 1e-9 and abs(syn + 0.9215684676) < 1e-9
    S = orc.gc_covariance(synth.planted_10())
    o_red, _, _ = orc.measures(S, [0, 1, 2])
    o_syn, _, _ = orc.measures(S, [3, 4, 5])
    o_ind, _, _ = orc.measures(S, [6, 7, 8])
    assert abs(o_red[2] - red) < 0.1 and o_red[2] > 0
    assert abs(o_syn[2] - syn) < 0.1 and o_syn[2] < 0
    assert abs(o_ind[2]) < 0.02
    # library cross-check of the whole chain (rankdata + ndtri + numpy cov + slogdet)
    X = synth.planted_10()
    Zl = scipy.special.ndtri(np.apply_along_axis(lambda v: scipy.stats.rankdata(v, method="ordinal"), 0, X) / 1001.0)
    Sl = np.cov(Zl, rowvar=False)
    assert np.allclose(S, Sl, rtol=1e-12, atol=1e-14)

    def om_lib(idx):
        sub = Sl[np.ix_(idx, idx)]
        ld = np.linalg.slogdet(sub)[1]
        ai = np.diag(np.linalg.inv(sub))
        return 0.5 * (np.log(np.diag(sub)).sum() - 2 * ld - np.log(ai).sum())

    for idx in ([0, 1, 2], [3, 4, 5], [0, 3, 5, 7], list(range(10))):
        out, _, _ = orc.measures(S, idx)
        assert abs(out[2] - om_lib(idx)) < 1e-10


def test_eval_list_matches_single_calls(orc):
    S = orc.gc_covariance(synth.planted_10())
    out, H, flags = orc.eval_range(S, 3, 10)
    assert out.shape == (4, 968)
    idx = orc.enumerate_nplets(10, 3, 10)
    for b in (0, 1, 119, 500, 967):
        k = int((idx[b] >= 0).sum())
        o, h, f = orc.measures(S, idx[b, :k])
        assert np.array_equal(o, out[:, b]) and h == H[b] and f == flags[b]
    assert np.allclose(out[3], out[0] + out[1], atol=1e-12)
    assert np.allclose(out[2], out[0] - out[1], atol=1e-12)
    assert np.all(out[0] >= -1e-12) and np.all(out[1] >= -1e-12)


def test_reducers_reference():
    import oracle
    v = np.array([0.5, -1.0, 0.5, 2.0, np.nan, -1.0, 0.0])
    k = np.array([3, 3, 3, 3, 3, 4, 4])
    g = np.arange(7)
    r = oracle.topk_per_order(v, k, g, 2)
    assert r[3][0] == [(2.0, 3), (0.5, 0)] and r[3][1] == [(-1.0, 1), (0.5, 0)]
    h = oracle.histogram(np.array([-2.0, 0.0, 0.99, 1.0, 3.0]), 0.0, 1.0, 4)
    assert list(h) == [1, 0, 0, 2, 1, 1]
