"""Pins of the FOURIER split (the paper's approximate median) in the oracle.

The paper's count approximation (Lemma 3.1, §3.1; Eq. (1) and Eq. (2), §3.2)
is evaluated here literally, term by term, with mpmath from the coefficient
formulas c_j, g_j, and compared with the oracle's moment form.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle

mp.mp.dps = 30


def c_fn(j, x):
    """c_j(x) of Lemma 3.1: c_0 = 1, c_{2k-1} = cos((2k-1)x), c_{2k} = sin((2k-1)x)."""
    if j == 0:
        return mp.mpf(1)
    k = (j + 1) // 2
    return mp.cos((2 * k - 1) * x) if j % 2 == 1 else mp.sin((2 * k - 1) * x)


def g_fn(j, a, b, ia=None, ib=None):
    """g_j(a, b) of Lemma 3.1; ia / ib are the boundary flags 1(a > 0), 1(b < 1)
    (given explicitly when the interval is not inside (0, 1))."""
    ia = (1 if a > 0 else 0) if ia is None else ia
    ib = (1 if b < 1 else 0) if ib is None else ib
    if j == 0:
        return 1 - mp.mpf(ia + ib) / 2
    k = (j + 1) // 2
    w = 2 / (mp.pi * (2 * k - 1))
    if j % 2 == 1:
        return w * (ib * mp.sin((2 * k - 1) * b) - ia * mp.sin((2 * k - 1) * a))
    return w * (ia * mp.cos((2 * k - 1) * a) - ib * mp.cos((2 * k - 1) * b))


def one_J(x, a, b, J, ia=None, ib=None):
    """Partial sum 1_J(x, a, b) = sum_{j=0}^{2J} c_j(x) g_j(a, b) (§3.1)."""
    return mp.fsum(c_fn(j, x) * g_fn(j, a, b, ia, ib) for j in range(2 * J + 1))


@pytest.mark.parametrize("a,b", [(0.2, 0.7), (0.0, 0.4), (0.35, 1.0), (0.0, 1.0)])
def test_lemma_expansion_converges_to_indicator(a, b):
    # Lemma 3.1 with Lemma 3.2(A): away from the ends the partial sums
    # approach 1(a < x < b).
    for x in [0.05, 0.3, 0.5, 0.66, 0.9]:
        if min(abs(x - a), abs(x - b)) < 0.05:
            continue
        target = 1.0 if a < x < b else 0.0
        err = abs(float(one_J(mp.mpf(x), mp.mpf(a), mp.mpf(b), 400)) - target)
        assert err < 0.02, (x, a, b, err)


def _scaled_keys(x):
    keys = oracle.keys_of_floats(np.asarray(x, dtype=np.float32))
    lo, hi = int(keys.min()), int(keys.max())
    e = oracle.fourier_exponent(lo, hi)
    return keys, lo, hi, e


def _mapped(x, e):
    """The cell map u = (x - min) * 2^-e of every key (exact in double)."""
    xmin = float(np.float32(x.min()))
    return [float(np.float32((float(xi) - xmin) * 2.0 ** -e)) for xi in x]


def test_cell_map_lands_in_unit_interval():
    """§2 takes the data to lie in (0, 1): the smallest key maps to 0, the
    largest into [1/2, 1), for spreads from subnormal to near the fp32 limit."""
    rng = np.random.default_rng(2)
    for scale in [1e-42, 1e-30, 1e-3, 1.0, 7.0, 1e20, 1e38]:
        x = (rng.standard_normal(50) * scale).astype(np.float32)
        keys, lo, hi, e = _scaled_keys(x)
        if lo == hi:
            continue
        u = _mapped(x, e)
        assert min(u) == 0.0 and 0.5 <= max(u) < 1.0, (scale, e, max(u))


def test_moment_form_equals_paper_equal_count_difference():
    """(4/pi) * F(v) == sum_i [1_J(u_i, 0, v) - 1_J(u_i, v, 1)] (Eq. (1), (2)):
    the left child is the interval (0, v), the right child (v, 1), with the
    boundary flags of Lemma 3.1 as the paper defines them for (a, b) inside
    (0, 1)."""
    rng = np.random.default_rng(3)
    J = 7
    x = rng.uniform(-2.0, 3.0, size=40).astype(np.float32)
    keys, lo, hi, e = _scaled_keys(x)
    Cc, Cs = oracle.fourier_map(keys, lo, e, J)
    u = _mapped(x, e)
    assert 0.5 <= max(u) < 1.0
    for v in [0.05, 0.2, 0.37, 0.5, 0.68, 0.9]:
        lhs = mp.fsum(one_J(mp.mpf(ui), 0, mp.mpf(v), J) for ui in u)
        rhs = mp.fsum(one_J(mp.mpf(ui), mp.mpf(v), 1, J) for ui in u)
        paper = float(lhs - rhs)
        ours = 4.0 / math.pi * oracle.fourier_F(Cc, Cs, v)
        assert abs(paper - ours) < 1e-4 * len(x), (v, paper, ours)


def test_F_is_sum_of_odd_harmonic_kernels():
    """F(v) == sum_i S_J(v - u_i), S_J(z) = sum_j sin((2j-1) z) / (2j-1)."""
    rng = np.random.default_rng(4)
    J = 15
    x = rng.standard_normal(300).astype(np.float32)
    keys, lo, hi, e = _scaled_keys(x)
    Cc, Cs = oracle.fourier_map(keys, lo, e, J)
    u = np.array(_mapped(x, e), dtype=np.longdouble)
    for v in np.linspace(0.0, 1.0, 21):
        z = np.longdouble(v) - u
        direct = sum(np.sin((2 * j - 1) * z) / (2 * j - 1) for j in range(1, J + 1)).sum()
        assert abs(float(direct) - oracle.fourier_F(Cc, Cs, float(v))) < 2e-5 * len(x)


def test_bracket_and_bisection_invariant():
    rng = np.random.default_rng(8)
    for trial in range(40):
        n = int(rng.integers(2, 200))
        x = (rng.standard_normal(n) * 10 ** rng.uniform(-3, 3)).astype(np.float32)
        keys, lo, hi, e = _scaled_keys(x)
        if lo == hi:
            continue
        Cc, Cs = oracle.fourier_map(keys, lo, e, 15)
        assert oracle.fourier_F(Cc, Cs, 0.0) < 0.0
        xmin = float(np.float32(x.min()))

        def v_of(k):
            return (float(np.uint32(oracle.bits_of_key(k)).view(np.float32)) - xmin) * 2.0 ** -e

        vmax = v_of(hi)
        assert 0.5 <= vmax < 1.0
        assert oracle.fourier_F(Cc, Cs, vmax) > 0.0
        m = oracle.fourier_solve(Cc, Cs, lo, hi, e)
        assert lo < m <= hi
        assert oracle.fourier_F(Cc, Cs, v_of(m - 1)) < 0.0 or m - 1 == lo
        assert oracle.fourier_F(Cc, Cs, v_of(m)) >= 0.0 or m == hi


def test_symmetric_three_points_split_at_middle():
    # u = {0, 0.3, 0.6}: F is odd about 0.3, so the root is the middle point.
    x = np.array([0.1, 0.25, 0.4], dtype=np.float32)
    keys, lo, hi, e = _scaled_keys(x)
    assert e == -1
    u = _mapped(x, e)
    assert u[0] == 0.0 and abs(u[1] - 0.3) < 1e-6 and abs(u[2] - 0.6) < 1e-6
    Cc, Cs = oracle.fourier_map(keys, lo, e, 15)
    m = oracle.fourier_solve(Cc, Cs, lo, hi, e)
    val = float(np.uint32(oracle.bits_of_key(m)).view(np.float32))
    assert abs(val - 0.25) < 1e-5


def test_statistics_additive_over_any_partition():
    """C_j(X) = sum_r C_j(X_r) (§3.2) holds exactly for the quantized sums."""
    rng = np.random.default_rng(12)
    x = rng.standard_normal(1000).astype(np.float32)
    keys, lo, hi, e = _scaled_keys(x)
    Cc, Cs = oracle.fourier_map(keys, lo, e, 15)
    cuts = np.sort(rng.choice(np.arange(1, 1000), size=9, replace=False))
    parts = np.split(rng.permutation(keys), cuts)
    sc = sum(oracle.fourier_map(p, lo, e, 15)[0] for p in parts)
    ss = sum(oracle.fourier_map(p, lo, e, 15)[1] for p in parts)
    assert (sc == Cc).all() and (ss == Cs).all()


@pytest.mark.parametrize("J,tol", [(15, 0.004), (60, 0.002)])
def test_split_balances_as_J_grows(J, tol):
    # Thm 3.6/3.7 (§3.2): the children approach half the parent each.
    from paper_2201_08288_amd import synth
    x = synth.uniform24(20000, 1, seed=77)
    ok, dim, split, cand = oracle.cell_split(x, np.arange(20000), split_rule=oracle.SPLIT_FOURIER,
                                             fourier_J=J, leaf_size=1, num_subsets=1)
    keys = oracle.keys_of_floats(x[0])
    frac = float((keys <= split).mean())
    assert abs(frac - 0.5) < tol, frac


def test_fourier_split_invariant_to_subsets():
    from paper_2201_08288_amd import synth
    x = synth.gmm(3000, 2, seed=5)
    pool = synth.dirichlet_pool(32, 8, seed=1)
    res = set()
    for S, pl in [(1, None), (7, None), (64, None), (8, pool)]:
        res.add(oracle.cell_split(x, np.arange(3000), split_rule=oracle.SPLIT_FOURIER, fourier_J=15,
                                  num_subsets=S, pool=pl, leaf_size=1)[1:])
    assert len(res) == 1
