"""Pins of the oracle's FSR (Sec. 2.1 / 3.2): closed forms for inputs made of
a single basis function, the exact per-iteration energy decrement of the
greedy update, agreement of the two independently written forms (re-FFT of
the spatial residual vs in-place spectral update), exact scale and
translation equivariance, the overwrite rule and garbage invariance."""
import numpy as np
import pytest

import oracle as O
from oracle import fsr as F
import synth

M = 32


def quarter_weights(rng, rho=0.7):
    m = synth.fixed_mask(M, M, rng).astype(np.float64)
    return m * O.rho_table(rho, M)


@pytest.mark.parametrize("K", [1, 7, 100])
def test_constant_block_closed_form(K):
    """s = c * phi_0: DC is chosen every iteration (|W_k| < W_0 for k != 0
    off a lattice coset), c_0 = c (1 - (1-gamma)^K)."""
    rng = np.random.default_rng(K)
    w = quarter_weights(rng)[None]
    s = np.full((1, M, M), 100.0)
    c, picks, _, _ = F.fsr_spatial(s, w, 0.5, K)
    expect = 100.0 * (1 - 0.5 ** K)
    assert abs(c[0, 0, 0] - expect) < 1e-9
    out = F.synthesize(c, 4)
    assert np.allclose(out, expect, atol=1e-9, rtol=0)


@pytest.mark.parametrize("b", [(3, 5), (5, 3), (16, 0), (31, 1)])
def test_single_complex_bin_closed_form(b):
    """s = z * phi_b (complex): coefficient z (1 - (1-gamma)^K) at bin b and
    the model is that multiple of phi_b.  Catches a swapped index, a wrong
    exponent sign, a missing gamma or W0."""
    rng = np.random.default_rng(sum(b))
    w = quarter_weights(rng)[None]
    m = np.arange(M)
    z = 3.0 - 7.0j
    phi = np.exp(2j * np.pi * (b[0] * m[:, None] + b[1] * m[None, :]) / M)
    for K, g in ((10, 0.5), (40, 0.3)):
        c, picks, _, _ = F.fsr_spatial((z * phi)[None], w, g, K)
        assert (picks[0, :5] == b[0] * M + b[1]).all()
        expect = z * (1 - (1 - g) ** K)
        assert abs(c[0, b[0], b[1]] - expect) < 1e-12 * abs(z)
        g_model = (M * M) * np.fft.ifft2(c[0])
        assert np.allclose(g_model, expect * phi, atol=1e-10)


def test_energy_decrement_identity():
    """E' = E - gamma (2 - gamma) |R_b|^2 / W0 with E = sum w |r|^2:
    exact for this update, so it is checked to rounding each iteration."""
    rng = np.random.default_rng(5)
    nb = 6
    w = np.stack([quarter_weights(rng) for _ in range(nb)])
    s = rng.uniform(0, 255, (nb, M, M))
    for g in (0.5, 1.0, 1.7):
        c, picks, _, (energies, chosen) = F.fsr_spatial(s, w, g, 60)
        W0 = w.sum(axis=(1, 2))
        E_prev = (w * s ** 2).sum(axis=(1, 2))
        for it in range(60):
            pred = E_prev - g * (2 - g) * chosen[it] / W0
            assert np.allclose(energies[it], pred, rtol=1e-9, atol=1e-9 * E_prev.max())
            assert (energies[it] <= E_prev * (1 + 1e-12)).all()     # monotone
            E_prev = energies[it]


def test_spatial_and_spectral_forms_agree():
    rng = np.random.default_rng(6)
    nb = 8
    w = np.stack([quarter_weights(rng) for _ in range(nb)])
    s = rng.uniform(0, 255, (nb, M, M)) * (w > 0)
    c1, p1, _, _ = F.fsr_spatial(s, w, 0.5, 50)
    c2, p2 = F.fsr_spectral(s, w, 0.5, 50)
    # picks agree up to the conjugate-partner tie of real data: where the two
    # forms round a tie differently they follow conjugate trajectories
    conj = lambda p: ((-(p // M)) % M) * M + (-(p % M)) % M
    assert ((p1 == p2) | (p1 == conj(p2))).all()
    o1, o2 = F.synthesize(c1, 4), F.synthesize(c2, 4)
    assert np.max(np.abs(o1 - o2)) < 1e-9


def _frame(seed, H=48, W=56, kind="dynamic"):
    rng = np.random.default_rng(seed)
    f = synth.video_regions(1, H, W, rng, grid=2, vmax=1)[0]
    m = synth.mask_sequence(kind, 1, H, W, rng)[0]
    return f, m, synth.measured(f, m)


def test_scale_equivariance_exact():
    f, m, meas = _frame(1)
    v = meas.astype(np.float64)
    o1, _ = O.fsr_frame(v, m, K=30)
    o2, _ = O.fsr_frame(2.0 * v, m, K=30)
    assert (o2 == 2.0 * o1).all()       # power-of-two scaling commutes with rounding
    o3, _ = O.fsr_frame(3.0 * v, m, K=30)
    assert np.max(np.abs(o3 - 3.0 * o1)) < 1e-9 * 255


def test_translation_by_block_multiples():
    """Shifting frame and mask by a multiple of the block size shifts the
    output of every block whose support lies inside both frames, bitwise."""
    f, m, meas = _frame(2, 64, 64)
    v = meas.astype(np.float64)
    o1, _ = O.fsr_frame(v, m, K=20)
    v2 = np.zeros_like(v)
    m2 = np.zeros_like(m)
    v2[4:, 8:] = v[:-4, :-8]
    m2[4:, 8:] = m[:-4, :-8]
    o2, _ = O.fsr_frame(v2, m2, K=20)
    # blocks with supports inside both: rows 32..44 of frame 2 map to 28..40 of frame 1
    assert (o2[32:36, 32:36] == o1[28:32, 24:28]).all()


def test_overwrite_and_garbage_invariance():
    f, m, meas = _frame(3)
    v = meas.astype(np.float64)
    cls = m.copy()
    o, _ = O.fsr_frame(v, cls, K=20)
    assert (o[m == 1] == v[m == 1]).all()
    vg = v.copy()
    vg[m == 0] = np.nan
    og, _ = O.fsr_frame(vg, cls, K=20)
    assert (og == o).all()
    # projected pixels: modelled but not overwritten by D-FSR, overwritten by R-FSR
    cls2 = cls.copy()
    rng = np.random.default_rng(0)
    proj = (m == 0) & (rng.random(m.shape) < 0.3)
    cls2[proj] = 2
    v2 = v.copy()
    v2[proj] = f[proj]
    od, _ = O.fsr_frame(v2, cls2, K=20, overwrite="dfsr")
    orr, _ = O.fsr_frame(v2, cls2, K=20, overwrite="rfsr")
    assert (orr[proj] == v2[proj]).all()
    assert not (od[proj] == v2[proj]).all()
    assert (od[m == 1] == v[m == 1]).all()
    # projected samples help: closer to the truth than without them
    assert np.abs(od - f)[m == 0].mean() < np.abs(o - f)[m == 0].mean()


def test_no_samples_gives_zero_model():
    v = np.zeros((8, 8))
    cls = np.zeros((8, 8), np.uint8)
    o, _ = O.fsr_frame(v, cls, K=5)
    assert (o == 0).all()


def test_near_tie_gap_conjugate_rule():
    """For real data the spectrum is Hermitian until a non-self-conjugate
    bin is chosen, so that choice ties with its conjugate partner; the gap
    measure must exclude the partner (else every block would look tied)."""
    rng = np.random.default_rng(8)
    w = quarter_weights(rng)[None]
    s = (rng.uniform(0, 255, (M, M)) * (w[0] > 0))[None]
    c, picks, gaps, (_, chosen) = F.fsr_spatial(s, w, 0.5, 30, track_gaps=True)
    first = next(i for i in range(30) if picks[0, i] != 0)
    b = picks[0, first]
    partner = ((-(b // M)) % M) * M + (-(b % M)) % M
    assert partner != b
    assert gaps[0] > 1e-6


# ------------------------------------------------- concealed weighting delta --
def _conc_case(seed, H=32, W=40):
    import synth
    rng = np.random.default_rng(seed)
    f, _ = synth.video_translate_edges(1, H, W, rng, n_edges=3)
    m = synth.fixed_mask(H, W, rng)
    cls = m.astype(np.uint8)
    # a few projected pixels as well
    proj = (m == 0) & (rng.random((H, W)) < 0.2)
    cls[proj] = 2
    return f[0].astype(np.float64), cls


def test_concealed_delta_zero_is_plain_fsr():
    v, cls = _conc_case(1)
    a, _ = O.fsr_frame_concealed(v, cls, 0.0, K=30)
    b, _ = O.fsr_frame(v, cls, K=30, track_gaps=False)
    assert np.array_equal(a, b)


def test_concealed_first_block_has_no_concealed_samples():
    v, cls = _conc_case(2)
    a, _ = O.fsr_frame_concealed(v, cls, 0.5, K=30)
    b, _ = O.fsr_frame(v, cls, K=30, track_gaps=False)
    assert np.array_equal(a[:4, :4], b[:4, :4])
    assert not np.allclose(a, b)


def test_concealed_equals_independent_block_with_explicit_concealed_class():
    """Block (i, j) of the sequential result equals an independent FSR of
    that block whose support marks every class-0 pixel of the raster-earlier
    blocks as a sample of weight delta carrying its reconstructed value."""
    from oracle.fsr import _gather, rho_table, fsr_spatial, synthesize, class_weight
    v, cls = _conc_case(3)
    delta = 0.4
    out, _ = O.fsr_frame_concealed(v, cls, delta, K=25)
    H, W = v.shape
    for bi, bj in [(0, 3), (2, 0), (3, 5), (7, 9)]:
        yy, xx = np.mgrid[0:H, 0:W]
        earlier = (yy // 4 < bi) | ((yy // 4 == bi) & (xx // 4 < bj))
        conc = earlier & (cls == 0)
        vv = np.where(cls > 0, v, 0.0)
        vv[conc] = out[conc]
        aa = class_weight(cls, 1.0)
        aa[conc] = delta
        s, aw = _gather(vv, aa, [(bi, bj)], 4, 32)
        c, _, _, _ = fsr_spatial(s, aw * rho_table(0.7)[None], 0.5, 25)
        o = synthesize(c, 4)[0]
        cb = cls[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4]
        o[cb == 1] = v[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4][cb == 1]
        assert np.allclose(o, out[4 * bi:4 * bi + 4, 4 * bj:4 * bj + 4], atol=1e-9), (bi, bj)


def test_concealed_given_own_output_is_identity():
    v, cls = _conc_case(4)
    a, ga = O.fsr_frame_concealed(v, cls, 0.5, K=20)
    b, gb = O.fsr_frame_concealed(v, cls, 0.5, K=20, given=a)
    assert np.array_equal(a, b) and np.array_equal(ga, gb)


# ----------------------------------------------------------- conjugate pairs --
def _uniform(M=32):
    return np.ones((1, M, M))


@pytest.mark.parametrize("b1,b2,phase", [(3, 5, 0.4), (0, 7, 1.1), (16, 3, -0.3), (9, 0, 2.0)])
def test_pairs_single_cosine_closed_form(b1, b2, phase):
    """Uniform weights make the basis orthogonal: the pair loop recovers a
    real cosine as A (1 - (1 - gamma)^K) cos(...), picking b every time."""
    M, A, g, K = 32, 37.0, 0.5, 7
    m = np.arange(M)
    s = A * np.cos(2 * np.pi * (b1 * m[:, None] + b2 * m[None, :]) / M + phase)[None]
    c, picks = O.fsr_pairs_spatial(s, _uniform(), g, K)
    model = (M * M * np.fft.ifft2(c[0]))
    assert np.abs(model.imag).max() < 1e-9
    assert np.allclose(model.real, s[0] * (1 - (1 - g) ** K), atol=1e-9)
    first = min(b1 * M + b2, ((-b1) % M) * M + ((-b2) % M))
    assert (picks[0] == first).all()


def test_pairs_self_conjugate_basis():
    M, A, g, K = 32, 20.0, 0.5, 5
    m = np.arange(M)
    s = (A * (-1.0) ** m[:, None] * np.ones((1, M)))[None]      # bin (16, 0)
    c, picks = O.fsr_pairs_spatial(s, _uniform(), g, K)
    assert (picks[0] == 16 * M).all()
    model = (M * M * np.fft.ifft2(c[0])).real
    assert np.allclose(model, s[0] * (1 - (1 - g) ** K), atol=1e-9)


def test_pairs_equal_two_complex_iterations_on_orthogonal_basis():
    """With orthogonal bases the complex loop alternates b, -b: 2K complex
    iterations give the model of K pair iterations."""
    M, g = 32, 0.5
    m = np.arange(M)
    s = (30 * np.cos(2 * np.pi * (4 * m[:, None] + 9 * m[None, :]) / M + 0.7)
         + 12 * np.cos(2 * np.pi * (11 * m[:, None] + 2 * m[None, :]) / M - 0.2))[None]
    cp, _ = O.fsr_pairs_spatial(s, _uniform(), g, 6)
    cc, _, _, _ = O.fsr_spatial(s, _uniform(), g, 12)
    assert np.allclose(cp, cc, atol=1e-9)


def test_pairs_spatial_and_spectral_forms_agree():
    rng = np.random.default_rng(5)
    M = 32
    s = rng.normal(100, 30, (6, M, M))
    w = (rng.random((6, M, M)) < 0.4) * O.rho_table(0.7)[None]
    ca, pa = O.fsr_pairs_spatial(s, w, 0.5, 30)
    cb, pb = O.fsr_pairs_spectral(s, w, 0.5, 30)
    # b and -b tie up to rounding and add the same real pair: compare modulo conjugation
    canon = lambda p: np.minimum(p, ((-(p // M)) % M) * M + ((-(p % M)) % M))
    assert (canon(pa) == canon(pb)).all()
    assert np.allclose(ca, cb, atol=1e-8 * np.abs(ca).max())
    model = np.fft.ifft2(ca, axes=(1, 2))
    assert np.abs(model.imag).max() < 1e-9 * np.abs(model.real).max()


# ------------------------------------------------------------- early stop --
def test_early_stop_zero_ratio_is_plain_loop():
    rng = np.random.default_rng(8)
    s = rng.normal(100, 30, (5, 32, 32))
    w = (rng.random((5, 32, 32)) < 0.3) * O.rho_table(0.7)[None]
    a = O.fsr_spatial(s, w, 0.5, 40)
    b = O.fsr_spatial(s, w, 0.5, 40, stop_ratio=0.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_early_stop_single_basis_iteration_count():
    """Uniform weights, one complex basis function: the chosen energy after i
    iterations is (1-gamma)^(2i) E0, so with ratio r the loop stops before
    the first i with (1-gamma)^(2i) < r."""
    M, g = 32, 0.5
    m = np.arange(M)
    s = 50 * np.exp(2j * np.pi * (3 * m[:, None] + 5 * m[None, :]) / M)[None]
    for r, n in ((0.5, 1), (0.2, 2), (0.01, 4), (1e-4, 7)):
        c, picks, _, _ = O.fsr_spatial(s, np.ones((1, M, M)), g, 20, stop_ratio=r)
        done = int((picks[0] >= 0).sum())
        assert done == n, (r, done)
        assert (picks[0, done:] == -1).all()
        assert np.isclose(np.abs(c[0, 3, 5]), 50 * (1 - (1 - g) ** n))


def test_early_stop_prefix_of_full_loop():
    rng = np.random.default_rng(9)
    s = rng.normal(100, 30, (6, 32, 32))
    w = (rng.random((6, 32, 32)) < 0.3) * O.rho_table(0.7)[None]
    full = O.fsr_spatial(s, w, 0.5, 60)[1]
    stop = O.fsr_spatial(s, w, 0.5, 60, stop_ratio=1e-3)[1]
    for i in range(6):
        n = int((stop[i] >= 0).sum())
        assert 1 <= n <= 60
        assert np.array_equal(stop[i, :n], full[i, :n])


# ------------------------------------------------- frequency-weighting prior --
def test_prior_table_closed_form():
    s = 0.8
    T = O.prior_table(s, 32)
    assert T[0, 0] == 1.0 and np.isclose(T[0, 1], s) and np.isclose(T[1, 1], s ** np.sqrt(2))
    assert np.isclose(T[16, 16], s ** np.sqrt(512)) and np.isclose(T[31, 30], s ** np.sqrt(5))
    k = np.arange(32)
    assert np.array_equal(T, T[(-k) % 32][:, (-k) % 32])      # even: conjugate bins weigh the same
    assert (O.prior_table(0.0, 32) == 1).all()


def test_prior_off_is_plain_loop():
    rng = np.random.default_rng(11)
    s = rng.normal(100, 30, (4, 32, 32))
    w = (rng.random((4, 32, 32)) < 0.3) * O.rho_table(0.7)[None]
    a = O.fsr_spatial(s, w, 0.5, 30)
    b = O.fsr_spatial(s, w, 0.5, 30, prior=O.prior_table(0.0, 32))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def _brute_prior_loop(s, w, prior, gamma, K):
    """Direct loops on one small support: residual DFT as explicit sums, the
    pick maximising prior * |R|^2 (first in row-major order), the usual
    update.  Returns the picks and the coefficients."""
    M = w.shape[0]
    r = s.astype(complex).copy()
    W0 = w.sum()
    c = np.zeros((M, M), complex)
    picks = []
    for _ in range(K):
        best, bk = -1.0, None
        for k1 in range(M):
            for k2 in range(M):
                R = 0j
                for m in range(M):
                    for n in range(M):
                        R += w[m, n] * r[m, n] * np.exp(-2j * np.pi * (k1 * m + k2 * n) / M)
                crit = prior[k1, k2] * abs(R) ** 2
                if crit > best:
                    best, bk, Rb = crit, (k1, k2), R
        d = gamma * Rb / W0
        c[bk] += d
        picks.append(bk[0] * M + bk[1])
        m = np.arange(M)
        r -= d * np.exp(2j * np.pi * (bk[0] * m[:, None] + bk[1] * m[None, :]) / M)
    return np.array(picks), c


def test_prior_against_brute_force_loops():
    rng = np.random.default_rng(12)
    M = 8
    s = rng.normal(0, 1, (M, M)) + 1j * rng.normal(0, 1, (M, M))
    w = rng.random((M, M)) * (rng.random((M, M)) < 0.6)
    prior = O.prior_table(0.7, M)
    picks, c = _brute_prior_loop(s, w, prior, 0.5, 5)
    co, po, _, _ = O.fsr_spatial(s[None], w[None], 0.5, 5, prior=prior)
    assert np.array_equal(po[0], picks)
    assert np.allclose(co[0], c, atol=1e-12 * np.abs(c).max())
    # the prior changes the picks here (without it the loop differs)
    assert not np.array_equal(O.fsr_spatial(s[None], w[None], 0.5, 5)[1][0], picks)


def test_prior_prefers_the_lower_frequency():
    """Two real cosines, the higher one with 1.1x the amplitude: the plain
    loop picks the higher first (energy ratio 1.21), the prior with sigma 0.9
    the lower (0.9 vs 1.21 * 0.9^5)."""
    M = 32
    m = np.arange(M)
    s = (np.cos(2 * np.pi * 1 * m / M)[None, :] + 1.1 * np.cos(2 * np.pi * 5 * m / M)[None, :]) * np.ones((M, 1))
    w = np.ones((1, M, M))
    first_plain = O.fsr_spatial(s[None], w, 0.5, 1)[1][0, 0] % M
    first_prior = O.fsr_spatial(s[None], w, 0.5, 1, prior=O.prior_table(0.9, M))[1][0, 0] % M
    assert first_plain in (5, M - 5) and first_prior in (1, M - 1)


def test_prior_and_stop_spatial_and_spectral_forms_agree():
    # complex samples: no conjugate-partner ties, so both forms pick the same bins
    rng = np.random.default_rng(13)
    s = rng.normal(100, 30, (5, 32, 32)) + 1j * rng.normal(0, 30, (5, 32, 32))
    w = (rng.random((5, 32, 32)) < 0.3) * O.rho_table(0.7)[None]
    prior = O.prior_table(0.85, 32)
    ca, pa, _, _ = O.fsr_spatial(s, w, 0.5, 40, prior=prior, stop_ratio=1e-3)
    cb, pb = O.fsr_spectral(s, w, 0.5, 40, prior=prior, stop_ratio=1e-3)
    assert np.array_equal(pa, pb)
    assert np.allclose(ca, cb, atol=1e-9 * np.abs(ca).max())
