"""Oracle (test infrastructure only): block-wise frequency selective
reconstruction (FSR), Sec. 2.1, with the recursive use of projected pixels
of Sec. 3.2 (D-FSR / R-FSR), float64.

The paper describes FSR only at the level of Sec. 2.1: the image is split
into blocks, each block is modelled in the Fourier domain (where the image is
assumed approximately sparse) using the samples of neighbouring blocks too,
and the model is finally overwritten with the available measurements
(Sec. 3.2).  Concealed weighting is set to zero (Sec. 4), so every block is
independent.  The FSR internals are the standard greedy (matching-pursuit
type) FSR of the literature the paper cites; the readings used here:

  * Block b = (bi, bj) covers rows [B*bi, B*bi+B) and columns
    [B*bj, B*bj+B); its support is the M x M window whose top-left corner is
    (B*bi - o, B*bj - o), o = (M - B) / 2, so the block sits in the middle.
  * Weights w[m,n] = a[m,n] * rho ** sqrt((m-c)^2 + (n-c)^2), c = (M-1)/2,
    with a = 1 for measured pixels, a = pi_w for projected pixels, 0 for
    unknown pixels and positions outside the frame.
  * Basis phi_k[m,n] = exp(2*pi*i*(k1*m + k2*n)/M), complex, M x M bins.
  * Greedy loop, K times, starting from the residual r = s and c = 0:
      R   = sum_{m} w[m] r[m] conj(phi_k[m])         (the weighted residual DFT)
      b   = first argmax_k |R_k|^2 in row-major order
      dlt = gamma * R_b / W0,  W0 = sum w           (orthogonality-deficiency
                                                     compensation gamma)
      c_b += dlt ;  r -= dlt * phi_b
  * Model g = sum_k c_k phi_k; the block output is Re g on the block pixels.
  * Overwrite: D-FSR writes the measured values over the model, R-FSR the
    measured and the projected values (Sec. 3.2).
  * W0 = 0 gives g = 0.
  * Options of the FSR literature that the paper's configuration does not
    use (both off by default):
      - frequency-weighting prior: the pick maximises prior_k |R_k|^2 with
        prior_k = sigma ** |k|, |k| the Euclidean distance of
        (min(k1, M-k1), min(k2, M-k2)) from DC (0 < sigma <= 1), favouring
        low frequencies; the update dlt is unchanged;
      - residual-energy early stop: a block stops before iteration i >= 1
        once its pick's criterion value (prior_b |R_b|^2, or |R_b|^2) is
        below stop_ratio times that of iteration 0; a stopped block picks
        -1 and changes nothing.

Two forms are given: `fsr_spatial` recomputes the weighted residual DFT from
the spatial residual every iteration (the plain form), `fsr_spectral`
updates the residual spectrum in place (R_k -= dlt * W_{k-b}, W = DFT(w)).
They must agree to rounding.
"""
from __future__ import annotations

import numpy as np


def rho_table(rho: float, M: int = 32) -> np.ndarray:
    """Isotropic decay rho ** distance-to-support-centre, (M, M) float64."""
    c = (M - 1) / 2.0
    m = np.arange(M, dtype=np.float64)
    d = np.sqrt((m[:, None] - c) ** 2 + (m[None, :] - c) ** 2)
    return rho ** d


def prior_table(sigma: float, M: int = 32) -> np.ndarray:
    """(M, M) frequency-weighting prior sigma ** |k| (all ones for sigma = 0,
    the option switched off)."""
    if sigma == 0:
        return np.ones((M, M))
    f = np.minimum(np.arange(M), M - np.arange(M)).astype(np.float64)
    return sigma ** np.sqrt(f[:, None] ** 2 + f[None, :] ** 2)


def _basis(b1, b2, M):
    """phi_b[m,n] = exp(2 pi i b1 m / M) * exp(2 pi i b2 n / M)."""
    m = np.arange(M, dtype=np.float64)
    e1 = np.exp(2j * np.pi * b1[:, None] * m[None, :] / M)
    e2 = np.exp(2j * np.pi * b2[:, None] * m[None, :] / M)
    return e1[:, :, None] * e2[:, None, :]


def fsr_spatial(s, w, gamma, K, track_gaps=False, stop_ratio=0.0, prior=None):
    """Greedy FSR on a batch of supports (independent blocks).

    s: (nb, M, M) real or complex samples (0 where unknown), w: (nb, M, M)
    real weights.  Returns (c (nb,M,M) complex coefficients,
    picks (nb,K) flat bin indices (-1 after an early stop), gaps (nb,) or
    None, (energies, chosen)): energies[i] = sum w |r|^2 after iteration i,
    chosen[i] = the criterion value (|R_b|^2, times prior_b with a prior) of
    the bin chosen at iteration i (0 once stopped).

    prior: optional (M, M) frequency weights (`prior_table`); stop_ratio > 0:
    residual-energy early stop (module docstring).

    With track_gaps, gaps[b] is the minimum over iterations of
    (E_best - E_next) / E_best, where E_next excludes the chosen bin and,
    while the residual spectrum is Hermitian (real data and only
    self-conjugate bins chosen so far), also its conjugate partner: choosing
    the partner then gives the conjugate trajectory and the same real model.
    """
    s = np.asarray(s)
    w = np.asarray(w, np.float64)
    nb, M, _ = w.shape
    idx = np.arange(nb)
    r = s.astype(np.complex128).copy()
    c = np.zeros((nb, M * M), np.complex128)
    W0 = w.sum(axis=(1, 2))
    safe = W0 > 0
    picks = np.zeros((nb, K), np.int64)
    gaps = np.full(nb, np.inf) if track_gaps else None
    herm = np.full(nb, bool(np.isrealobj(s) or not np.any(np.imag(s))))
    pw = None if prior is None else np.asarray(prior, np.float64).reshape(M * M)
    energies = []      # weighted residual energy sum w|r|^2 after each iteration
    chosen = []        # criterion value of the chosen bin at each iteration
    active = np.ones(nb, bool)
    E0 = None
    for it in range(K):
        Rs = np.fft.fft2(w * r).reshape(nb, M * M)
        E = Rs.real ** 2 + Rs.imag ** 2
        if pw is not None:
            E = E * pw[None]
        b = E.argmax(axis=1)
        Rb = Rs[idx, b]
        if stop_ratio > 0:
            Eb = E[idx, b]
            if it == 0:
                E0 = Eb.copy()
            else:
                thr = stop_ratio * E0
                if track_gaps:   # a decision within rounding of the threshold is a near tie too
                    with np.errstate(divide="ignore", invalid="ignore"):
                        tg = np.where(active & (Eb > 0), np.abs(Eb - thr) / Eb, np.inf)
                    gaps = np.minimum(gaps, tg)
                active &= Eb >= thr
        picks[:, it] = np.where(active, b, -1)
        chosen.append(np.where(active, E[idx, b], 0.0))
        dlt = np.where(safe & active, gamma * Rb / np.where(safe, W0, 1.0), 0.0)
        c[idx, b] += dlt
        b1, b2 = b // M, b % M
        r -= dlt[:, None, None] * _basis(b1, b2, M)
        if track_gaps:
            E1 = E[idx, b]
            Es = E.copy()
            Es[idx, b] = -np.inf
            partner = ((-b1) % M) * M + ((-b2) % M)
            hp = herm & (partner != b)
            Es[idx[hp], partner[hp]] = -np.inf
            E2 = Es.max(axis=1)
            with np.errstate(divide="ignore", invalid="ignore"):
                g = np.where(active & (E1 > 0), (E1 - E2) / E1, np.inf)
            gaps = np.minimum(gaps, g)
            herm &= partner == b
        energies.append((w * np.abs(r) ** 2).sum(axis=(1, 2)))
    return c.reshape(nb, M, M), picks, gaps, (energies, chosen)


def fsr_spectral(s, w, gamma, K, stop_ratio=0.0, prior=None):
    """Same loop with an in-place residual-spectrum update
    R_k <- R_k - dlt * W_{(k-b) mod M}.  Returns (c, picks)."""
    s = np.asarray(s)
    w = np.asarray(w, np.float64)
    nb, M, _ = w.shape
    idx = np.arange(nb)
    R = np.fft.fft2(w * s.astype(np.complex128))
    Wsp = np.fft.fft2(w)
    W0 = w.sum(axis=(1, 2))
    safe = W0 > 0
    c = np.zeros((nb, M * M), np.complex128)
    picks = np.zeros((nb, K), np.int64)
    m = np.arange(M)
    pw = None if prior is None else np.asarray(prior, np.float64).reshape(M * M)
    active = np.ones(nb, bool)
    E0 = None
    for it in range(K):
        Rf = R.reshape(nb, M * M)
        E = Rf.real ** 2 + Rf.imag ** 2
        if pw is not None:
            E = E * pw[None]
        b = E.argmax(axis=1)
        if stop_ratio > 0:
            if it == 0:
                E0 = E[idx, b].copy()
            else:
                active &= E[idx, b] >= stop_ratio * E0
        picks[:, it] = np.where(active, b, -1)
        dlt = np.where(safe & active, gamma * Rf[idx, b] / np.where(safe, W0, 1.0), 0.0)
        c[idx, b] += dlt
        b1, b2 = b // M, b % M
        i1 = (m[None, :] - b1[:, None]) % M
        i2 = (m[None, :] - b2[:, None]) % M
        R = R - dlt[:, None, None] * Wsp[idx[:, None, None], i1[:, :, None], i2[:, None, :]]
    return c.reshape(nb, M, M), picks


def fsr_pairs_spatial(s, w, gamma, K, track_gaps=False):
    """Real-valued FSR with conjugate pairs (the form the FSR literature
    uses for real images; a variant beside the complex single-bin loop that
    is read as the paper's FSR).  Each iteration picks the first bin b in
    row-major order maximising |R_b|^2 of the weighted residual DFT (the
    spectrum of a real residual is Hermitian, so b and -b tie and the first
    is the one with b1 <= 16), dlt = gamma R_b / W0, and adds the real pair
    dlt phi_b + conj(dlt) phi_-b to the model (dlt phi_b alone, real, when
    b = -b); the residual stays real.  Returns (c (nb,M,M) complex,
    picks (nb,K)) and, with track_gaps, gaps (nb,): the minimum over
    iterations of (E_best - E_next) / E_best with the chosen bin and its
    conjugate partner excluded from E_next."""
    s = np.asarray(s, np.float64)
    w = np.asarray(w, np.float64)
    nb, M, _ = w.shape
    idx = np.arange(nb)
    r = s.copy()
    c = np.zeros((nb, M * M), np.complex128)
    W0 = w.sum(axis=(1, 2))
    safe = W0 > 0
    picks = np.zeros((nb, K), np.int64)
    gaps = np.full(nb, np.inf)
    for it in range(K):
        Rs = np.fft.fft2(w * r).reshape(nb, M * M)
        E = Rs.real ** 2 + Rs.imag ** 2
        b = E.argmax(axis=1)
        picks[:, it] = b
        dlt = np.where(safe, gamma * Rs[idx, b] / np.where(safe, W0, 1.0), 0.0)
        b1, b2 = b // M, b % M
        partner = ((-b1) % M) * M + ((-b2) % M)
        self_conj = partner == b
        if track_gaps:
            E1 = E[idx, b]
            Es = E.copy()
            Es[idx, b] = -np.inf
            Es[idx, partner] = -np.inf
            with np.errstate(divide="ignore", invalid="ignore"):
                gaps = np.minimum(gaps, np.where(E1 > 0, (E1 - Es.max(axis=1)) / E1, np.inf))
        c[idx, b] += dlt
        c[idx[~self_conj], partner[~self_conj]] += np.conj(dlt[~self_conj])
        phi = _basis(b1, b2, M)
        # real update: dlt phi_b (+ its conjugate for a pair)
        upd = dlt[:, None, None] * phi
        r -= np.where(self_conj[:, None, None], upd.real, 2.0 * upd.real)
    if track_gaps:
        return c.reshape(nb, M, M), picks, gaps
    return c.reshape(nb, M, M), picks


def fsr_pairs_spectral(s, w, gamma, K):
    """The same loop on the residual spectrum:
    R_k <- R_k - dlt W_{k-b} - conj(dlt) W_{k+b}  (one term for b = -b)."""
    s = np.asarray(s, np.float64)
    w = np.asarray(w, np.float64)
    nb, M, _ = w.shape
    idx = np.arange(nb)
    R = np.fft.fft2(w * s)
    Wsp = np.fft.fft2(w)
    W0 = w.sum(axis=(1, 2))
    safe = W0 > 0
    c = np.zeros((nb, M * M), np.complex128)
    picks = np.zeros((nb, K), np.int64)
    m = np.arange(M)
    for it in range(K):
        Rf = R.reshape(nb, M * M)
        E = Rf.real ** 2 + Rf.imag ** 2
        b = E.argmax(axis=1)
        picks[:, it] = b
        dlt = np.where(safe, gamma * Rf[idx, b] / np.where(safe, W0, 1.0), 0.0)
        b1, b2 = b // M, b % M
        partner = ((-b1) % M) * M + ((-b2) % M)
        self_conj = partner == b
        c[idx, b] += dlt
        c[idx[~self_conj], partner[~self_conj]] += np.conj(dlt[~self_conj])
        i1 = (m[None, :] - b1[:, None]) % M
        i2 = (m[None, :] - b2[:, None]) % M
        j1 = (m[None, :] + b1[:, None]) % M
        j2 = (m[None, :] + b2[:, None]) % M
        Wm = Wsp[idx[:, None, None], i1[:, :, None], i2[:, None, :]]
        Wp = Wsp[idx[:, None, None], j1[:, :, None], j2[:, None, :]]
        d = dlt[:, None, None]
        R = R - d * Wm - np.where(self_conj[:, None, None], 0.0, np.conj(d) * Wp)
    return c.reshape(nb, M, M), picks


def fsr_pairs_blocks_out(values, cls, blocks, B=4, M=32, rho=0.7, gamma=0.5, K=50,
                         proj_weight=1.0, overwrite="dfsr", chunk=2048):
    """Conjugate-pair FSR of the listed blocks (overwrite as fsr_blocks_out).
    Returns (out (nb, B, B) float64, gaps (nb,))."""
    blocks = np.asarray(blocks, np.int64).reshape(-1, 2)
    tab = rho_table(rho, M)
    outs, gaps = [], []
    for i in range(0, blocks.shape[0], chunk):
        blk = blocks[i:i + chunk]
        s, a = gather_supports(values, cls, blk, B, M, proj_weight)
        c, _, g = fsr_pairs_spatial(s, a * tab[None], gamma, K, track_gaps=True)
        gaps.append(g)
        out = synthesize(c, B)
        for j, (bi, bj) in enumerate(blk):
            cb = cls[B * bi:B * bi + B, B * bj:B * bj + B]
            vb = values[B * bi:B * bi + B, B * bj:B * bj + B]
            keep = (cb == 1) if overwrite == "dfsr" else (cb >= 1)
            out[j][keep] = vb[keep]
        outs.append(out)
    return np.concatenate(outs), np.concatenate(gaps)


def synthesize(c, B):
    """Block output Re(sum_k c_k phi_k) on the B x B block pixels."""
    nb, M, _ = c.shape
    g = (M * M) * np.fft.ifft2(c)
    o = (M - B) // 2
    return g[:, o:o + B, o:o + B].real


def class_weight(cls, proj_weight):
    """a = 1 measured, pi_w projected, 0 unknown."""
    return np.where(cls == 1, 1.0, np.where(cls == 2, proj_weight, 0.0))


def gather_supports(values, cls, blocks, B=4, M=32, proj_weight=1.0):
    """Samples and class weights on the supports of the listed blocks.

    blocks: (nb, 2) int block indices (bi, bj).  Positions outside the frame
    and unknown positions get weight 0 and sample 0 (never read)."""
    H, W = values.shape
    o = (M - B) // 2
    a = class_weight(cls, proj_weight)
    v = np.where(cls > 0, values, 0.0)
    pad_lo, pad_hi = o, M - B - o
    vp = np.pad(v, ((pad_lo, pad_hi + B), (pad_lo, pad_hi + B)))
    ap = np.pad(a, ((pad_lo, pad_hi + B), (pad_lo, pad_hi + B)))
    blocks = np.asarray(blocks, np.int64).reshape(-1, 2)
    nb = blocks.shape[0]
    s = np.empty((nb, M, M))
    aw = np.empty((nb, M, M))
    for i, (bi, bj) in enumerate(blocks):
        y0, x0 = B * bi, B * bj   # = (B*bi - o) + pad_lo
        s[i] = vp[y0:y0 + M, x0:x0 + M]
        aw[i] = ap[y0:y0 + M, x0:x0 + M]
    return s, aw


def fsr_blocks_out(values, cls, blocks, B=4, M=32, rho=0.7, gamma=0.5, K=100,
                   proj_weight=1.0, overwrite="dfsr", track_gaps=True, chunk=2048,
                   prior_sigma=0.0, stop_ratio=0.0):
    """FSR of the listed blocks.  Returns (out (nb,B,B) float64, gaps (nb,))."""
    blocks = np.asarray(blocks, np.int64).reshape(-1, 2)
    tab = rho_table(rho, M)
    prior = prior_table(prior_sigma, M) if prior_sigma > 0 else None
    outs, gaps = [], []
    for i in range(0, blocks.shape[0], chunk):
        blk = blocks[i:i + chunk]
        s, a = gather_supports(values, cls, blk, B, M, proj_weight)
        c, _, g, _ = fsr_spatial(s, a * tab[None], gamma, K, track_gaps=track_gaps, stop_ratio=stop_ratio,
                                 prior=prior)
        out = synthesize(c, B)
        # overwrite with measured (D-FSR) or measured + projected (R-FSR) values
        for j, (bi, bj) in enumerate(blk):
            cb = cls[B * bi:B * bi + B, B * bj:B * bj + B]
            vb = values[B * bi:B * bi + B, B * bj:B * bj + B]
            keep = (cb == 1) if overwrite == "dfsr" else (cb >= 1)
            out[j][keep] = vb[keep]
        outs.append(out)
        gaps.append(g if g is not None else np.full(blk.shape[0], np.inf))
    return np.concatenate(outs), np.concatenate(gaps)


def fsr_frame_concealed(values, cls, delta, B=4, M=32, rho=0.7, gamma=0.5, K=100,
                        proj_weight=1.0, overwrite="dfsr", given=None):
    """FSR with a non-zero concealed weighting `delta` (the setting of the
    FSR literature that Sec. 4 sets to zero).  Blocks are reconstructed one
    after another in raster order (block rows top to bottom, each left to
    right); a pixel of an earlier block that had no sample (class 0) enters
    the supports of later blocks as a sample with weight delta * rho^dist
    and its reconstructed value (the block output, float).  delta = 0 is
    `fsr_frame`.  given: optional (H, W) reconstruction whose values the
    concealed pixels take instead of this function's own outputs (to check
    another implementation block by block on its own upstream values).
    Returns (out (H, W) float64, gaps (H/B, W/B)) as `fsr_frame`.

    Reading: the reconstructed value is the unclamped model output; measured
    and projected pixels keep their own weights and values."""
    H, W = values.shape
    v = np.where(cls > 0, values, 0.0).astype(np.float64)
    a = class_weight(cls, proj_weight)          # concealed pixels get `delta` below
    out = np.zeros((H, W))
    gaps = np.zeros((H // B, W // B))
    tab = rho_table(rho, M)
    for bi in range(H // B):
        for bj in range(W // B):
            blk = np.array([[bi, bj]])
            s, aw = _gather(v, a, blk, B, M)
            c, _, g, _ = fsr_spatial(s, aw * tab[None], gamma, K, track_gaps=True)
            gaps[bi, bj] = g[0]
            o = synthesize(c, B)[0]
            sl = (slice(B * bi, B * bi + B), slice(B * bj, B * bj + B))
            cb, vb = cls[sl], values[sl]
            keep = (cb == 1) if overwrite == "dfsr" else (cb >= 1)
            o[keep] = vb[keep]
            out[sl] = o
            unknown = cb == 0
            src = o if given is None else np.asarray(given, np.float64)[sl]
            v[sl][unknown] = src[unknown]        # concealed from now on
            a[sl][unknown] = delta
    return out, gaps


def _gather(v, a, blocks, B, M):
    """Samples v and weights a on the supports of `blocks` (zero outside)."""
    o = (M - B) // 2
    pad = ((o, M - B - o + B), (o, M - B - o + B))
    vp, ap = np.pad(v, pad), np.pad(a, pad)
    s = np.empty((len(blocks), M, M))
    aw = np.empty((len(blocks), M, M))
    for i, (bi, bj) in enumerate(blocks):
        s[i] = vp[B * bi:B * bi + M, B * bj:B * bj + M]
        aw[i] = ap[B * bi:B * bi + M, B * bj:B * bj + M]
    return s, aw


def all_blocks(H, W, B=4):
    bi, bj = np.mgrid[0:H // B, 0:W // B]
    return np.stack([bi.ravel(), bj.ravel()], axis=1)


def fsr_frame(values, cls, B=4, M=32, rho=0.7, gamma=0.5, K=100, proj_weight=1.0,
              overwrite="dfsr", track_gaps=True, prior_sigma=0.0, stop_ratio=0.0):
    """FSR of a whole frame.  Returns (out (H,W) float64, gaps (H/B, W/B))."""
    H, W = values.shape
    blocks = all_blocks(H, W, B)
    out_b, gaps = fsr_blocks_out(values, cls, blocks, B, M, rho, gamma, K, proj_weight,
                                 overwrite, track_gaps, prior_sigma=prior_sigma, stop_ratio=stop_ratio)
    out = out_b.reshape(H // B, W // B, B, B).transpose(0, 2, 1, 3).reshape(H, W)
    return out, gaps.reshape(H // B, W // B)
