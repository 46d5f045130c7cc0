"""Plain FP64 oracle of distributed FastMNMF (block-diagonal spatial covariances).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It is slow on
purpose: NumPy complex128 / float64, each step written the way the paper states
it, no blocking, fusion or reordering beyond the factorisation the paper itself
gives for the model variance (Sec. III-B, complexity discussion).  It shares no
code with the HIP path.

Notation (the paper's symbols -> names used here):

* frequency i -> f, frame j -> t, mic m, subarray l with M_l mics, in-subarray
  mic mu, global mic m = o_l + mu where o_l = M_1 + ... + M_{l-1}.
* transformation W_i^(l) -> Q_fl = W_i^(l)H, so row mu of Q_fl is w_mu^H and
  the decorrelated signal y_ij^(l) = Q_fl x_ft^(l).
* spectral basis t_ikn -> W[n, f, k]; activation v_kjn -> H[n, k, t];
  diagonal SCM entries [Lambda_in]_mm -> g[f, n, m]; model variance
  eta_ijm -> y[f, t, m]; |y_ijm|^2 -> P[f, t, m]; IP covariance Q_imu^(l) -> V.

State layout (the same interface the C ABI takes):
  X [F, T, M] complex; Q [F, sum_l M_l^2] complex, block l row-major
  M_l x M_l starting at sum_{l'<l} M_l'^2; g [F, N, M]; W [N, F, K]; H [N, K, T].

Readings of points the paper leaves open (each listed in the design notes):
  * one iteration = IP sweep over every subarray (eqs. (14)-(16)), then the
    MM updates (8), (9), (10) in that order, with eta refreshed after each
    (Sec. II-A, last paragraph; Sec. III-B, last paragraphs);
  * inside a subarray the rows mu are updated in ascending order, each solve
    using the rows already updated (IP, eq. (15));
  * the 1e-6 floors (Sec. IV-A) are absolute maxima on eta, on the MM
    denominators and on the normaliser w^H Q w of eq. (16);
  * a singular system in eq. (15) falls back to the pseudo-inverse
    (Sec. IV-A);
  * no rescaling of Q, g, W, H between iterations (the paper states none).
"""
from __future__ import annotations

import numpy as np

EPS = 1e-6


# ---------------------------------------------------------------- layout
def block_offsets(mics):
    """(mic offset o_l, packed-Q offset) of each subarray."""
    mo, qo, outs = 0, 0, []
    for ml in mics:
        outs.append((mo, qo))
        mo += ml
        qo += ml * ml
    return outs


def q_blocks(Q, mics):
    """Split packed Q [F, sum M_l^2] into a list of Q_fl arrays [F, M_l, M_l]."""
    F = Q.shape[0]
    return [np.array(Q[:, qo:qo + ml * ml].reshape(F, ml, ml), dtype=np.complex128)
            for ml, (_, qo) in zip(mics, block_offsets(mics))]


def q_pack(blocks):
    """Inverse of :func:`q_blocks`."""
    F = blocks[0].shape[0]
    return np.concatenate([b.reshape(F, -1) for b in blocks], axis=1)


# ---------------------------------------------------------------- model
def source_psd(W, H):
    """lambda[f, t, n] = sum_k t_fkn v_ktn -- the NMF source spectrogram, eq. (2)."""
    return np.einsum("nfk,nkt->ftn", W, H, optimize=True)


def model_variance(lam, g, eps=EPS):
    """y[f, t, m] = max(sum_n lambda_ftn g_fnm, eps).

    This is eta_ijm of eq. (14) (and of eqs. (8)-(10)) in the factorised
    form sum_n (sum_k t v) [Lambda]_mm that Sec. III-B gives; the floor is the
    1e-6 floor on eta of Sec. IV-A.
    """
    y = np.einsum("ftn,fnm->ftm", lam, g, optimize=True)
    return np.maximum(y, eps)


def powers(X, Q, mics):
    """P[f, t, o_l + mu] = |(Q_fl x_ft^(l))_mu|^2, the |y^(l)_ijmu|^2 of eq. (13)."""
    F, T, M = X.shape
    P = np.empty((F, T, M))
    for Ql, ml, (mo, _) in zip(q_blocks(Q, mics), mics, block_offsets(mics)):
        z = np.einsum("fua,fta->ftu", Ql, X[:, :, mo:mo + ml], optimize=True)
        P[:, :, mo:mo + ml] = z.real ** 2 + z.imag ** 2
    return P


# ---------------------------------------------------------------- IP, eqs. (14)-(16)
def weighted_covariances(X, y, mics):
    """V_l[f, mu] = (1/T) sum_t x^(l)_ft x^(l)H_ft / y_{f,t,o_l+mu}, eq. (14).

    Returns a list over subarrays of arrays [F, M_l (mu), M_l, M_l].
    """
    T = X.shape[1]
    out = []
    for ml, (mo, _) in zip(mics, block_offsets(mics)):
        xl = X[:, :, mo:mo + ml]
        w = 1.0 / y[:, :, mo:mo + ml]
        out.append(np.einsum("ftu,fta,ftb->fuab", w, xl, xl.conj(), optimize=True) / T)
    return out


def _solve_or_pinv(A, e):
    """Solve A b = e for a stack of systems; pseudo-inverse where A is singular (Sec. IV-A)."""
    try:
        return np.linalg.solve(A, e[..., None])[..., 0]
    except np.linalg.LinAlgError:
        out = np.empty_like(e)
        for f in range(A.shape[0]):
            try:
                out[f] = np.linalg.solve(A[f], e[f])
            except np.linalg.LinAlgError:
                out[f] = np.linalg.pinv(A[f]) @ e[f]
        return out


def ip_update_row(Ql, Vmu, mu, eps=EPS):
    """One IP row update for every frequency: eqs. (15) and (16).

    Ql [F, M_l, M_l] holds rows w_mu^H.  Solves (W^H V_mu) w = e_mu, then scales
    w by (max(w^H V_mu w, eps))^(-1/2) and stores w^H as row mu.  Returns a new
    array (the input is not modified).
    """
    F, ml, _ = Ql.shape
    A = Ql @ Vmu                                        # W_i^(l)H Q^(l)_imu
    e = np.zeros((F, ml), dtype=np.complex128)
    e[:, mu] = 1.0
    w = _solve_or_pinv(A, e)
    s = np.einsum("fa,fab,fb->f", w.conj(), Vmu, w).real
    w = w / np.sqrt(np.maximum(s, eps))[:, None]
    out = Ql.copy()
    out[:, mu, :] = w.conj()
    return out


def ip_sweep(Q, V, mics, eps=EPS):
    """Update every subarray's transformation by IP, rows in ascending order, eqs. (15)-(16).

    V is the list returned by :func:`weighted_covariances`; it is formed once
    before the sweep since eta does not depend on Q.
    """
    blocks = q_blocks(Q, mics)
    for l, ml in enumerate(mics):
        for mu in range(ml):
            blocks[l] = ip_update_row(blocks[l], V[l][:, mu], mu, eps)
    return q_pack(blocks)


def logabsdet(Q, mics):
    """ln|det Q_fl| for every (f, l): [F, L]."""
    return np.stack([np.linalg.slogdet(b)[1] for b in q_blocks(Q, mics)], axis=1)


# ---------------------------------------------------------------- MM, eqs. (8)-(10)
def mm_terms_W(W, H, g, P, eps=EPS):
    """Numerator and denominator of eq. (8) for every t_ikn -> W[n, f, k].

    num = sum_{t,m} H[n,k,t] g[f,n,m] P[f,t,m] / y^2, den = sum_{t,m} H g / y.
    """
    y = model_variance(source_psd(W, H), g, eps)
    a = np.einsum("fnm,ftm->ftn", g, P / y ** 2, optimize=True)
    b = np.einsum("fnm,ftm->ftn", g, 1.0 / y, optimize=True)
    num = np.einsum("nkt,ftn->nfk", H, a, optimize=True)
    den = np.einsum("nkt,ftn->nfk", H, b, optimize=True)
    return num, den


def mm_terms_H(W, H, g, P, eps=EPS):
    """Numerator and denominator of eq. (9) for every v_kjn -> H[n, k, t] (sums over f and m)."""
    y = model_variance(source_psd(W, H), g, eps)
    a = np.einsum("fnm,ftm->ftn", g, P / y ** 2, optimize=True)
    b = np.einsum("fnm,ftm->ftn", g, 1.0 / y, optimize=True)
    num = np.einsum("nfk,ftn->nkt", W, a, optimize=True)
    den = np.einsum("nfk,ftn->nkt", W, b, optimize=True)
    return num, den


def mm_terms_g(W, H, g, P, eps=EPS):
    """Numerator and denominator of eq. (10) for every [Lambda_in]_mm -> g[f, n, m] (sums over t and k)."""
    lam = source_psd(W, H)
    y = model_variance(lam, g, eps)
    num = np.einsum("ftn,ftm->fnm", lam, P / y ** 2, optimize=True)
    den = np.einsum("ftn,ftm->fnm", lam, 1.0 / y, optimize=True)
    return num, den


def _mm_apply(x, num, den, eps):
    return x * np.sqrt(num / np.maximum(den, eps))


def update_W(W, H, g, P, eps=EPS):
    """Eq. (8), with the denominator floored at eps (Sec. IV-A)."""
    return _mm_apply(W, *mm_terms_W(W, H, g, P, eps), eps)


def update_H(W, H, g, P, eps=EPS):
    """Eq. (9), with the denominator floored at eps."""
    return _mm_apply(H, *mm_terms_H(W, H, g, P, eps), eps)


def update_g(W, H, g, P, eps=EPS):
    """Eq. (10), with the denominator floored at eps."""
    return _mm_apply(g, *mm_terms_g(W, H, g, P, eps), eps)


# ---------------------------------------------------------------- iteration
def iterate(X, Q, g, W, H, mics, n_iter, eps=EPS, callback=None):
    """Run n_iter iterations of distributed FastMNMF (Sec. III-B, last paragraphs).

    Each iteration: eta from the current (W, H, g); V by eq. (14); IP sweep by
    eqs. (15)-(16); P = |Q x|^2; then eq. (8), eq. (9), eq. (10), each with eta
    recomputed from the freshest parameters.  ``callback(stage, Q, g, W, H)``
    is called after each stage ("ip", "W", "H", "g") when given.
    Returns (Q, g, W, H) as new arrays.
    """
    Q, g, W, H = (np.array(a) for a in (Q, g, W, H))
    for _ in range(n_iter):
        y = model_variance(source_psd(W, H), g, eps)
        Q = ip_sweep(Q, weighted_covariances(X, y, mics), mics, eps)
        if callback:
            callback("ip", Q, g, W, H)
        P = powers(X, Q, mics)
        W = update_W(W, H, g, P, eps)
        if callback:
            callback("W", Q, g, W, H)
        H = update_H(W, H, g, P, eps)
        if callback:
            callback("H", Q, g, W, H)
        g = update_g(W, H, g, P, eps)
        if callback:
            callback("g", Q, g, W, H)
    return Q, g, W, H


# ---------------------------------------------------------------- cost and outputs
def nll(X, Q, g, W, H, mics, eps=EPS):
    """Cost (13): sum_{f,t,m} (P/y + ln y) - 2T sum_{f,l} ln|det Q_fl| (no additive constant)."""
    T = X.shape[1]
    P = powers(X, Q, mics)
    y = model_variance(source_psd(W, H), g, eps)
    return float(np.sum(P / y + np.log(y)) - 2.0 * T * np.sum(logabsdet(Q, mics)))


def separate(X, Q, g, W, H, mics, eps=EPS):
    """Source images at every subarray by the multichannel Wiener filter.

    With R_fn = Q_f^{-1} diag(g_fn) Q_f^{-H} (eqs. (3), (11), (12)) and the
    model covariance Q_f^{-1} diag(y_ft) Q_f^{-H} of eq. (1), the Wiener
    estimate lambda_ftn R_fn (sum)^{-1} x_ft becomes, per subarray,
    Q_fl^{-1} diag(lambda_ftn g_fn / y_ft) Q_fl x_ft^(l).
    Returns S[N, F, T, M] complex128.
    """
    F, T, M = X.shape
    N = W.shape[0]
    lam = source_psd(W, H)
    y = model_variance(lam, g, eps)
    S = np.empty((N, F, T, M), dtype=np.complex128)
    for Ql, ml, (mo, _) in zip(q_blocks(Q, mics), mics, block_offsets(mics)):
        Qinv = np.linalg.inv(Ql)
        z = np.einsum("fua,fta->ftu", Ql, X[:, :, mo:mo + ml], optimize=True)
        for n in range(N):
            gain = lam[:, :, n, None] * g[:, None, n, mo:mo + ml] / y[:, :, mo:mo + ml]
            S[n, :, :, mo:mo + ml] = np.einsum("fab,ftb->fta", Qinv, gain * z, optimize=True)
    return S
