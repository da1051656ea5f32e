"""Plain FP64 CPU oracle for matrix-free stochastic reconfiguration (SR) and the
linear method (LM), after Neuscamman, Umrigar and Chan, "Optimizing large parameter
sets in variational quantum Monte Carlo" (arXiv:1108.0900).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this module; only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may call
it.  It shares no code with the GPU path: it is written directly from the paper's
equations in numpy/scipy, float64 throughout, with no blocking, fusion or
reordering beyond what each definition states.

Notation (all arrays float64 unless stated):
  O[k, i]   derivative ratio Psi^i_n / Psi_n of parameter i on sample k
            (Sec. II.A, the ratios inside Eq. sr_overlap); N_s rows, N_p columns.
  E[k]      local energy (H Psi)_n / Psi_n of sample k.
  w[k]      weight of sample k.  Eq. sr_overlap sums over all configurations with
            weight |Psi_n|^2/<Psi|Psi>; Monte Carlo sampling from that distribution
            replaces it by the uniform weight 1/N_s, which is the default here.
  S         overlap matrix, centred form (see the reading below).
  g         energy gradient, the right-hand side of the centred SR system.

Reading of the SR system (Sec. II.A, Eq. sr_lin_eq).  The paper's system is posed in
the (N_p+1)-dimensional basis {Psi, d_i Psi}.  Eliminating x_0 (the coefficient of
Psi) by a Schur complement leaves the centred N_p-dimensional system
    S_c x = -(tau/2) g,  S_c = <(O_i - <O_i>)(O_j - <O_j>)>,  g_i = 2<(E - <E>)(O_i - <O_i>)>,
and x_0 = 1 - tau<E> - <O>.x.  The hot path solves (S_c + eps I) x = g; the caller
applies the -(tau/2) factor.  `paper_linear_system` builds the uncentred system so
the test suite can check this equivalence.

Functions and the passage each follows:
  sample_weights, sample_mean ............ Sec. II.A, Eq. sr_overlap (weights)
  overlap_matrix ......................... Sec. II.A, Eq. sr_overlap (formed explicitly)
  overlap_matrix_uncentred ............... Sec. II.A, Eq. sr_overlap with Psi^0 = Psi
  energy_gradient, diag_overlap .......... Sec. II.A, Eq. sr_lin_eq (centred right-hand side)
  sv_product_dense ....................... Sec. II.A, Eq. sr_multiply_1 (explicit S times z)
  sv_product_swapped ..................... Sec. II.A, Eq. sr_multiply_2 (sums interchanged)
  paper_linear_system, sr_update ......... Sec. II.A, Eq. sr_lin_eq and alpha' = alpha + x_i/x_0
  solve_dense ............................ Sec. II.A, Eq. sr_lin_eq solved by Cholesky
  solve_dual ............................. the same solution through the N_s x N_s dual system
  cg_solve ............................... Sec. II.A, conjugate gradient (Hestenes-Stiefel)
  lm_matrices, lm_hv_dense ............... Sec. II.B, Eq. linear_eigen (H and S in Omega)
  lm_lowest_eigenpair .................... Sec. II.B, Eq. linear_eigen (dense generalized solve)
  quantize_bf16/_f16/_split, dequantize_* . precision form of the stored ratios (not in the paper)
  quantize_cols, dequantize_cols ......... remainder codes kept only for the columns that need them
  solve_adjoint_gradients ................ implicit-adjoint derivative of the solve (not in the paper)
  cps_expand ............................. Sec. II.C, Eq. ansatz: the derivative ratios of an
                                           index-coded correlator-product state, written out

Every function is pinned by the CPU tests against something other than itself
(library routines, closed forms, invariants, exact enumeration of a tiny Hilbert
space, finite differences).  Parity pins are listed in the test files.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = [
    "sample_weights", "sample_mean", "centred", "overlap_matrix", "overlap_matrix_uncentred",
    "energy_gradient", "energy_mean", "diag_overlap", "sv_product_dense", "sv_product_swapped",
    "paper_linear_system", "sr_update", "solve_dense", "solve_dual", "cg_solve", "lm_matrices", "lm_hv_dense", "lm_hv_swapped",
    "lm_lowest_eigenpair", "quantize_bf16", "dequantize_bf16", "quantize_f16", "dequantize_f16",
    "quantize_split", "dequantize_split", "quantize_cols", "dequantize_cols", "REMAINDER_TOL", "cps_expand",
    "solve_adjoint_gradients",
]


# ----------------------------------------------------------------------------------------------
# Sampled averages (Sec. II.A, Eq. sr_overlap)
# ----------------------------------------------------------------------------------------------
def sample_weights(n_s: int, w=None) -> np.ndarray:
    """Weights of the sampled configurations.

    Eq. sr_overlap weights each configuration by |Psi_n|^2/<Psi|Psi>; sampling from that
    distribution turns the sum into a plain average, i.e. weight 1/N_s per sample.
    An explicit `w` (summing to one) is used for exact enumeration of small spaces.
    """
    if w is None:
        return np.full(n_s, 1.0 / n_s)
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (n_s,)
    return w


def sample_mean(O, w=None) -> np.ndarray:
    """<O_i> = sum_n w_n O_ni, the overlap of Psi with Psi^i over <Psi|Psi>."""
    O = np.asarray(O, dtype=np.float64)
    w = sample_weights(O.shape[0], w)
    return w @ O


def energy_mean(E, w=None) -> float:
    """<E> = sum_n w_n E_n, the sampled energy."""
    E = np.asarray(E, dtype=np.float64)
    w = sample_weights(E.shape[0], w)
    return float(w @ E)


def centred(O, w=None) -> np.ndarray:
    """Ratios of the centred derivatives Psi^i - <O_i> Psi (R1 reading of Eq. sr_lin_eq)."""
    O = np.asarray(O, dtype=np.float64)
    return O - sample_mean(O, w)[None, :]


def overlap_matrix(O, w=None) -> np.ndarray:
    """Centred overlap S_ij = <(O_i - <O_i>)(O_j - <O_j>)>, formed explicitly.

    This is Eq. sr_overlap (the sampled <Psi^i|Psi^j>/<Psi|Psi>) taken in the centred basis;
    building it costs O(N_s N_p^2), which the matrix-free method avoids.
    """
    Oc = centred(O, w)
    w = sample_weights(Oc.shape[0], w)
    return Oc.T @ (w[:, None] * Oc)


def overlap_matrix_uncentred(O, w=None) -> np.ndarray:
    """The paper's (N_p+1)-dimensional overlap of Eq. sr_overlap, with Psi^0 = Psi (ratio 1)."""
    O = np.asarray(O, dtype=np.float64)
    A = np.concatenate([np.ones((O.shape[0], 1)), O], axis=1)
    w = sample_weights(O.shape[0], w)
    return A.T @ (w[:, None] * A)


def energy_gradient(O, E, w=None) -> np.ndarray:
    """g_i = 2 <(E - <E>)(O_i - <O_i>)>, the energy gradient dE/dalpha_i of a real Psi.

    It is the right-hand side of the centred SR system (R1 reading of Eq. sr_lin_eq).
    """
    Oc = centred(O, w)
    E = np.asarray(E, dtype=np.float64)
    w = sample_weights(Oc.shape[0], w)
    ec = E - energy_mean(E, w)
    return 2.0 * (Oc.T @ (w * ec))


def diag_overlap(O, w=None) -> np.ndarray:
    """Diagonal of the centred overlap, S_ii = <(O_i - <O_i>)^2>."""
    Oc = centred(O, w)
    w = sample_weights(Oc.shape[0], w)
    return (w[:, None] * Oc * Oc).sum(axis=0)


# ----------------------------------------------------------------------------------------------
# Products with S (Sec. II.A, Eqs. sr_multiply_1 and sr_multiply_2)
# ----------------------------------------------------------------------------------------------
def sv_product_dense(O, v, eps: float = 0.0, w=None) -> np.ndarray:
    """(S + eps I) v with S formed explicitly first (Eq. sr_multiply_1 summed as written)."""
    S = overlap_matrix(O, w)
    v = np.asarray(v, dtype=np.float64)
    return S @ v + eps * v


def sv_product_swapped(O, v, eps: float = 0.0, w=None) -> np.ndarray:
    """(S + eps I) v with the sums interchanged (Eq. sr_multiply_2): per sample, the scalar
    sum_j O_nj v_j first, then sum_n w_n O_ni times that scalar.  Never forms S.
    Used as the CPU timing baseline of the matrix-free method."""
    Oc = centred(O, w)
    w = sample_weights(Oc.shape[0], w)
    v = np.asarray(v, dtype=np.float64)
    t = Oc @ v
    return Oc.T @ (w * t) + eps * v


# ----------------------------------------------------------------------------------------------
# The SR linear system (Sec. II.A, Eq. sr_lin_eq)
# ----------------------------------------------------------------------------------------------
def paper_linear_system(O, E, tau: float, w=None):
    """Uncentred system of Eq. sr_lin_eq: <Psi^i|(1 - tau H)|Psi> = sum_j <Psi^i|Psi^j> x_j.

    With Psi^0 = Psi, the left side sampled is <O_i (1 - tau E)> (O_0 = 1).
    Returns (A, b) with A the (N_p+1)^2 overlap and b the (N_p+1) right-hand side.
    """
    O = np.asarray(O, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    w = sample_weights(O.shape[0], w)
    A = overlap_matrix_uncentred(O, w)
    Ofull = np.concatenate([np.ones((O.shape[0], 1)), O], axis=1)
    b = Ofull.T @ (w * (1.0 - tau * E))
    return A, b


def sr_update(alpha, x_full) -> np.ndarray:
    """Parameter update alpha'_i = alpha_i + x_i / x_0 (Sec. II.A)."""
    x_full = np.asarray(x_full, dtype=np.float64)
    return np.asarray(alpha, dtype=np.float64) + x_full[1:] / x_full[0]


def solve_dense(O, g, eps: float, w=None) -> np.ndarray:
    """x = (S + eps I)^{-1} g with S built explicitly and factored by Cholesky.

    For eps = 0 and singular S the system is consistent (g lies in the range of S) and the
    result is defined as the minimum-norm solution pinv(S) g.
    """
    S = overlap_matrix(O, w)
    g = np.asarray(g, dtype=np.float64)
    n = S.shape[0]
    if eps > 0.0:
        c = sla.cho_factor(S + eps * np.eye(n), lower=True)
        return sla.cho_solve(c, g)
    return np.linalg.pinv(S, rcond=1e-12, hermitian=True) @ g


def solve_dual(O, g, eps: float, w=None) -> np.ndarray:
    """x = (S + eps I)^{-1} g through the N_s-dimensional dual system, for N_s << N_p:
    with S = Oc^T W Oc (W = diag(w)) the Woodbury identity gives
        x = (g - Oc^T W^{1/2} (eps I + W^{1/2} Oc Oc^T W^{1/2})^{-1} W^{1/2} Oc g) / eps,
    one N_s x N_s Cholesky solve (eps > 0).  Never forms S."""
    assert eps > 0.0
    Oc = centred(O, w)
    w = sample_weights(Oc.shape[0], w)
    g = np.asarray(g, dtype=np.float64)
    B = np.sqrt(w)[:, None] * Oc
    K = B @ B.T + eps * np.eye(B.shape[0])
    c = sla.cho_factor(K, lower=True)
    return (g - B.T @ sla.cho_solve(c, B @ g)) / eps


def cg_solve(apply_A, b, rtol: float = 1e-10, max_iter: int | None = None,
             refresh_every: int = 0, x0=None):
    """Conjugate gradient (Hestenes-Stiefel) for a symmetric positive (semi)definite A.

    Sec. II.A: iterate with matrix-vector products only, until the requested accuracy.
    Stops when ||r|| <= rtol ||b|| on the recurrence residual.  With refresh_every = m > 0,
    every m-th iteration replaces r by the true residual b - A x (keeping p).
    Returns (x, iterations, relative recurrence residual).
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    if max_iter is None:
        max_iter = n + 100
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rho = float(r @ r)
    bnorm = float(np.sqrt(b @ b))
    if bnorm == 0.0:
        return np.zeros(n), 0, 0.0
    it = 0
    while it < max_iter and np.sqrt(rho) > rtol * bnorm:
        q = apply_A(p)
        alpha = rho / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if refresh_every and it % refresh_every == 0:
            r = b - apply_A(x)
        rho_new = float(r @ r)
        beta = rho_new / rho
        p = r + beta * p
        rho = rho_new
    return x, it, float(np.sqrt(rho) / bnorm)


# ----------------------------------------------------------------------------------------------
# Linear method (Sec. II.B, Eq. linear_eigen)
# ----------------------------------------------------------------------------------------------
def lm_matrices(O, E, D, w=None):
    """Sampled H and S of the linear method in the basis {Psi, Psi^i - <O_i> Psi}.

    Reading: the paper's H.x (Eq. linear_multiply) needs the Hamiltonian itself; the
    sampled estimator used here needs only local energies E and their parameter
    derivatives D[k, j] = d E_L / d alpha_j, through (H Psi^j)_n / Psi_n = D_nj + E_n O_nj.
    In the centred basis that gives
        H_00 = <E>,  H_i0 = <Oc_i E>,  H_0j = <E Oc_j> + <D_j>,  H_ij = <Oc_i E Oc_j> + <Oc_i D_j>,
    and S = 1 (+) S_c (block diagonal).
    """
    O = np.asarray(O, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    w = sample_weights(O.shape[0], w)
    Oc = centred(O, w)
    n = O.shape[1]
    H = np.empty((n + 1, n + 1))
    H[0, 0] = w @ E
    H[1:, 0] = Oc.T @ (w * E)
    H[0, 1:] = (w * E) @ Oc + w @ D
    H[1:, 1:] = Oc.T @ (w[:, None] * (E[:, None] * Oc + D))
    S = np.zeros((n + 1, n + 1))
    S[0, 0] = 1.0
    S[1:, 1:] = Oc.T @ (w[:, None] * Oc)
    return H, S


def lm_hv_dense(O, E, D, v, w=None) -> np.ndarray:
    """H v with H from `lm_matrices`, formed explicitly."""
    H, _ = lm_matrices(O, E, D, w)
    return H @ np.asarray(v, dtype=np.float64)


def lm_hv_swapped(O, E, D, v, w=None) -> np.ndarray:
    """H v without forming H (the interchange of sums of Eq. sr_multiply_2 applied to the
    blocks of `lm_matrices`): per sample t_k = Oc_k . v_rest, u_k = D_k . v_rest, then
        (H v)_0 = <E> v_0 + sum_k w_k (E_k t_k + u_k)
        (H v)_i = sum_k w_k Oc_ki (E_k (v_0 + t_k) + u_k),  i >= 1.
    Used where H is too large to form."""
    O = np.asarray(O, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = sample_weights(O.shape[0], w)
    Oc = centred(O, w)
    t = Oc @ v[1:]
    u = D @ v[1:]
    y = np.empty(O.shape[1] + 1)
    y[0] = (w @ E) * v[0] + w @ (E * t + u)
    y[1:] = Oc.T @ (w * (E * (v[0] + t) + u))
    return y


def lm_lowest_eigenpair(H, S):
    """Lowest real eigenpair of H x = E S x (Eq. linear_eigen) by a dense generalized solve."""
    vals, vecs = sla.eig(H, S)
    vals = np.real_if_close(vals)
    finite = np.isfinite(vals)
    idx = np.where(finite)[0][np.argmin(np.real(vals[finite]))]
    return float(np.real(vals[idx])), np.real(vecs[:, idx])


# ----------------------------------------------------------------------------------------------
# Precision form: bf16 storage with a per-column float32 scale (not in the paper)
# ----------------------------------------------------------------------------------------------
def _f64_to_f32_round_to_odd(t: np.ndarray) -> np.ndarray:
    """float64 -> float32 bit patterns with round-to-odd (truncate, then set the last bit
    if anything was discarded).  Rounding to odd first and to nearest-even second gives the
    same bf16 value as one nearest-even rounding of the float64 value."""
    t = np.asarray(t, dtype=np.float64)
    f = t.astype(np.float32)                     # nearest-even
    fb = f.view(np.uint32).copy()
    back = f.astype(np.float64)
    # step toward zero where nearest rounded away from zero
    away = np.abs(back) > np.abs(t)
    fb[away] -= np.uint32(1)
    inexact = back != t
    fb[inexact] |= np.uint32(1)
    return fb


def quantize_bf16(O):
    """Per-column float32 scale s_j = max_k |O_kj| (1 for an all-zero column) and
    q_kj = round-to-nearest-even bf16 of O_kj / s_j (the quotient taken in float64).

    Returns (q as uint16 bit patterns, s as float32)."""
    O = np.asarray(O, dtype=np.float64)
    amax = np.abs(O).max(axis=0) if O.shape[0] else np.zeros(O.shape[1])
    s = amax.astype(np.float32)
    s[s == 0] = np.float32(1.0)
    t = O / s.astype(np.float64)[None, :]
    fb = _f64_to_f32_round_to_odd(t)
    rounded = (fb.astype(np.uint64) + np.uint64(0x7FFF) + ((fb.astype(np.uint64) >> np.uint64(16)) & np.uint64(1)))
    q = (rounded >> np.uint64(16)).astype(np.uint16)
    return q, s


def _rne_bf16_bits_from_f64(t: np.ndarray) -> np.ndarray:
    fb = _f64_to_f32_round_to_odd(t).astype(np.uint64)
    return ((fb + np.uint64(0x7FFF) + ((fb >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)).astype(np.uint16)


def _bf16_bits_to_f64(q: np.ndarray) -> np.ndarray:
    return (np.asarray(q, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def quantize_split(O, code: str = "bf16"):
    """Two-plane codes: q_hi as in quantize_bf16/_f16, and q_lo = nearest-even code of the
    remainder O_kj / s_j - q_hi_kj (in float64), so that s_j (q_hi + q_lo) represents O_kj
    to about 2^-18 (bf16) of the column scale.  Returns (q_hi, q_lo, s)."""
    O = np.asarray(O, dtype=np.float64)
    q_hi, s = quantize_bf16(O) if code == "bf16" else quantize_f16(O)
    t = O / s.astype(np.float64)[None, :]
    hi = _bf16_bits_to_f64(q_hi) if code == "bf16" else q_hi.view(np.float16).astype(np.float64)
    rem = t - hi
    if code == "bf16":
        q_lo = _rne_bf16_bits_from_f64(rem)
    else:
        q_lo = _f64_to_f32_round_to_odd(rem).view(np.float32).astype(np.float16).view(np.uint16)
    return q_hi, q_lo, s


def dequantize_split(q_hi, q_lo, s, code: str = "bf16") -> np.ndarray:
    """Stored value s_j (q_hi + q_lo) lifted to float64 (the sum taken in float64)."""
    if code == "bf16":
        v = _bf16_bits_to_f64(q_hi) + _bf16_bits_to_f64(q_lo)
    else:
        v = (np.asarray(q_hi, dtype=np.uint16).view(np.float16).astype(np.float64)
             + np.asarray(q_lo, dtype=np.uint16).view(np.float16).astype(np.float64))
    return v * np.asarray(s, dtype=np.float32).astype(np.float64)[None, :]


# Default selection bound of quantize_cols: the error bound of the two-plane codes relative
# to the column scale (bf16: the remainder is at most 2^-9 and its nearest bf16 code is
# within 2^-18 of it; f16: remainder at most 2^-12, code within 2^-22 even in the subnormal
# range of the remainder), with one bit of slack.
REMAINDER_TOL = {"bf16": 2.0 ** -17, "f16": 2.0 ** -21}


def quantize_cols(O, code: str = "bf16", tol: float | None = None):
    """Codes with the remainder plane kept only where it is needed.

    q_hi and s are those of quantize_bf16 / quantize_f16.  Column j gets a remainder code
    (the nearest code of O_kj / s_j - q_hi_kj, as in quantize_split) iff its single-plane
    error max_k |O_kj / s_j - q_hi_kj| (in float64) exceeds `tol` (default REMAINDER_TOL), so
    that every stored value is within max(tol, two-plane bound) s_j of O_kj.
    Returns (q_hi, s, lo_cols, q_lo): lo_cols the selected columns in increasing order
    (int64), q_lo their remainder codes, shape (n_s, len(lo_cols))."""
    O = np.asarray(O, dtype=np.float64)
    tol = REMAINDER_TOL[code] if tol is None else float(tol)
    q_hi, q_lo_full, s = quantize_split(O, code)
    t = O / s.astype(np.float64)[None, :]
    hi = _bf16_bits_to_f64(q_hi) if code == "bf16" else q_hi.view(np.float16).astype(np.float64)
    err = np.abs(t - hi).max(axis=0) if O.shape[0] else np.zeros(O.shape[1])
    lo_cols = np.nonzero(err > tol)[0].astype(np.int64)
    return q_hi, s, lo_cols, np.ascontiguousarray(q_lo_full[:, lo_cols])


def dequantize_cols(q_hi, s, lo_cols, q_lo, code: str = "bf16") -> np.ndarray:
    """Stored values of quantize_cols: s_j (q_hi_kj + q_lo_kj) for the columns j in lo_cols
    (the sum taken in float64), s_j q_hi_kj for the others."""
    if code == "bf16":
        v = _bf16_bits_to_f64(q_hi)
        lo = _bf16_bits_to_f64(q_lo)
    else:
        v = np.asarray(q_hi, dtype=np.uint16).view(np.float16).astype(np.float64)
        lo = np.asarray(q_lo, dtype=np.uint16).view(np.float16).astype(np.float64)
    v = v.copy()
    v[:, np.asarray(lo_cols, dtype=np.int64)] += lo
    return v * np.asarray(s, dtype=np.float32).astype(np.float64)[None, :]


def quantize_f16(O):
    """As quantize_bf16 but with float16 codes: q_kj = nearest-even float16 of O_kj / s_j
    (the quotient taken in float64).  Returns (q as uint16 bit patterns, s as float32)."""
    O = np.asarray(O, dtype=np.float64)
    amax = np.abs(O).max(axis=0) if O.shape[0] else np.zeros(O.shape[1])
    s = amax.astype(np.float32)
    s[s == 0] = np.float32(1.0)
    t = O / s.astype(np.float64)[None, :]
    f = _f64_to_f32_round_to_odd(t).view(np.float32)
    q = f.astype(np.float16).view(np.uint16)
    return q, s


def dequantize_f16(q, s) -> np.ndarray:
    """Stored value s_j * q_kj (float16 codes) lifted to float64."""
    f = np.asarray(q, dtype=np.uint16).view(np.float16).astype(np.float64)
    return f * np.asarray(s, dtype=np.float32).astype(np.float64)[None, :]


def dequantize_bf16(q, s) -> np.ndarray:
    """Stored value s_j * q_kj lifted to float64."""
    q = np.asarray(q, dtype=np.uint16)
    f = (q.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    return f * np.asarray(s, dtype=np.float32).astype(np.float64)[None, :]


# ----------------------------------------------------------------------------------------------
# Implicit-adjoint derivatives of the solve (not in the paper)
# ----------------------------------------------------------------------------------------------
def solve_adjoint_gradients(O, E, eps: float, dL_dx):
    """Derivatives of a scalar L(x) with x = (S + eps I)^{-1} g, g = energy_gradient(O, E).

    With lambda = (S + eps I)^{-1} dL/dx, p1 = Oc x, p2 = Oc lambda, e_c = E - <E> and
    uniform weights 1/N:
        dL/dO = (1/N) [ (2 e_c - p1) lambda^T - p2 x^T ],  dL/dE = (2/N) p2,
        dL/dg = lambda,  dL/deps = -lambda . x.
    Returns a dict with x, lam, dO, dE, dg, deps.
    """
    O = np.asarray(O, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    n_s = O.shape[0]
    g = energy_gradient(O, E)
    x = solve_dense(O, g, eps)
    lam = solve_dense(O, np.asarray(dL_dx, dtype=np.float64), eps)
    Oc = centred(O)
    ec = E - E.mean()
    p1 = Oc @ x
    p2 = Oc @ lam
    dO = (np.outer(2.0 * ec - p1, lam) - np.outer(p2, x)) / n_s
    dE = 2.0 * p2 / n_s
    return {"x": x, "lam": lam, "dO": dO, "dE": dE, "dg": lam, "deps": -float(lam @ x)}


def cps_expand(idx, val, n_states: int, dense=None) -> np.ndarray:
    """The N_s x N_p derivative-ratio matrix of a correlator-product state stored by index
    (Sec. II.C, Eq. ansatz).  A sample occupies one state of each correlator, so the ratio
    of correlator p's parameter for state s is val[p * n_states + s] when the sample is in
    state s and 0 otherwise.

    idx: (n_corr, N_s) integer states, correlator-major (a state >= n_states selects no
    column); val: (n_corr * n_states,) column values; dense: (N_s, n_d) the remaining
    parameters or None.  Columns: [correlator 0's states | correlator 1 | ... | dense].
    """
    idx = np.asarray(idx).astype(np.int64)
    val = np.asarray(val, dtype=np.float64)
    n_corr, n_s = idx.shape
    n_sp = n_corr * n_states
    n_d = 0 if dense is None else np.asarray(dense).shape[1]
    O = np.zeros((n_s, n_sp + n_d))
    for p in range(n_corr):
        rows = np.nonzero(idx[p] < n_states)[0]        # samples whose state of p is a column
        cols = p * n_states + idx[p, rows]
        O[rows, cols] = val[cols]
    if n_d:
        O[:, n_sp:] = np.asarray(dense, dtype=np.float64)
    return O
