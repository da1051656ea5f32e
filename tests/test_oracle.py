"""Pins of the FP64 CPU oracle against things other than itself.

Each test ties an oracle function to a library routine, a closed form, an invariant,
exact quantum mechanics in a tiny Hilbert space, finite differences, or a number the
paper prints, so that a dropped term, a wrong sign or index, a wrong normalisation or
a transposed operand fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import torch

import oracle as orc
import synth

pytestmark = []


def _rand(n_s, n_p, seed=0, offset=0.0):
    rng = np.random.default_rng(seed)
    s = np.exp(0.5 * rng.standard_normal(n_p))
    O = rng.standard_normal((n_s, n_p)) * s + offset
    E = -20.0 + O @ rng.standard_normal(n_p) * 0.3 / math.sqrt(n_p) + rng.standard_normal(n_s)
    return O, E


# ------------------------------------------------------------------------------------------
# Overlap matrix (Eq. sr_overlap, centred reading)
# ------------------------------------------------------------------------------------------
def test_overlap_matches_numpy_cov():
    """Library pin: the centred sampled overlap is the biased (1/N) covariance."""
    O, _ = _rand(57, 13, seed=1, offset=0.7)
    S = orc.overlap_matrix(O)
    np.testing.assert_allclose(S, np.cov(O, rowvar=False, bias=True), rtol=1e-12, atol=1e-13)


def test_overlap_symmetric_psd():
    O, _ = _rand(9, 20, seed=2)      # N_s < N_p: singular
    S = orc.overlap_matrix(O)
    assert np.array_equal(S, S.T) or np.allclose(S, S.T, rtol=0, atol=1e-15)
    ev = np.linalg.eigvalsh(S)
    assert ev.min() >= -1e-13 * np.abs(ev).max()
    # rank is at most N_s - 1 after centring
    assert (ev > 1e-10 * ev.max()).sum() <= 8


def test_overlap_invariances():
    """Row permutation, row duplication and a constant added to every row leave S and g fixed."""
    O, E = _rand(40, 7, seed=3)
    S, g = orc.overlap_matrix(O), orc.energy_gradient(O, E)
    perm = np.random.default_rng(0).permutation(40)
    np.testing.assert_allclose(orc.overlap_matrix(O[perm]), S, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(orc.energy_gradient(O[perm], E[perm]), g, rtol=1e-12, atol=1e-14)
    OO, EE = np.vstack([O, O]), np.concatenate([E, E])
    np.testing.assert_allclose(orc.overlap_matrix(OO), S, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(orc.energy_gradient(OO, EE), g, rtol=1e-12, atol=1e-14)
    shift = np.linspace(-3.0, 5.0, 7)
    np.testing.assert_allclose(orc.overlap_matrix(O + shift), S, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(orc.energy_gradient(O + shift, E), g, rtol=1e-10, atol=1e-12)
    # a constant added to the energies leaves g unchanged
    np.testing.assert_allclose(orc.energy_gradient(O, E + 123.0), g, rtol=1e-10, atol=1e-11)


def test_constant_column_gives_zero_row_and_zero_solution():
    O, E = _rand(30, 6, seed=4)
    O[:, 2] = 1.7
    S = orc.overlap_matrix(O)
    assert np.abs(S[2]).max() < 1e-14 and np.abs(S[:, 2]).max() < 1e-14
    g = orc.energy_gradient(O, E)
    assert abs(g[2]) < 1e-13
    x = orc.solve_dense(O, g, 1e-3)
    assert abs(x[2]) < 1e-12


def test_gradient_matches_numpy_cov():
    """Library pin: g = 2 cov(O, E) with the biased normalisation."""
    O, E = _rand(61, 9, seed=5)
    C = np.cov(np.vstack([O.T, E[None, :]]), bias=True)
    np.testing.assert_allclose(orc.energy_gradient(O, E), 2.0 * C[-1, :-1], rtol=1e-11, atol=1e-12)


def test_diag_overlap():
    O, _ = _rand(33, 11, seed=6, offset=100.0)     # large offset: catches sum(O^2) - N mean^2
    d = orc.diag_overlap(O)
    np.testing.assert_allclose(d, np.var(O, axis=0), rtol=1e-9)


# ------------------------------------------------------------------------------------------
# Products (Eqs. sr_multiply_1, sr_multiply_2)
# ------------------------------------------------------------------------------------------
def test_swapped_product_equals_explicit():
    O, _ = _rand(45, 17, seed=7, offset=0.3)
    v = np.random.default_rng(1).standard_normal(17)
    np.testing.assert_allclose(orc.sv_product_swapped(O, v, 0.25), orc.sv_product_dense(O, v, 0.25),
                               rtol=1e-12, atol=1e-13)


def test_cps_gauge_null_vectors():
    """For each correlator p, the vector c_{p,.} on its columns is a null vector of S."""
    d = synth.small_cps_inputs(seed=3, n_s=500, n_corr=4, n_states=8, n_dense=5)
    O = d["O"].numpy()
    c = d["c"].numpy()
    S = orc.overlap_matrix(O)
    for p in range(c.shape[0]):
        u = np.zeros(O.shape[1])
        u[p * 8:(p + 1) * 8] = c[p]
        assert np.abs(S @ u).max() < 1e-13 * np.abs(S).max() * np.abs(u).max() * 10
        np.testing.assert_allclose(orc.sv_product_dense(O, u, 0.5), 0.5 * u, rtol=0, atol=1e-12)


def test_cps_expand_reproduces_the_scattered_matrix():
    """The index-coded form of the CPS generator expands to exactly the matrix the generator
    builds by scattering 1/c into the dense O (same seed), and its energies agree to
    rounding."""
    args = dict(n_s=301, n_corr=5, n_states=7, n_dense=11, seed=3)
    ref = synth.cps_inputs(args["n_s"], args["n_corr"], args["n_states"], args["n_dense"], args["seed"])
    ix = synth.cps_index_inputs(args["n_s"], args["n_corr"], args["n_states"], args["n_dense"], args["seed"])
    O = orc.cps_expand(ix["idx"].numpy(), ix["val"].numpy(), 7, ix["dense"].numpy())
    np.testing.assert_array_equal(O, ref["O"].numpy())
    np.testing.assert_allclose(ix["E"].numpy(), ref["E"].numpy(), rtol=1e-14, atol=0)
    np.testing.assert_array_equal(ix["idx"].numpy().T, ref["state"].numpy())


def test_cps_expand_structure_and_ignored_states():
    """One nonzero per correlator per sample, equal to the column's value; a state outside
    the correlator's columns leaves its block empty; the dense block follows unchanged."""
    rng = np.random.default_rng(4)
    n_corr, n_s, ns = 3, 40, 5
    idx = rng.integers(0, ns, size=(n_corr, n_s))
    idx[1, 7] = 200                                   # no column
    val = 1.0 + rng.random(n_corr * ns)
    dense = rng.standard_normal((n_s, 4))
    O = orc.cps_expand(idx, val, ns, dense)
    assert O.shape == (n_s, n_corr * ns + 4)
    for p in range(n_corr):
        blk = O[:, p * ns:(p + 1) * ns]
        for k in range(n_s):
            nz = np.nonzero(blk[k])[0]
            if idx[p, k] < ns:
                assert list(nz) == [idx[p, k]] and blk[k, idx[p, k]] == val[p * ns + idx[p, k]]
            else:
                assert len(nz) == 0
    np.testing.assert_array_equal(O[:, n_corr * ns:], dense)


def test_cps_column_statistics_closed_form():
    """A correlator column is val times an indicator, so its mean is val f and its variance
    the Bernoulli variance val^2 f (1 - f), f the fraction of samples in the state (checks
    the oracle's centred statistics on the expanded matrix)."""
    ix = synth.cps_index_inputs(500, 4, 6, 3, 9)
    idx, val = ix["idx"].numpy(), ix["val"].numpy()
    O = orc.cps_expand(idx, val, 6, ix["dense"].numpy())
    f = np.array([[np.mean(idx[p] == s) for s in range(6)] for p in range(4)]).reshape(-1)
    np.testing.assert_allclose(orc.sample_mean(O)[:24], val * f, rtol=1e-13, atol=0)
    np.testing.assert_allclose(orc.diag_overlap(O)[:24], val ** 2 * f * (1 - f), rtol=1e-12, atol=1e-15)
    E = ix["E"].numpy()
    ec = E - E.mean()
    gs = np.array([2.0 / 500 * val[p * 6 + s] * ec[idx[p] == s].sum() for p in range(4) for s in range(6)])
    np.testing.assert_allclose(orc.energy_gradient(O, E)[:24], gs, rtol=1e-10, atol=1e-12)


def test_cps_expand_gauge_null_vectors():
    """Each correlator's vector c_{p,.} (the inverse values) is a null vector of S of the
    expanded matrix: every sample holds exactly one state of every correlator."""
    ix = synth.cps_index_inputs(400, 3, 9, 4, 21)
    O = orc.cps_expand(ix["idx"].numpy(), ix["val"].numpy(), 9, ix["dense"].numpy())
    c = ix["c"].numpy()
    for p in range(3):
        u = np.zeros(O.shape[1])
        u[p * 9:(p + 1) * 9] = c[p]
        np.testing.assert_allclose(orc.sv_product_swapped(O, u, 0.0), 0.0, atol=1e-13)


# ------------------------------------------------------------------------------------------
# Exact quantum mechanics in a tiny Hilbert space
# ------------------------------------------------------------------------------------------
def _tiny_space(M=7, P=3, seed=11):
    """Real wavefunction Psi(alpha) in an M-dimensional space, with P parameters."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((M, M))
    H = 0.5 * (A + A.T)
    psi0 = 1.0 + rng.random(M)                         # nodeless, no zero amplitudes
    B = rng.standard_normal((M, P)) * 0.3
    C2 = rng.standard_normal((M, P)) * 0.1

    def psi(alpha):                                    # nonlinear in alpha
        return psi0 + B @ alpha + C2 @ (alpha ** 2)

    def dpsi(alpha):                                   # columns d Psi / d alpha_i
        return B + C2 * (2.0 * alpha)[None, :]

    return H, psi, dpsi


def _sampled_from_enumeration(H, psi, dpsi, alpha):
    """Per-configuration ratios with exact weights |Psi_n|^2 / <Psi|Psi>."""
    P0 = psi(alpha)
    dP = dpsi(alpha)
    w = P0 ** 2 / (P0 @ P0)
    O = dP / P0[:, None]
    E = (H @ P0) / P0
    D = (H @ dP) / P0[:, None] - E[:, None] * O        # d E_L / d alpha_j
    return O, E, D, w


def test_overlap_and_gradient_exact_enumeration():
    H, psi, dpsi = _tiny_space()
    alpha = np.array([0.2, -0.1, 0.3])
    O, E, _, w = _sampled_from_enumeration(H, psi, dpsi, alpha)
    P0, dP = psi(alpha), dpsi(alpha)
    nrm = P0 @ P0
    mean = (P0 @ dP) / nrm
    bar = dP - np.outer(P0, mean)                      # Psi^i - <O_i> Psi
    np.testing.assert_allclose(orc.overlap_matrix(O, w), bar.T @ bar / nrm, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(orc.energy_mean(E, w), P0 @ H @ P0 / nrm, rtol=1e-13)

    # g is the gradient of the Rayleigh quotient E(alpha) (central differences)
    def energy(a):
        p = psi(a)
        return p @ H @ p / (p @ p)
    h = 1e-6
    fd = np.array([(energy(alpha + h * e) - energy(alpha - h * e)) / (2 * h) for e in np.eye(3)])
    np.testing.assert_allclose(orc.energy_gradient(O, E, w), fd, rtol=1e-7, atol=1e-9)


def test_lm_matrices_exact_enumeration():
    """H and S of the linear method equal the exact matrices in {Psi, Psi^i - <O_i> Psi}."""
    H, psi, dpsi = _tiny_space()
    alpha = np.array([-0.3, 0.05, 0.2])
    O, E, D, w = _sampled_from_enumeration(H, psi, dpsi, alpha)
    P0, dP = psi(alpha), dpsi(alpha)
    nrm = P0 @ P0
    bar = dP - np.outer(P0, (P0 @ dP) / nrm)
    basis = np.concatenate([P0[:, None], bar], axis=1)
    Hx = basis.T @ H @ basis / nrm
    Sx = basis.T @ basis / nrm
    Hs, Ss = orc.lm_matrices(O, E, D, w)
    np.testing.assert_allclose(Hs, Hx, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(Ss, Sx, rtol=1e-11, atol=1e-13)
    # H_i0 = g_i / 2
    np.testing.assert_allclose(Hs[1:, 0], orc.energy_gradient(O, E, w) / 2, rtol=1e-12, atol=1e-13)
    v = np.random.default_rng(2).standard_normal(4)
    np.testing.assert_allclose(orc.lm_hv_dense(O, E, D, v, w), Hx @ v, rtol=1e-11, atol=1e-12)


def test_lm_matrix_free_product_equals_dense():
    """The matrix-free H v equals H v with H formed (weighted and uniform samples)."""
    rng = np.random.default_rng(17)
    O = rng.standard_normal((40, 7)) + 0.3
    E = rng.standard_normal(40) - 2.0
    D = 0.1 * rng.standard_normal((40, 7))
    v = rng.standard_normal(8)
    for w in (None, rng.random(40)):
        np.testing.assert_allclose(orc.lm_hv_swapped(O, E, D, v, w), orc.lm_hv_dense(O, E, D, v, w),
                                   rtol=1e-12, atol=1e-13)


def test_lm_eigenvalue_variational_and_exact_when_complete():
    """Lowest LM eigenvalue >= ground-state energy; equal when Omega spans the whole space."""
    H, psi, dpsi = _tiny_space(M=4, P=3, seed=5)       # 1 + 3 = 4 = M: Omega is complete
    alpha = np.array([0.1, 0.2, -0.1])
    O, E, D, w = _sampled_from_enumeration(H, psi, dpsi, alpha)
    Hs, Ss = orc.lm_matrices(O, E, D, w)
    e, _ = orc.lm_lowest_eigenpair(Hs, Ss)
    np.testing.assert_allclose(e, np.linalg.eigvalsh(H)[0], rtol=1e-10)
    H5, psi5, dpsi5 = _tiny_space(M=6, P=2, seed=6)    # incomplete subspace
    O, E, D, w = _sampled_from_enumeration(H5, psi5, dpsi5, np.array([0.1, 0.0]))
    e5, _ = orc.lm_lowest_eigenpair(*orc.lm_matrices(O, E, D, w))
    assert e5 >= np.linalg.eigvalsh(H5)[0] - 1e-12
    assert e5 <= orc.energy_mean(E, w) + 1e-12


def test_lm_constant_energy_closed_form():
    """D = 0 and E = E0 everywhere: H_00 = E0, H_i0 = H_0j = 0, H_block = E0 S."""
    O, _ = _rand(50, 6, seed=8)
    E = np.full(50, -3.5)
    H, S = orc.lm_matrices(O, E, np.zeros_like(O))
    assert abs(H[0, 0] + 3.5) < 1e-14
    assert np.abs(H[1:, 0]).max() < 1e-13 and np.abs(H[0, 1:]).max() < 1e-13
    np.testing.assert_allclose(H[1:, 1:], -3.5 * S[1:, 1:], rtol=1e-12, atol=1e-13)


def test_paper_system_projection_exact_enumeration():
    """Eq. sr_lin_eq is the orthogonal projection of (1 - tau H) Psi onto Omega."""
    H, psi, dpsi = _tiny_space(M=8, P=3, seed=9)
    alpha = np.array([0.0, 0.1, -0.2])
    O, E, _, w = _sampled_from_enumeration(H, psi, dpsi, alpha)
    tau = 0.05
    A, b = orc.paper_linear_system(O, E, tau, w)
    x = np.linalg.solve(A, b)
    P0, dP = psi(alpha), dpsi(alpha)
    basis = np.concatenate([P0[:, None], dP], axis=1)
    target = P0 - tau * (H @ P0)
    resid = target - basis @ x
    assert np.abs(basis.T @ resid).max() < 1e-12 * np.abs(target).max()


def test_sr_update_linear_ansatz_reproduces_projection():
    """For a wavefunction linear in its parameters, Psi(alpha) = psi0 + B alpha, the
    projected vector sum_j x_j Psi^j of Eq. sr_lin_eq equals x_0 Psi(alpha') exactly,
    with alpha' = alpha + x_i / x_0 (Sec. II.A): the update moves Psi to the projection."""
    rng = np.random.default_rng(90)
    M, P = 9, 4
    A = rng.standard_normal((M, M))
    H = 0.5 * (A + A.T)
    psi0 = 1.0 + rng.random(M)
    B = 0.3 * rng.standard_normal((M, P))
    alpha = np.array([0.2, -0.1, 0.05, 0.3])
    P0 = psi0 + B @ alpha
    O = B / P0[:, None]
    E = (H @ P0) / P0
    w = P0 ** 2 / (P0 @ P0)
    for tau in (0.01, 0.2):
        Asys, b = orc.paper_linear_system(O, E, tau, w)
        x = np.linalg.solve(Asys, b)
        projected = x[0] * P0 + B @ x[1:]
        a_new = orc.sr_update(alpha, x)
        np.testing.assert_allclose(x[0] * (psi0 + B @ a_new), projected, rtol=1e-12, atol=1e-13)
        # and the projection is the least-squares fit of (1 - tau H) Psi in the span
        basis = np.concatenate([P0[:, None], B], axis=1)
        c = np.linalg.lstsq(basis, P0 - tau * (H @ P0), rcond=None)[0]
        np.testing.assert_allclose(projected, basis @ c, rtol=1e-10, atol=1e-12)


def test_lm_eigenvector_is_the_ground_state_when_complete():
    """With Omega spanning the whole space, the lowest LM eigenvector c gives the exact
    ground state: sum_i c_i Psi_bar^i is proportional to the lowest eigenvector of H."""
    H, psi, dpsi = _tiny_space(M=4, P=3, seed=5)
    alpha = np.array([0.1, 0.2, -0.1])
    O, E, D, w = _sampled_from_enumeration(H, psi, dpsi, alpha)
    _, c = orc.lm_lowest_eigenpair(*orc.lm_matrices(O, E, D, w))
    P0, dP = psi(alpha), dpsi(alpha)
    bar = dP - np.outer(P0, (P0 @ dP) / (P0 @ P0))
    phi = np.concatenate([P0[:, None], bar], axis=1) @ c
    gs = np.linalg.eigh(H)[1][:, 0]
    cosang = abs(phi @ gs) / np.linalg.norm(phi)
    assert cosang == pytest.approx(1.0, abs=1e-12)


def test_centred_system_equals_paper_system():
    """R1 reading: eliminating x_0 from the (N_p+1) system gives S_c x = -(tau/2) g."""
    O, E = _rand(200, 9, seed=10, offset=0.4)
    tau = 0.01
    A, b = orc.paper_linear_system(O, E, tau)
    x = np.linalg.solve(A, b)
    S = orc.overlap_matrix(O)
    g = orc.energy_gradient(O, E)
    xc = np.linalg.solve(S, -0.5 * tau * g)
    np.testing.assert_allclose(x[1:], xc, rtol=1e-9, atol=1e-12)
    x0 = 1.0 - tau * E.mean() - orc.sample_mean(O) @ xc
    np.testing.assert_allclose(x[0], x0, rtol=1e-10)


# ------------------------------------------------------------------------------------------
# Solves
# ------------------------------------------------------------------------------------------
def test_solve_dense_library_and_woodbury():
    O, E = _rand(25, 40, seed=12)      # N_s < N_p: Woodbury dual form applies
    g = orc.energy_gradient(O, E)
    eps = 0.07
    x = orc.solve_dense(O, g, eps)
    S = np.cov(O, rowvar=False, bias=True)
    np.testing.assert_allclose(x, sla.solve(S + eps * np.eye(40), g, assume_a="pos"), rtol=1e-10)
    Oc = O - O.mean(0)
    n = O.shape[0]
    dual = (g - Oc.T @ np.linalg.solve(n * eps * np.eye(n) + Oc @ Oc.T, Oc @ g)) / eps
    np.testing.assert_allclose(x, dual, rtol=1e-9, atol=1e-12)
    # the oracle's dual solve (uniform and non-uniform weights) equals the Cholesky solve
    np.testing.assert_allclose(orc.solve_dual(O, g, eps), x, rtol=1e-9, atol=1e-12)
    wts = np.random.default_rng(4).random(25)
    wts /= wts.sum()
    np.testing.assert_allclose(orc.solve_dual(O, g, eps, wts), orc.solve_dense(O, g, eps, wts), rtol=1e-9,
                               atol=1e-12)


def test_solve_sherman_morrison_two_samples():
    """N_s = 2: S = d d^T / 4 with d = O_1 - O_2, so x = (g - d (d.g)/(4 eps + d.d)) / eps."""
    rng = np.random.default_rng(13)
    O = rng.standard_normal((2, 6))
    g = rng.standard_normal(6)
    eps = 0.3
    d = O[0] - O[1]
    closed = (g - d * (d @ g) / (4 * eps + d @ d)) / eps
    np.testing.assert_allclose(orc.solve_dense(O, g, eps), closed, rtol=1e-12)


def test_solve_eps_zero_is_min_norm():
    O, E = _rand(6, 15, seed=14)
    g = orc.energy_gradient(O, E)
    x = orc.solve_dense(O, g, 0.0)
    S = np.cov(O, rowvar=False, bias=True)
    xl = np.linalg.lstsq(S, g, rcond=1e-12)[0]
    np.testing.assert_allclose(x, xl, rtol=1e-8, atol=1e-10)


def test_cg_matches_dense_and_terminates_in_rank_steps():
    O, E = _rand(6, 15, seed=15)        # rank(S) <= 5
    g = orc.energy_gradient(O, E)
    x, it, rel = orc.cg_solve(lambda v: orc.sv_product_dense(O, v, 0.0), g, rtol=1e-12)
    assert it <= 6
    np.testing.assert_allclose(x, orc.solve_dense(O, g, 0.0), rtol=1e-8, atol=1e-10)
    O, E = _rand(300, 40, seed=16)
    g = orc.energy_gradient(O, E)
    eps = 1e-2
    for m in (0, 7):
        x, it, rel = orc.cg_solve(lambda v: orc.sv_product_swapped(O, v, eps), g, rtol=1e-13, refresh_every=m)
        assert rel <= 1e-13
        xd = orc.solve_dense(O, g, eps)
        assert np.linalg.norm(x - xd) <= 1e-11 * np.linalg.norm(xd)


def test_cg_warm_start():
    O, E = _rand(100, 20, seed=17)
    g = orc.energy_gradient(O, E)
    xs = orc.solve_dense(O, g, 0.1)
    x, it, _ = orc.cg_solve(lambda v: orc.sv_product_dense(O, v, 0.1), g, rtol=1e-12, x0=xs)
    assert it <= 1
    np.testing.assert_allclose(x, xs, rtol=1e-10)


# ------------------------------------------------------------------------------------------
# bf16 storage
# ------------------------------------------------------------------------------------------
def _nearest_bf16_fraction(t: float) -> float:
    """Nearest bf16 value to the float64 t by exact rational arithmetic, ties to even."""
    if t == 0.0:
        return 0.0
    sgn = -1.0 if t < 0 else 1.0
    a = Fraction(abs(t))
    e = math.floor(math.log2(abs(t)))
    if Fraction(2) ** e > a:
        e -= 1
    if Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -126)
    ulp = Fraction(2) ** (e - 7)
    lo = (a // ulp) * ulp
    hi = lo + ulp
    if a - lo < hi - a:
        r = lo
    elif a - lo > hi - a:
        r = hi
    else:
        r = lo if (lo / ulp) % 2 == 0 else hi
    return sgn * float(r)


def test_quantize_bf16_nearest_even_exact():
    rng = np.random.default_rng(20)
    O = rng.standard_normal((64, 9)) * np.exp(rng.standard_normal(9))
    O[3, 4] = 0.0
    # plant exact ties of the quotient: s is a power of two in column 0
    O[:, 0] = 0.0
    O[0, 0] = 2.0
    O[1, 0] = 2.0 * (1 + 2 ** -8 + 2 ** -9)       # halfway -> rounds to even (up)
    O[2, 0] = 2.0 * (1 + 2 ** -9) / 2             # halfway below 1 -> even (down)
    q, s = orc.quantize_bf16(O)
    deq = orc.dequantize_bf16(q, s)
    for k in range(O.shape[0]):
        for j in range(O.shape[1]):
            t = O[k, j] / float(s[j])
            assert deq[k, j] / float(s[j]) == _nearest_bf16_fraction(t), (k, j)
    # error bound: |stored - O| <= 2^-9 s_j
    assert np.all(np.abs(deq - O) <= 2.0 ** -9 * s.astype(np.float64)[None, :] * (1 + 1e-12))


def test_quantize_bf16_matches_torch_on_float32_exact_quotients():
    """Library pin: torch's float32 -> bfloat16 conversion rounds to nearest even."""
    rng = np.random.default_rng(21)
    O = rng.standard_normal((200, 5)).astype(np.float32).astype(np.float64)
    s_pow2 = 2.0 ** np.ceil(np.log2(np.abs(O).max(0)))
    O[0] = s_pow2          # make the column max a power of two, so O / s is exact in float32
    q, s = orc.quantize_bf16(O)
    t = torch.from_numpy((O / s.astype(np.float64)).astype(np.float32))
    ref = t.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(q, ref)


def test_quantize_cps_columns_exact_and_zero_column():
    d = synth.small_cps_inputs(seed=4, n_s=300, n_corr=3, n_states=8, n_dense=4)
    O = d["O"].numpy()
    O[:, -1] = 0.0
    q, s = orc.quantize_bf16(O)
    deq = orc.dequantize_bf16(q, s)
    nz = O[:, :24] != 0
    assert np.all(q[:, :24][nz] == 0x3F80)            # 1.0 in bf16
    np.testing.assert_allclose(deq[:, :24], O[:, :24], rtol=2.0 ** -24)
    assert s[-1] == 1.0 and np.all(q[:, -1] == 0)


def _nearest_f16_fraction(t: float) -> float:
    """Nearest float16 value to t by exact rational arithmetic, ties to even."""
    if t == 0.0:
        return 0.0
    sgn = -1.0 if t < 0 else 1.0
    a = Fraction(abs(t))
    e = math.floor(math.log2(abs(t)))
    if Fraction(2) ** e > a:
        e -= 1
    if Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, -14)
    ulp = Fraction(2) ** (e - 10)
    lo = (a // ulp) * ulp
    hi = lo + ulp
    if a - lo < hi - a:
        r = lo
    elif a - lo > hi - a:
        r = hi
    else:
        r = lo if (lo / ulp) % 2 == 0 else hi
    return sgn * float(r)


def test_quantize_f16_nearest_even_exact():
    rng = np.random.default_rng(22)
    O = rng.standard_normal((48, 7)) * np.exp(rng.standard_normal(7))
    O[5, 1] = 1e-9 * O[:, 1].max()          # float16 subnormal range of the quotient
    q, s = orc.quantize_f16(O)
    deq = orc.dequantize_f16(q, s)
    for k in range(O.shape[0]):
        for j in range(O.shape[1]):
            t = O[k, j] / float(s[j])
            assert deq[k, j] / float(s[j]) == _nearest_f16_fraction(t), (k, j)
    assert np.all(np.abs(deq - O) <= 2.0 ** -12 * s.astype(np.float64)[None, :] * (1 + 1e-12))
    # library pin: torch float32 -> float16 on float32-exact quotients
    O2 = rng.standard_normal((100, 4)).astype(np.float32).astype(np.float64)
    O2[0] = 2.0 ** np.ceil(np.log2(np.abs(O2).max(0)))
    q2, s2 = orc.quantize_f16(O2)
    ref = torch.from_numpy((O2 / s2.astype(np.float64)).astype(np.float32)).to(torch.float16)
    assert np.array_equal(q2, ref.view(torch.int16).numpy().view(np.uint16))


def test_quantize_split_two_planes():
    """hi + lo planes: the lo code is the nearest code of the remainder, so the stored value
    is within half a lo-ulp of O (about 2^-18 of the column scale for bf16, 2^-22 for f16)."""
    rng = np.random.default_rng(23)
    O = rng.standard_normal((40, 6)) * np.exp(rng.standard_normal(6))
    O[:, 2] = 0.0
    for code, nearest, bound in (("bf16", _nearest_bf16_fraction, 2.0 ** -17), ("f16", _nearest_f16_fraction, 2.0 ** -21)):
        hi, lo, s = orc.quantize_split(O, code)
        ref_hi, ref_s = (orc.quantize_bf16 if code == "bf16" else orc.quantize_f16)(O)
        assert np.array_equal(hi, ref_hi) and np.array_equal(s, ref_s)
        deq = orc.dequantize_split(hi, lo, s, code)
        assert np.all(np.abs(deq - O) <= bound * s.astype(np.float64)[None, :])
        # lo is the nearest code of the exact remainder (brute force on a few entries)
        deq_hi = (orc.dequantize_bf16(hi, s) if code == "bf16" else orc.dequantize_f16(hi, s))
        for (k, j) in [(0, 0), (5, 1), (17, 3), (39, 5)]:
            rem = O[k, j] / float(s[j]) - deq_hi[k, j] / float(s[j])
            assert (deq[k, j] - deq_hi[k, j]) / float(s[j]) == nearest(rem)
        assert np.all(lo[:, 2] == 0)


def test_quantize_cols_selects_exactly_the_columns_that_need_a_remainder():
    """Compact remainder plane on a CPS-shaped matrix with dense pairing columns: the CPS
    columns hold one value per column (1/c), so their single-plane codes are exact up to the
    float32 rounding of the scale (2^-24) and need no remainder; the dense columns do.  The
    stored values then meet the two-plane error bound everywhere."""
    d = synth.small_cps_inputs(seed=8, n_s=400, n_corr=3, n_states=8, n_dense=7)
    O = d["O"].numpy()
    n_sparse = 24
    for code, nearest, bound in (("bf16", _nearest_bf16_fraction, 2.0 ** -17),
                                 ("f16", _nearest_f16_fraction, 2.0 ** -21)):
        q_hi, s, lo_cols, q_lo = orc.quantize_cols(O, code)
        assert np.array_equal(lo_cols, np.arange(n_sparse, O.shape[1]))
        assert q_lo.shape == (O.shape[0], O.shape[1] - n_sparse)
        deq = orc.dequantize_cols(q_hi, s, lo_cols, q_lo, code)
        assert np.all(np.abs(deq - O) <= bound * s.astype(np.float64)[None, :])
        # every selected column's single-plane error exceeds the bound (computed entry by
        # entry with exact rational rounding), every other column's stays within it
        for j in range(O.shape[1]):
            err = max(abs(O[k, j] / float(s[j]) - nearest(O[k, j] / float(s[j]))) for k in range(0, O.shape[0], 7))
            if j < n_sparse:
                assert err <= 2.0 ** -23, (code, j, err)
            else:
                assert err > bound, (code, j, err)
        # the remainder codes are the nearest codes of the remainder
        for (k, jj) in [(0, 0), (13, 2), (399, 6)]:
            j = int(lo_cols[jj])
            hi = nearest(O[k, j] / float(s[j]))
            rem = O[k, j] / float(s[j]) - hi
            assert (deq[k, j] / float(s[j])) - hi == nearest(rem)


def test_quantize_cols_limits_equal_one_and_two_planes():
    """tol < 0 keeps a remainder for every column (the two-plane values); tol = inf for none
    (the single-plane values)."""
    rng = np.random.default_rng(24)
    O = rng.standard_normal((30, 9)) * np.exp(rng.standard_normal(9))
    O[:, 4] = 0.0
    for code in ("bf16", "f16"):
        q_hi, s, cols, q_lo = orc.quantize_cols(O, code, tol=-1.0)
        assert np.array_equal(cols, np.arange(9))
        np.testing.assert_array_equal(orc.dequantize_cols(q_hi, s, cols, q_lo, code),
                                      orc.dequantize_split(*orc.quantize_split(O, code), code))
        q_hi, s, cols, q_lo = orc.quantize_cols(O, code, tol=np.inf)
        assert cols.size == 0 and q_lo.shape == (30, 0)
        one = orc.dequantize_bf16(*orc.quantize_bf16(O)) if code == "bf16" else orc.dequantize_f16(*orc.quantize_f16(O))
        np.testing.assert_array_equal(orc.dequantize_cols(q_hi, s, cols, q_lo, code), one)


# ------------------------------------------------------------------------------------------
# Adjoint derivatives
# ------------------------------------------------------------------------------------------
def test_adjoint_gradients_finite_difference():
    O, E = _rand(12, 5, seed=30)
    eps = 0.05
    wv = np.random.default_rng(31).standard_normal(5)
    res = orc.solve_adjoint_gradients(O, E, eps, wv)

    def loss(O_, E_, eps_=eps):
        return wv @ orc.solve_dense(O_, orc.energy_gradient(O_, E_), eps_)
    h = 1e-5
    for (k, j) in [(0, 0), (3, 2), (11, 4), (7, 1)]:
        Op, Om = O.copy(), O.copy()
        Op[k, j] += h
        Om[k, j] -= h
        fd = (loss(Op, E) - loss(Om, E)) / (2 * h)
        assert abs(fd - res["dO"][k, j]) <= 1e-7 * max(1.0, abs(fd))
    for k in (0, 5, 11):
        Ep, Em = E.copy(), E.copy()
        Ep[k] += h
        Em[k] -= h
        fd = (loss(O, Ep) - loss(O, Em)) / (2 * h)
        assert abs(fd - res["dE"][k]) <= 1e-7 * max(1.0, abs(fd))
    fd = (loss(O, E, eps + h) - loss(O, E, eps - h)) / (2 * h)
    assert abs(fd - res["deps"]) <= 1e-7 * max(1.0, abs(fd))


def test_adjoint_gradients_torch_autograd():
    """Library pin: torch autograd through torch.linalg.solve (CPU, float64)."""
    O, E = _rand(20, 6, seed=32)
    eps = 0.02
    wv = np.random.default_rng(33).standard_normal(6)
    res = orc.solve_adjoint_gradients(O, E, eps, wv)
    Ot = torch.tensor(O, requires_grad=True)
    Et = torch.tensor(E, requires_grad=True)
    Oc = Ot - Ot.mean(0)
    S = Oc.T @ Oc / 20
    g = 2 * Oc.T @ (Et - Et.mean()) / 20
    x = torch.linalg.solve(S + eps * torch.eye(6, dtype=torch.float64), g)
    (torch.tensor(wv) @ x).backward()
    np.testing.assert_allclose(res["dO"], Ot.grad.numpy(), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(res["dE"], Et.grad.numpy(), rtol=1e-9, atol=1e-12)


# ------------------------------------------------------------------------------------------
# Parameter counts printed in the paper
# ------------------------------------------------------------------------------------------
def _golden_counts():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "param_counts.txt")
    out = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, count = line.split()[:2]
        out[name] = int(count)
    return out


def test_layout_reproduces_paper_parameter_counts():
    gold = _golden_counts()
    assert synth.hubbard_4x4_layout().n_params == gold["hubbard_4x4"]
    assert synth.hydrogen_4x4_layout().n_params == gold["hydrogen_4x4"]
    lay = synth.hubbard_8x8_plaquette_layout()
    assert len(lay.correlators) == 64 and lay.n_correlator_params == 64 * 256
    assert lay.n_pairing_params == 8128
