"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these tests retypes an oracle formula: each checks a consequence that
a dropped term, a wrong sign, a wrong index or a transposed operand would
violate (gamma algebra, gamma5-hermiticity, the free-field momentum-space
operator, gauge covariance, adjoint pairs written out independently, dense
linear algebra on a 2^4 lattice, the block-triangular structure of Sec. 4 and
its 4D effective operator, finite differences of the action).
"""
import numpy as np
import pytest
import scipy.linalg

import synth


def vdot(a, b):
    return np.vdot(np.ravel(a), np.ravel(b))


def spin(M, psi):
    """apply a 4x4 spin matrix to a field [..., spin, colour]"""
    return np.einsum("ab,...bc->...ac", M, psi)


def grid(dims):
    X, Y, Z, T = dims
    return np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")


# --------------------------------------------------------------------- gamma algebra
def test_gamma_algebra(ora):
    g = ora.gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2.0 * (mu == nu) * np.eye(4))
        assert np.allclose(g[4] @ g[mu] + g[mu] @ g[4], 0)
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))


def test_generators(ora):
    T = ora.generators()
    for a in range(8):
        assert np.allclose(T[a], -T[a].conj().T)          # anti-Hermitian
        assert abs(np.trace(T[a])) < 1e-15               # traceless
        for b in range(8):
            assert abs(np.trace(T[a] @ T[b]) + 0.5 * (a == b)) < 1e-14
    # [T_1, T_2] = -T_3 for T = i lambda/2 (f_123 = 1)
    assert np.allclose(T[0] @ T[1] - T[1] @ T[0], -T[2])


# --------------------------------------------------------------------- Wilson operator
def test_wilson_gamma5_hermiticity(ora):
    dims = (4, 4, 2, 6)
    p = ora.params(dims, 1, M5=1.8)
    U = synth.random_links(dims, 0.5, 11)
    x = synth.gaussian_spinor(dims, 1, 12)[0]
    y = synth.gaussian_spinor(dims, 1, 13)[0]
    g5 = ora.gammas()[4]
    lhs = vdot(x, spin(g5, ora.dw4(p, U, spin(g5, y))))
    rhs = vdot(ora.dw4(p, U, x), y)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)
    # the written-out adjoint equals gamma5 D_W gamma5
    d1 = ora.dw4(p, U, y, dagger=True)
    d2 = spin(g5, ora.dw4(p, U, spin(g5, y)))
    assert np.max(np.abs(d1 - d2)) < 1e-12


@pytest.mark.parametrize("dims,tbc", [((4, 6, 4, 8), 0), ((4, 6, 4, 8), 1), ((2, 2, 2, 2), 0),
                                      ((2, 4, 2, 4), 1)])
def test_free_field_momentum_space(ora, dims, tbc):
    """Unit links: a plane wave e^{ip.x} chi is an eigenvector of the hop; D_W(p) =
    -M5 + sum(1 - cos p) + i sum gamma_mu sin p_mu.  Extent-2 directions check that both
    neighbour terms are accumulated when x+mu = x-mu."""
    X, Y, Z, T = dims
    M5 = 1.8
    p = ora.params(dims, 1, M5=M5, tbc=tbc)
    U = synth.unit_links(dims)
    g = ora.gammas()
    t, z, y, x = grid(dims)
    rng = np.random.default_rng(5)
    for _ in range(4):
        n = rng.integers(0, [X, Y, Z, T])
        k = 2 * np.pi * n / np.array(dims, float)
        if tbc:
            k[3] = (2 * n[3] + 1) * np.pi / T
        chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (k[0] * x + k[1] * y + k[2] * z + k[3] * t))
        psi = phase[..., None, None] * chi
        Dp = (-M5 + np.sum(1 - np.cos(k))) * np.eye(4) + 1j * sum(g[m] * np.sin(k[m]) for m in range(4))
        expect = phase[..., None, None] * (Dp @ chi)
        assert np.max(np.abs(ora.dw4(p, U, psi) - expect)) < 1e-12


def gauge_transform(U, G):
    """U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dag in the (mu, t, z, y, x) layout."""
    UG = np.empty_like(U)
    for mu in range(4):
        ax = 3 - mu
        Gf = np.roll(G, -1, axis=ax)
        UG[mu] = G @ U[mu] @ np.conj(np.swapaxes(Gf, -1, -2))
    return UG


@pytest.mark.parametrize("bc,tbc", [((1.0, 0.0), 0), ((1.5, 0.5), 1)])
def test_gauge_covariance(ora, bc, tbc):
    dims, Ls = (4, 2, 4, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.05, b=bc[0], c=bc[1], tbc=tbc)
    U = synth.random_links(dims, 0.5, 21)
    G = synth.random_gauge_transform(dims, 22)
    UG = gauge_transform(U, G)
    psi = synth.gaussian_spinor(dims, Ls, 23)
    Gpsi = np.einsum("tzyxab,stzyxpb->stzyxpa", G, psi)
    lhs = ora.dwf(p, UG, Gpsi)
    rhs = np.einsum("tzyxab,stzyxpb->stzyxpa", G, ora.dwf(p, U, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))
    po = synth.gaussian_spinor_parity(dims, Ls, 24, 1)
    Gpo = np.einsum("tzyxab,stzyxpb->stzyxpa", G, po)
    lhs = ora.mprec(p, UG, Gpo)
    rhs = np.einsum("tzyxab,stzyxpb->stzyxpa", G, ora.mprec(p, U, po))
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


# --------------------------------------------------------------------- adjoint pairs
@pytest.mark.parametrize("bc", [(1.0, 0.0), (1.5, 0.5), (2.0, 1.0)])
def test_adjoint_identities(ora, bc):
    dims, Ls = (4, 4, 2, 4), 6
    p = ora.params(dims, Ls, M5=1.8, mass=0.1, b=bc[0], c=bc[1], tbc=1)
    U = synth.random_links(dims, 0.6, 31)
    x = synth.gaussian_spinor(dims, Ls, 32)
    y = synth.gaussian_spinor(dims, Ls, 33)
    xo = synth.gaussian_spinor_parity(dims, Ls, 34, 1)
    yo = synth.gaussian_spinor_parity(dims, Ls, 35, 1)
    pairs = [
        (lambda v: ora.dwf(p, U, v), lambda v: ora.dwf(p, U, v, dagger=True), x, y),
        (lambda v: ora.hop5(p, U, v), lambda v: ora.hop5(p, U, v, dagger=True), x, y),
        (lambda v: ora.bhop(p, U, v), lambda v: ora.bhop(p, U, v, dagger=True), x, y),
        (lambda v: ora.stilde(p, v), lambda v: ora.stilde(p, v, dagger=True), x, y),
        (lambda v: ora.fifth(p, v, "A"), lambda v: ora.fifth(p, v, "Adag"), x, y),
        (lambda v: ora.fifth(p, v, "Ainv"), lambda v: ora.fifth(p, v, "Ainvdag"), x, y),
        (lambda v: ora.fifth(p, v, "F"), lambda v: ora.fifth(p, v, "Fdag"), x, y),
        (lambda v: ora.mprec(p, U, v), lambda v: ora.mprec(p, U, v, dagger=True), xo, yo),
    ]
    for M, Md, a, b in pairs:
        lhs = vdot(a, M(b))
        rhs = vdot(Md(a), b)
        assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


@pytest.mark.parametrize("dagger", [False, True])
def test_hop5_sample_is_the_whole_lattice_hop(ora, dagger):
    """The sampled hop (the reference of the full-size parity test) equals the whole-lattice hop at
    every sampled (4D site, s) of both parities, and every slice of the whole-lattice hop is the
    hopping term of the pinned 4D Wilson operator, H = 2 ((4 - M5) - D_W).  All extents and Ls
    differ, so that a transposed or mis-strided (site, s) mapping fails."""
    dims, Ls, M5 = (4, 6, 2, 8), 5, 1.8
    p = ora.params(dims, Ls, M5=M5, tbc=1)
    p4 = ora.params(dims, 1, M5=M5, tbc=1)
    U = synth.random_links(dims, 0.6, 51)
    psi = synth.gaussian_spinor(dims, Ls, 52)
    V = int(np.prod(dims))
    whole = ora.hop5(p, U, psi, dagger=dagger)
    for s in range(Ls):
        h = 2.0 * ((4.0 - M5) * psi[s] - ora.dw4(p4, U, psi[s], dagger=dagger))
        assert np.max(np.abs(whole[s] - h)) < 1e-13 * np.max(np.abs(h))
    rng = np.random.default_rng(53)
    n = 400
    sites = rng.integers(0, V, n)
    svals = rng.integers(0, Ls, n)
    got = ora.hop5_sample(p, U, psi, sites, svals, dagger=dagger)
    ref = whole.reshape(Ls, V, 4, 3)[svals, sites]
    assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref))
    par = synth.parity_array(dims).ravel()[sites]
    assert 0 < par.sum() < n  # both output parities sampled


def reflect5(psi):
    return psi[::-1].copy()


def test_shamir_gamma5_r5_hermiticity(ora):
    """Shamir DWF: Gamma5 D Gamma5 = D^dag with Gamma5 = R5 gamma5 (R5: s -> Ls-1-s)."""
    dims, Ls = (4, 4, 4, 2), 8
    p = ora.params(dims, Ls, M5=1.8, mass=0.03)
    U = synth.random_links(dims, 0.5, 41)
    y = synth.gaussian_spinor(dims, Ls, 42)
    g5 = ora.gammas()[4]
    G5 = lambda v: spin(g5, reflect5(v))
    lhs = G5(ora.dwf(p, U, G5(y)))
    rhs = ora.dwf(p, U, y, dagger=True)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


# --------------------------------------------------------------------- fifth-dimension blocks
@pytest.mark.parametrize("Ls,bc,m", [(16, (1.0, 0.0), 0.01), (16, (1.5, 0.5), 0.005), (5, (2.0, 1.0), 1.0)])
def test_fifth_inverse_closed_form(ora, Ls, bc, m):
    """A^-1 from Gauss-Jordan equals the geometric-series closed form per chirality:
    (alpha + beta S)^-1 = sum_{k<Ls} (-z)^k S^k / (alpha (1 + m (-z)^Ls)), z = beta/alpha,
    where S is the cyclic s-shift carrying the factor -m across the boundary."""
    M5 = 1.8
    p = ora.params((2, 2, 2, 2), Ls, M5=M5, mass=m, b=bc[0], c=bc[1])
    A = ora.fifth_matrix(p, "A")
    Ainv = ora.fifth_matrix(p, "Ainv")
    n = 4 * Ls
    assert np.max(np.abs(A @ Ainv - np.eye(n))) < 1e-13
    d = 4 - M5
    alpha, beta = bc[0] * d + 1, bc[1] * d - 1
    z = beta / alpha
    Sp = np.zeros((Ls, Ls)); Sm = np.zeros((Ls, Ls))
    for s in range(Ls):
        if s + 1 < Ls:
            Sp[s, s + 1] = 1
        else:
            Sp[s, 0] = -m
        if s >= 1:
            Sm[s, s - 1] = 1
        else:
            Sm[s, Ls - 1] = -m
    norm = 1.0 / (alpha * (1 + m * (-z) ** Ls))
    inv_minus = norm * sum((-z) ** k * np.linalg.matrix_power(Sp, k) for k in range(Ls))  # P- chirality
    inv_plus = norm * sum((-z) ** k * np.linalg.matrix_power(Sm, k) for k in range(Ls))   # P+ chirality
    Ainv4 = Ainv.reshape(Ls, 4, Ls, 4)
    for al in range(4):
        ref = inv_plus if al < 2 else inv_minus
        assert np.max(np.abs(Ainv4[:, al, :, al] - ref)) < 1e-13
        for be in range(4):
            if be != al:
                assert np.max(np.abs(Ainv4[:, al, :, be])) < 1e-15


# --------------------------------------------------------------------- dense 2^4 checks
def dense_matrix(apply, shape, dtype=np.complex128):
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype)
    e = np.zeros(n, dtype)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        M[:, j] = apply(e.reshape(shape)).ravel()
    return M


@pytest.fixture(scope="module")
def dense_setup(ora):
    dims, Ls = (2, 2, 2, 2), 4
    U = synth.random_links(dims, 0.5, 51)
    return dims, Ls, U


def test_dense_solve_and_schur(ora, dense_setup):
    dims, Ls, U = dense_setup
    p = ora.params(dims, Ls, M5=1.8, mass=0.01)
    shape = (Ls, 2, 2, 2, 2, 4, 3)
    D = dense_matrix(lambda v: ora.dwf(p, U, v), shape)
    b = synth.gaussian_spinor(dims, Ls, 52)
    x_dense = np.linalg.solve(D, b.ravel())
    x, info = ora.solve(p, U, b, tol=1e-13)
    assert info["converged"] and info["true_rel_resid"] <= 1e-13
    assert np.linalg.norm(x.ravel() - x_dense) <= 1e-10 * np.linalg.norm(x_dense)
    # Schur complement on odd sites: M_prec = A_oo^-1 (D_oo - D_oe D_ee^-1 D_eo)
    par = np.broadcast_to(synth.parity_array(dims)[None, ..., None, None], shape).ravel()
    e, o = np.where(par == 0)[0], np.where(par == 1)[0]
    S = D[np.ix_(o, o)] - D[np.ix_(o, e)] @ np.linalg.solve(D[np.ix_(e, e)], D[np.ix_(e, o)])
    A_oo = D[np.ix_(o, o)]  # the hop never connects equal parities, so D_oo = A
    Mdense = np.linalg.solve(A_oo, S)
    Morc = dense_matrix(lambda v: ora.mprec(p, U, v), shape)[np.ix_(o, o)]
    assert np.max(np.abs(Morc - Mdense)) < 1e-12


def parity5_flat(dims, Ls):
    shape = (Ls, dims[3], dims[2], dims[1], dims[0], 4, 3)
    p5 = (np.arange(Ls)[:, None, None, None, None] + synth.parity_array(dims)[None]) & 1
    return np.broadcast_to(p5[..., None, None], shape).ravel()


@pytest.fixture(scope="module")
def dense_shamir5(ora, dense_setup):
    """Dense Shamir D(m) on 2^4 x Ls=4 (m = 0.1, antiperiodic in T) and the 5D parities"""
    dims, Ls, U = dense_setup
    p = ora.params(dims, Ls, M5=1.8, mass=0.1, tbc=1)
    D = dense_matrix(lambda v: ora.dwf(p, U, v), (Ls, 2, 2, 2, 2, 4, 3))
    return D, parity5_flat(dims, Ls)


def test_shamir_operator_on_the_5d_checkerboard(ora, dense_setup, dense_shamir5):
    """Shamir D(m) - (5 - M5) has no matrix element between sites of equal 5D parity
    (x + y + z + t + s) mod 2 (the 4D hop changes x, the fifth-dimension hop changes s); a Moebius
    operator's c D_W (P- psi_{s+1} + P+ psi_{s-1}) term does couple them (x and s change together):
    a point source at (x, s) reaches (x + mu, s + 1)."""
    D, par = dense_shamir5
    K = (5 - 1.8) * np.eye(D.shape[0]) - D
    assert np.max(np.abs(K[np.equal.outer(par, par)])) < 1e-15
    assert np.max(np.abs(K)) > 0.4
    dims, Ls, U = dense_setup
    pm = ora.params(dims, Ls, M5=1.8, mass=0.1, b=1.5, c=0.5)
    v = np.zeros((Ls, 2, 2, 2, 2, 4, 3), complex)
    v[1, 0, 0, 0, 0, 0, 0] = 1.0  # s = 1, site 0, spin 0 (P+): P+ psi_{s-1} feeds s = 2
    Dv = ora.dwf(pm, U, v)
    assert np.max(np.abs(Dv[2, 0, 0, 0, 1])) > 0.1  # (x + 1, s + 1): equal 5D parity


def test_5d_schur_route_solves_d(ora, dense_shamir5):
    """The route of the 5D even-odd solver: b'_e = b_e + K_eo b_o / d0, S x_e = b'_e with
    S = d0 - K_eo K_oe / d0, x_o = (b_o + K_oe x_e) / d0, gives the dense solution of D x = b."""
    D, par = dense_shamir5
    d0 = 5 - 1.8
    K = d0 * np.eye(D.shape[0]) - D
    e, o = np.where(par == 0)[0], np.where(par == 1)[0]
    b = synth.gaussian_spinor((2, 2, 2, 2), 4, 53).ravel()
    S = d0 * np.eye(len(e)) - K[np.ix_(e, o)] @ K[np.ix_(o, e)] / d0
    xe = np.linalg.solve(S, b[e] + K[np.ix_(e, o)] @ b[o] / d0)
    xo = (b[o] + K[np.ix_(o, e)] @ xe) / d0
    x = np.zeros_like(b)
    x[e], x[o] = xe, xo
    x_dense = np.linalg.solve(D, b)
    assert np.linalg.norm(x - x_dense) <= 1e-12 * np.linalg.norm(x_dense)


def dense_dw(ora, dims, U, M5):
    p4 = ora.params(dims, 1, M5=M5)
    return dense_matrix(lambda v: ora.dw4(p4, U, v), (2, 2, 2, 2, 4, 3))


def overlap_closed_form(ora, DW, Ls, b, c, m, nsite):
    """D_OV(m) = (1+m)/2 + (1-m)/2 gamma5 eps_L(H_M), H_M = gamma5 (b+c) D_W [2 + (b-c) D_W]^-1,
    eps_L(H) = [(1+H)^L - (1-H)^L][(1+H)^L + (1-H)^L]^-1  (the Moebius domain-wall/overlap relation)."""
    g5 = np.kron(np.kron(np.eye(nsite), ora.gammas()[4]), np.eye(3))
    n = DW.shape[0]
    I = np.eye(n)
    HM = g5 @ ((b + c) * DW) @ np.linalg.inv(2 * I + (b - c) * DW)
    Pp = np.linalg.matrix_power(I + HM, Ls)
    Pm = np.linalg.matrix_power(I - HM, Ls)
    eps = (Pp - Pm) @ np.linalg.inv(Pp + Pm)
    return 0.5 * (1 + m) * I + 0.5 * (1 - m) * g5 @ eps


@pytest.mark.parametrize("Ls,bc", [(4, (1.0, 0.0)), (6, (1.5, 0.5)), (4, (0.5, 0.5))])
def test_block_triangular_overlap_structure(ora, dense_setup, Ls, bc):
    """Sec. 4: P^-1 D(1)^-1 D(m) P is the identity except for its first block column,
    whose (1,1) block is the effective 4D operator D_OV(m)."""
    dims, _, U = dense_setup
    m, M5 = 0.04, 1.8
    shape = (Ls, 2, 2, 2, 2, 4, 3)
    pm = ora.params(dims, Ls, M5=M5, mass=m, b=bc[0], c=bc[1])
    p1 = ora.params(dims, Ls, M5=M5, mass=1.0, b=bc[0], c=bc[1])
    Dm = dense_matrix(lambda v: ora.dwf(pm, U, v), shape)
    D1 = dense_matrix(lambda v: ora.dwf(p1, U, v), shape)
    Pm_ = dense_matrix(lambda v: ora.P(pm, v), shape)
    Pinv = dense_matrix(lambda v: ora.P(pm, v, inverse=True), shape)
    assert np.max(np.abs(Pinv @ Pm_ - np.eye(Pm_.shape[0]))) < 1e-15
    K = Pinv @ np.linalg.solve(D1, Dm @ Pm_)
    n4 = 16 * 12
    # identity beyond the first block column
    assert np.max(np.abs(K[:, n4:] - np.eye(K.shape[0])[:, n4:])) < 1e-12
    DW = dense_dw(ora, dims, U, M5)
    DOV = overlap_closed_form(ora, DW, Ls, bc[0], bc[1], m, 16)
    assert np.max(np.abs(K[:n4, :n4] - DOV)) < 1e-12


def test_moebius_route_to_y1(ora, dense_setup):
    """Sec. 4: solving D'(m) P y' = D'(1) P c' with c' = (c_1, 0, ..., 0) gives the first slice
    y'_1 of P'^-1 y' = D'_OV(m)^-1 c_1; the reconstruction's first block is -D_OV y'_1."""
    dims, _, U = dense_setup
    Lp, b, c, m, M5 = 4, 1.5, 0.5, 0.04, 1.8
    pm = ora.params(dims, Lp, M5=M5, mass=m, b=b, c=c)
    p1 = ora.params(dims, Lp, M5=M5, mass=1.0, b=b, c=c)
    c1 = synth.gaussian_spinor(dims, 1, 61)[0]
    cp = np.zeros((Lp,) + c1.shape, np.complex128)
    cp[0] = c1
    rhs = ora.dwf(p1, U, ora.P(pm, cp))
    z, info = ora.solve(pm, U, rhs, tol=1e-13)
    y1 = ora.P(pm, z, inverse=True)[0]
    DW = dense_dw(ora, dims, U, M5)
    DOVp = overlap_closed_form(ora, DW, Lp, b, c, m, 16)
    assert np.linalg.norm(DOVp @ y1.ravel() - c1.ravel()) < 1e-11 * np.linalg.norm(c1)
    # reconstruction (target Shamir L=6): first slice of P^-1 D(1)^-1 D(m) P (-y1, c_2..c_L) is -D_OV y1
    L = 6
    pt = ora.params(dims, L, M5=M5, mass=m)
    pt1 = ora.params(dims, L, M5=M5, mass=1.0)
    cc = synth.gaussian_spinor(dims, L, 62)
    v = cc.copy()
    v[0] = -y1
    w, _ = ora.solve(pt1, U, ora.dwf(pt, U, ora.P(pt, v)), tol=1e-13)
    w = ora.P(pt, w, inverse=True)
    DOV = overlap_closed_form(ora, DW, L, 1.0, 0.0, m, 16)
    assert np.linalg.norm(w[0].ravel() + DOV @ y1.ravel()) < 1e-10 * np.linalg.norm(y1)


# --------------------------------------------------------------------- solvers
def test_cg_reaches_true_residual_cfg1(ora):
    """4^4, Ls=8, M5=1.8, m=0.01, eps=0.3: even-odd CGNR to a full-system true residual 1e-10."""
    dims, Ls = (4, 4, 4, 4), 8
    p = ora.params(dims, Ls, M5=1.8, mass=0.01)
    U = synth.random_links(dims, 0.3, synth.link_seed(1))
    b = synth.gaussian_spinor(dims, Ls, synth.source_seed(1))
    x, info = ora.solve(p, U, b, tol=1e-10)
    r = b - ora.dwf(p, U, x)
    assert info["converged"]
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)


def test_madwf_exact_inner_is_direct(ora):
    """With the inner operator equal to the target and tight solves, one MADWF step
    (Sec. 4 algorithm) already yields the solution."""
    dims, L = (4, 4, 2, 2), 4
    pt = ora.params(dims, L, M5=1.8, mass=0.05)
    U = synth.random_links(dims, 0.4, 71)
    b = synth.gaussian_spinor(dims, L, 72)
    x, info = ora.madwf(pt, pt, U, b, n_dc=1, tol_pv=1e-13, tol_mob=1e-13, tol=1e-10)
    assert info["resid_after_dc"][0] < 1e-10
    assert info["final_iters"] == 0


def test_madwf_defect_correction_decreases(ora):
    """Sec. 5: each defect-correction step lowers the true residual of the guess."""
    dims, L = (4, 4, 4, 4), 8
    pt = ora.params(dims, L, M5=1.8, mass=0.02)
    pi = ora.params(dims, 4, M5=1.8, mass=0.02, b=1.5, c=0.5)
    U = synth.random_links(dims, 0.3, 81)
    b = synth.gaussian_spinor(dims, L, 82)
    x, info = ora.madwf(pt, pi, U, b, n_dc=3, tol_pv=1e-10, tol_mob=1e-8, tol=1e-10)
    r = info["resid_after_dc"]
    assert r[0] < 1 and r[1] < r[0] and r[2] < r[1]
    assert info["converged"] and info["true_rel_resid"] <= 1e-10
    assert np.linalg.norm(b - ora.dwf(pt, U, x)) <= 1e-10 * np.linalg.norm(b)


# --------------------------------------------------------------------- force
def perturb_link(U, mu, t, z, y, x, M):
    V = U.copy()
    V[mu, t, z, y, x] = M @ U[mu, t, z, y, x]
    return V


@pytest.mark.parametrize("bc,tbc", [((1.0, 0.0), 0), ((1.5, 0.5), 1)])
def test_force_finite_difference(ora, bc, tbc):
    """e_a(S) = d/dw S[exp(w T_a) U] (Sec. 2) against central differences, h = 1e-4."""
    dims, Ls = (2, 2, 4, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.05, b=bc[0], c=bc[1], tbc=tbc)
    U = synth.random_links(dims, 0.5, 91)
    phi = synth.gaussian_spinor_parity(dims, Ls, 92, 1)
    S0, X, _ = ora.action(p, U, phi, tol=1e-14)
    F, e = ora.force(p, U, X)
    T = ora.generators()
    h = 1e-4
    for (mu, t, z, y, x, a) in synth.sample_links(dims, 12, 93):
        Sp, _, _ = ora.action(p, perturb_link(U, mu, t, z, y, x, scipy.linalg.expm(h * T[a])), phi,
                              x0=X, tol=1e-14)
        Sm, _, _ = ora.action(p, perturb_link(U, mu, t, z, y, x, scipy.linalg.expm(-h * T[a])), phi,
                              x0=X, tol=1e-14)
        fd = (Sp - Sm) / (2 * h)
        assert abs(fd - e[mu, t, z, y, x, a]) <= 1e-6 * max(abs(fd), 1e-2)
    # F = sum_a e_a T_a is traceless anti-Hermitian
    assert np.max(np.abs(F + np.conj(np.swapaxes(F, -1, -2)))) < 1e-12
    assert np.max(np.abs(np.trace(F, axis1=-2, axis2=-1))) < 1e-12


def test_force_sample_is_the_whole_lattice_force(ora):
    """The sampled force (the reference of the full-size force test) equals the whole-lattice
    force on every sampled link of both parities and all four directions (all extents differ, so
    a mis-strided (site, mu) mapping fails)."""
    dims, Ls = (4, 6, 2, 8), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.1, b=1.5, c=0.5, tbc=1)
    U = synth.random_links(dims, 0.5, 81)
    X = synth.gaussian_spinor_parity(dims, Ls, 82, 1)
    F, e = ora.force(p, U, X)
    V = int(np.prod(dims))
    rng = np.random.default_rng(83)
    sites = rng.integers(0, V, 200)
    mus = rng.integers(0, 4, 200)
    Fs, es = ora.force_sample(p, U, X, sites, mus)
    Fw = F.reshape(4, V, 3, 3)[mus, sites]
    ew = e.reshape(4, V, 8)[mus, sites]
    assert np.max(np.abs(Fs - Fw)) <= 1e-14 * np.max(np.abs(Fw))
    assert np.max(np.abs(es - ew)) <= 1e-14 * np.max(np.abs(ew))
    par = synth.parity_array(dims).ravel()[sites]
    assert 0 < par.sum() < len(sites) and set(mus) == {0, 1, 2, 3}


def test_force_gauge_covariance(ora):
    dims, Ls = (4, 2, 2, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.05)
    U = synth.random_links(dims, 0.5, 101)
    G = synth.random_gauge_transform(dims, 102)
    phi = synth.gaussian_spinor_parity(dims, Ls, 103, 1)
    S, X, _ = ora.action(p, U, phi, tol=1e-14)
    F, _ = ora.force(p, U, X)
    UG = gauge_transform(U, G)
    Gphi = np.einsum("tzyxab,stzyxpb->stzyxpa", G, phi)
    SG, XG, _ = ora.action(p, UG, Gphi, tol=1e-14)
    FG, _ = ora.force(p, UG, XG)
    assert abs(S - SG) < 1e-11 * abs(S)
    expect = G[None] @ F @ np.conj(np.swapaxes(G, -1, -2))[None]
    assert np.max(np.abs(FG - expect)) < 1e-9 * np.max(np.abs(F))


def test_force_gradient_step_scaling(ora):
    """Sec. 2: the force at U' = exp(-tau^2/24 F) U differs from the force at U by
    -tau^2/24 times the derivative of the force along F (F held fixed), up to terms of
    relative size tau^2 |F| / 24; the difference therefore scales as tau^2.  The forces on
    this small rough lattice are large (|F| ~ 1e2), so tau is taken small enough that
    tau^2 |F| / 24 << 1."""
    dims, Ls = (2, 2, 2, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.05)
    U = synth.random_links(dims, 0.5, 111)
    phi = synth.gaussian_spinor_parity(dims, Ls, 112, 1)
    S, X, _ = ora.action(p, U, phi, tol=1e-14)
    F, _ = ora.force(p, U, X)
    diffs = {}
    for tau in (0.02, 0.01):
        Fp, Xp, _, iters = ora.fg_force(p, U, phi, tau, tol=1e-14)
        diffs[tau] = Fp - F
        assert iters[1] < iters[0]  # the warm start from X(U) saves iterations
    ratio = np.linalg.norm(diffs[0.02]) / np.linalg.norm(diffs[0.01])
    assert abs(ratio - 4.0) < 0.1
    # directional derivative of the force along -F by central differences
    h = 1e-4
    def force_at(Uv):
        _, Xv, _ = ora.action(p, Uv, phi, x0=X, tol=1e-14)
        return ora.force(p, Uv, Xv)[0]
    dF = (force_at(ora.mat3_exp(-h * F) @ U) - force_at(ora.mat3_exp(h * F) @ U)) / (2 * h)
    eps = 0.02 ** 2 / 24
    rel = np.linalg.norm(diffs[0.02] - eps * dF) / np.linalg.norm(diffs[0.02])
    assert rel < 0.03


def test_mat3_exp_matches_expm(ora):
    rng = np.random.default_rng(121)
    A = rng.standard_normal((20, 3, 3)) + 1j * rng.standard_normal((20, 3, 3))
    A *= 1.5
    E = ora.mat3_exp(A)
    for k in range(20):
        assert np.max(np.abs(E[k] - scipy.linalg.expm(A[k]))) < 1e-12 * np.max(np.abs(E[k]))


@pytest.mark.parametrize("bc", [(1.0, 0.0), (1.5, 0.5)])
def test_quotient_force_finite_difference(ora, bc):
    """Hasenbusch quotient action of Sec. 3, S = phi^dag M(m_n) (M(m_d)^dag M(m_d))^-1 M(m_n)^dag phi:
    e_a(S) against central differences of S along exp(+-h T_a) on sampled links."""
    dims, Ls = (2, 2, 4, 4), 4
    pn = ora.params(dims, Ls, M5=1.8, mass=0.3, b=bc[0], c=bc[1])
    pd = ora.params(dims, Ls, M5=1.8, mass=0.05, b=bc[0], c=bc[1])
    U = synth.random_links(dims, 0.5, 131)
    phi = synth.gaussian_spinor_parity(dims, Ls, 132, 1)
    S0, F, e, X, _ = ora.quotient_force(pn, pd, U, phi, tol=1e-14)
    assert S0 > 0
    T = ora.generators()
    # fourth-order central differences, h = 1e-3: truncation ~h^4, and the solver's 1e-14
    # relative accuracy of S contributes about |S| 1e-14 / h
    h = 1e-3

    def S_at(mu, t, z, y, x, a, w):
        Uw = perturb_link(U, mu, t, z, y, x, scipy.linalg.expm(w * T[a]))
        return ora.quotient_force(pn, pd, Uw, phi, x0=X, tol=1e-14)[0]

    for (mu, t, z, y, x, a) in synth.sample_links(dims, 12, 133):
        Sv = {k: S_at(mu, t, z, y, x, a, k * h) for k in (-2, -1, 1, 2)}
        fd = (8 * (Sv[1] - Sv[-1]) - (Sv[2] - Sv[-2])) / (12 * h)
        assert abs(fd - e[mu, t, z, y, x, a]) <= 1e-7 * max(abs(fd), 1e-2) + 1e-10 * abs(S0)
    assert np.max(np.abs(F + np.conj(np.swapaxes(F, -1, -2)))) < 1e-12
    assert np.max(np.abs(np.trace(F, axis1=-2, axis2=-1))) < 1e-12


def test_quotient_of_equal_masses_is_constant(ora):
    """With equal masses M (M^dag M)^-1 M^dag = 1: S = |phi|^2 for every gauge field, so the two
    force terms cancel (a sign or mass mix-up in either term leaves a force of the size of the
    one-flavour force)."""
    dims, Ls = (2, 2, 2, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.1, b=1.5, c=0.5)
    U = synth.random_links(dims, 0.5, 141)
    phi = synth.gaussian_spinor_parity(dims, Ls, 142, 1)
    S, F, e, X, _ = ora.quotient_force(p, p, U, phi, tol=1e-14)
    assert abs(S - np.vdot(phi, phi).real) < 1e-10 * abs(S)
    _, X1, _ = ora.action(p, U, phi, tol=1e-14)
    F1, _ = ora.force(p, U, X1)
    assert np.max(np.abs(F)) < 1e-9 * np.max(np.abs(F1))


def _momenta(ora, dims, seed):
    T = ora.generators()
    V = int(np.prod(dims))
    c = synth.random_su3_algebra(4 * V, seed)
    return np.einsum("na,aij->nij", c, T).reshape((4,) + tuple(dims[::-1]) + (3, 3)), c


def test_gauge_action_and_force(ora):
    """Plaquette action: zero on unit links, gauge invariant; its force against fourth-order
    central differences of the action along exp(+-h T_a)."""
    dims = (2, 4, 2, 4)
    p = ora.params(dims, 2)
    beta = 2.3
    assert abs(ora.gauge_action(p, synth.unit_links(dims), beta)) < 1e-12
    U = synth.random_links(dims, 0.5, 151)
    S0 = ora.gauge_action(p, U, beta)
    G = synth.random_gauge_transform(dims, 152)
    assert abs(ora.gauge_action(p, gauge_transform(U, G), beta) - S0) < 1e-11 * abs(S0)
    F = ora.gauge_force(p, U, beta)
    T = ora.generators()
    h = 1e-3
    for (mu, t, z, y, x, a) in synth.sample_links(dims, 12, 153):
        Sv = {k: ora.gauge_action(p, perturb_link(U, mu, t, z, y, x, scipy.linalg.expm(k * h * T[a])), beta)
              for k in (-2, -1, 1, 2)}
        fd = (8 * (Sv[1] - Sv[-1]) - (Sv[2] - Sv[-2])) / (12 * h)
        e_a = -2.0 * np.trace(T[a] @ F[mu, t, z, y, x]).real  # F = sum_a e_a T_a, tr(T_a T_b) = -delta/2
        assert abs(fd - e_a) <= 1e-8 * max(abs(fd), 1.0)


def test_fgi_trajectory_is_reversible(ora):
    """Sec. 2: the force-gradient integrator is symmetric -- integrating back from (U', -P')
    returns to (U, -P) up to the solver tolerance."""
    dims, Ls = (2, 2, 2, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.1)
    U = synth.random_links(dims, 0.3, 161)
    phi = ora.mprec(p, U, synth.gaussian_spinor_parity(dims, Ls, 162, 1), dagger=True)
    P, _ = _momenta(ora, dims, 163)
    U1, P1, H, _ = ora.fgi_trajectory(p, 2.0, 0.125, 4, U, P, phi)
    U2, P2, H2, _ = ora.fgi_trajectory(p, 2.0, 0.125, 4, U1, -P1, phi)
    assert np.max(np.abs(U2 - U)) < 1e-11
    assert np.max(np.abs(P2 + P)) < 1e-10
    assert abs(H2[1] - H[0]) < 1e-9
    assert abs(H2[0] - H[1]) < 1e-9


def test_fgi_energy_violation_scales_as_tau4(ora):
    """The integrator is fourth order with the two-step force-gradient term (Sec. 2): at fixed
    trajectory length dH ~ tau^4.  Gauge action alone (exact asymptotics at these step sizes),
    and with the fermion action (rougher: smaller steps).  A sign error in the force-gradient
    term leaves a second-order integrator (ratio 4 per halving)."""
    dims, Ls = (2, 2, 2, 4), 4
    p = ora.params(dims, Ls, M5=1.8, mass=0.1)
    U = synth.random_links(dims, 0.3, 171)
    eta = synth.gaussian_spinor_parity(dims, Ls, 172, 1)
    phi = ora.mprec(p, U, eta, dagger=True)
    P, c = _momenta(ora, dims, 173)
    # kinetic energy of P = sum p_a T_a is sum p_a^2 / 2
    _, _, H, _ = ora.fgi_trajectory(p, 2.0, 0.1, 1, U, P, 0 * phi)
    assert abs((H[0] - ora.gauge_action(p, U, 2.0)) - 0.5 * np.sum(c ** 2)) < 1e-9
    dH = {}
    for n in (8, 16):
        _, _, H, _ = ora.fgi_trajectory(p, 2.0, 0.5 / n, n, U, P, 0 * phi)
        dH[n] = H[1] - H[0]
    assert abs(dH[8] / dH[16] - 16.0) < 0.5
    for n in (16, 32):
        _, _, H, _ = ora.fgi_trajectory(p, 2.0, 0.5 / n, n, U, P, phi)
        dH[n] = H[1] - H[0]
    assert 12.0 < dH[16] / dH[32] < 20.0


def test_random_momenta_distribution(ora):
    """synth.random_momenta draws P = sum_a p_a T_a with p_a ~ N(0, 1): traceless
    anti-Hermitian, and its generator coefficients p_a = -2 tr(T_a P) have unit variance and
    no correlation."""
    dims = (8, 8, 8, 8)  # 16384 links: sampling error of the covariance about 0.01
    P = synth.random_momenta(dims, 181).reshape(-1, 3, 3)
    assert np.max(np.abs(P + np.conj(np.swapaxes(P, -1, -2)))) < 1e-15
    assert np.max(np.abs(np.trace(P, axis1=-2, axis2=-1))) < 1e-15
    T = ora.generators()
    c = -2 * np.einsum("aij,nji->na", T, P).real
    cov = np.cov(c.T)
    assert np.max(np.abs(cov - np.eye(8))) < 0.06


# --------------------------------------------------------------------- s-dependent Moebius coefficients
def mask(psi, dims, parity):
    """psi restricted to one 4D parity (the other parity set to zero)."""
    keep = synth.parity_array(dims) == parity
    return psi * keep[None, ..., None, None]


def test_s_dependent_coefficients_constant_arrays_match_scalars(ora):
    """Arrays b_s = b, c_s = c reproduce the constant-coefficient operator exactly."""
    dims, Ls = (2, 2, 2, 4), 6
    U = synth.random_links(dims, 0.5, 191)
    psi = synth.gaussian_spinor(dims, Ls, 192)
    p0 = ora.params(dims, Ls, mass=0.07, b=1.5, c=0.5, tbc=1)
    p1 = ora.params(dims, Ls, mass=0.07, b=9.0, c=-3.0, tbc=1, bs=np.full(Ls, 1.5), cs=np.full(Ls, 0.5))
    for dag in (False, True):
        assert np.max(np.abs(ora.dwf(p0, U, psi, dagger=dag) - ora.dwf(p1, U, psi, dagger=dag))) == 0.0
    po = mask(psi, dims, 1)
    assert np.max(np.abs(ora.mprec(p0, U, po) - ora.mprec(p1, U, po))) < 1e-14


def test_s_dependent_coefficients_adjoints(ora):
    """<phi, D psi> = <D^dag phi, psi> and the same for M_prec with varying b_s, c_s (the
    adjoint of diag(c) S~ is S~^dag diag(c): the order matters once c varies)."""
    dims, Ls = (2, 2, 2, 4), 6
    rng = np.random.default_rng(193)
    bs, cs = 1.0 + rng.random(Ls), rng.random(Ls) - 0.3
    p = ora.params(dims, Ls, mass=0.07, tbc=1, bs=bs, cs=cs)
    U = synth.random_links(dims, 0.5, 194)
    psi, phi = synth.gaussian_spinor(dims, Ls, 195), synth.gaussian_spinor(dims, Ls, 196)
    lhs = np.vdot(phi, ora.dwf(p, U, psi))
    rhs = np.vdot(ora.dwf(p, U, phi, dagger=True), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    po, fo = mask(psi, dims, 1), mask(phi, dims, 1)
    lhs = np.vdot(fo, ora.mprec(p, U, po))
    rhs = np.vdot(ora.mprec(p, U, fo, dagger=True), po)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_s_dependent_overlap_structure(ora, dense_setup):
    """Sec. 4 with an s-dependent Moebius operator, b_s - c_s = 1 and omega_s = b_s + c_s:
    P^-1 D(1)^-1 D(m) P is the identity beyond its first block column, whose first block is
    D_OV(m) = (1+m)/2 + (1-m)/2 gamma5 eps(H), eps(H) = [prod(1 + omega_s H) - prod(1 - omega_s H)]
    [prod(1 + omega_s H) + prod(1 - omega_s H)]^-1, H = gamma5 D_W (2 + D_W)^-1."""
    dims, _, U = dense_setup
    Ls, m, M5 = 4, 0.04, 1.8
    omega = np.array([0.6, 1.3, 2.1, 0.9])
    bs, cs = (omega + 1) / 2, (omega - 1) / 2
    shape = (Ls, 2, 2, 2, 2, 4, 3)
    pm = ora.params(dims, Ls, M5=M5, mass=m, bs=bs, cs=cs)
    p1 = ora.params(dims, Ls, M5=M5, mass=1.0, bs=bs, cs=cs)
    Dm = dense_matrix(lambda v: ora.dwf(pm, U, v), shape)
    D1 = dense_matrix(lambda v: ora.dwf(p1, U, v), shape)
    Pm_ = dense_matrix(lambda v: ora.P(pm, v), shape)
    Pinv = dense_matrix(lambda v: ora.P(pm, v, inverse=True), shape)
    K = Pinv @ np.linalg.solve(D1, Dm @ Pm_)
    n4 = 16 * 12
    assert np.max(np.abs(K[:, n4:] - np.eye(K.shape[0])[:, n4:])) < 1e-12
    DW = dense_dw(ora, dims, U, M5)
    g5 = np.kron(np.kron(np.eye(16), ora.gammas()[4]), np.eye(3))
    I = np.eye(DW.shape[0])
    H = g5 @ DW @ np.linalg.inv(2 * I + DW)
    Pp, Pm = I.copy(), I.copy()
    for w in omega:
        Pp, Pm = Pp @ (I + w * H), Pm @ (I - w * H)
    eps = (Pp - Pm) @ np.linalg.inv(Pp + Pm)
    DOV = 0.5 * (1 + m) * I + 0.5 * (1 - m) * g5 @ eps
    assert np.max(np.abs(K[:n4, :n4] - DOV)) < 1e-12
