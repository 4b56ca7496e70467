"""Pins for the CPU oracle (no GPU).  Each test ties the oracle to something
other than itself: closed forms, limits, invariants stated in the paper, a
second and third route, brute force on tiny inputs, and planted mistakes that
must be caught."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import oracle.routes as ox
from x2c_inputs import C_LIGHT, ag_2c, neon_s20, atom_block
from x2c_inputs import integrals as gi
from tests.dirac_ref import dirac_1s, dirac_energy

C = C_LIGHT


def _args(blk, twocomp):
    return blk.S, blk.T, blk.V, (blk.W if twocomp else blk.W[0])


@pytest.fixture(scope="module")
def neon():
    blk = neon_s20()
    h, eps, parts = ox.x2c_direct(*_args(blk, False), C, False, return_parts=True)
    return blk, h, eps, parts


@pytest.fixture(scope="module")
def silver():
    blk = ag_2c()
    h, eps, parts = ox.x2c_direct(*_args(blk, True), C, True, return_parts=True)
    return blk, h, eps, parts


def random_spd_problem(N, seed, twocomp):
    rng = np.random.default_rng(seed)

    def spd(scale):
        A = rng.standard_normal((N, N))
        return scale * (A @ A.T / N + np.eye(N))

    S = spd(1.0)
    T = spd(3.0)
    Vr = rng.standard_normal((N, N))
    V = -(Vr @ Vr.T / N + 2 * np.eye(N)) * 5.0
    W = np.zeros((4, N, N))
    Wr = rng.standard_normal((N, N))
    W[0] = -(Wr @ Wr.T / N + np.eye(N)) * 40.0
    for k in (1, 2, 3):
        A = rng.standard_normal((N, N))
        W[k] = 3.0 * (A - A.T)
    return S, T, V, (W if twocomp else W[0])


# ---------------------------------------------------------------- P1 brute force 4c

@pytest.mark.parametrize("which", ["neon", "silver"])
def test_P1_eigenvalues_equal_positive_4c_branch(which, neon, silver):
    blk, h, eps, _ = neon if which == "neon" else silver
    tc = which == "silver"
    e4 = oracle.dirac_positive_spectrum(*_args(blk, tc), C, tc)
    e2 = oracle.spectrum_of(h, blk.S, tc)
    scale = np.abs(e4).max()
    assert np.abs(e2 - e4).max() <= 1e-10 * scale
    assert np.abs(np.sort(eps) - e4).max() <= 1e-12 * scale


# ---------------------------------------------------------------- P2 Dirac closed form

def test_P2_neon_1s_converges_to_dirac():
    Z = 10.0
    exact = dirac_1s(Z, C)
    assert abs(exact - (-50.066742016894)) < 1e-9
    ladders = [
        gi.Shell(0, 0.05 * 3.0 ** np.arange(20)),
        gi.Shell(0, 0.02 * 2.5 ** np.arange(30)),
        gi.Shell(0, 0.02 * 2.0 ** np.arange(40)),
    ]
    errs = []
    for sh in ladders:
        blk = gi.build_block(Z, [sh])
        h, eps = ox.x2c_direct(*_args(blk, False), C, False)
        errs.append(eps[0] - exact)
    # variational from above, monotone, last rung converged to < 1e-6 Eh
    assert all(e > 0 for e in errs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6
    assert abs(errs[0] - 2.047e-3) < 5e-6


def test_P2_silver_spin_orbit_levels(silver):
    """Z=47 two-component levels: 1s, then 2s1/2 and 2p1/2 (degenerate in
    Dirac-Coulomb), then 2p3/2 above them -- pins the sign of the
    spin-orbit matrices."""
    blk, h, eps, _ = silver
    e = np.sort(eps)
    Z = 47.0
    e1s = dirac_energy(Z, 1, -1, C)
    e2s = dirac_energy(Z, 2, -1, C)
    e2p1 = dirac_energy(Z, 2, 1, C)
    e2p3 = dirac_energy(Z, 2, -2, C)
    assert abs(e2s - e2p1) < 1e-9
    assert abs(e[0] - e1s) < 0.02 and abs(e[1] - e1s) < 0.02
    assert np.all(np.abs(e[2:6] - e2s) < 0.05)
    assert np.all(np.abs(e[6:10] - e2p3) < 0.05)
    assert e[6] - e[5] > 8.0          # 2p3/2 well above 2p1/2


# ---------------------------------------------------------------- P3 c -> infinity

def test_P3_nonrelativistic_limit_is_T_plus_V():
    blk = neon_s20()
    S, T, V, W = _args(blk, False)
    ref = T + V
    devs = []
    for c in (1e5, 1e6, 1e7):
        h, _ = ox.x2c_direct(S, T, V, W, c, False)
        devs.append(np.abs(h - ref).max() / np.abs(ref).max())
    r1 = devs[0] / devs[1]
    r2 = devs[1] / devs[2]
    assert 80 < r1 < 120 and 80 < r2 < 120
    assert devs[2] < 1e-5


# ---------------------------------------------------------------- P4 first-order shift

def test_P4_leading_relativistic_shift_of_1s():
    """(E_X2C - E_NR) c^2 -> -Z^4/8 for the hydrogenic 1s (Dirac expansion)."""
    Z = 10.0
    blk = gi.build_block(Z, [gi.Shell(0, 0.02 * 2.0 ** np.arange(40))])
    S, T, V, W = _args(blk, False)
    e_nr = sla.eigh(T + V, S, eigvals_only=True)[0]
    c = 2.0e3
    _, eps = ox.x2c_direct(S, T, V, W, c, False)
    shift = (eps[0] - e_nr) * c * c
    assert abs(shift - (-Z ** 4 / 8.0)) < 0.01 * Z ** 4 / 8.0


# ---------------------------------------------------------------- P5 free particle

def test_P5_free_particle_spectrum():
    blk = neon_s20()
    S, T = blk.S, blk.T
    N = S.shape[0]
    Z0 = np.zeros((N, N))
    _, eps = ox.x2c_direct(S, T, Z0, Z0, C, False)
    t = sla.eigh(T, S, eigvals_only=True)
    ref = 2 * C * C * t / (np.sqrt(C ** 4 + 2 * C * C * t) + C * C)
    assert np.abs(np.sort(eps) - ref).max() <= 1e-10 * ref.max()


# ---------------------------------------------------------------- P6 renormalisation

@pytest.mark.parametrize("which", ["neon", "silver"])
def test_P6_renormalisation_condition(which, neon, silver):
    blk, h, eps, parts = neon if which == "neon" else silver
    tc = which == "silver"
    Sx = oracle.spin_blockdiag(blk.S) if tc else blk.S
    R, St = parts["R"], parts["St"]
    lhs = R.conj().T @ St @ R
    assert np.abs(lhs - Sx).max() <= 1e-13 * np.abs(Sx).max()
    # U^L, U^S satisfy Eq. renorm with the 4c metric
    X = parts["X"]
    Tx = oracle.spin_blockdiag(blk.T) if tc else blk.T
    UL, US = R, X @ R
    m = UL.conj().T @ Sx @ UL + US.conj().T @ Tx @ US / (2 * C * C)
    assert np.abs(m - Sx).max() <= 1e-13 * np.abs(Sx).max()


# ---------------------------------------------------------------- P7 three routes

@pytest.mark.parametrize("which", ["neon", "silver"])
def test_P7_routes_agree(which, neon, silver):
    blk, h, eps, _ = neon if which == "neon" else silver
    tc = which == "silver"
    h2, e2 = ox.x2c_kbasis(*_args(blk, tc), C, tc)
    h3, e3 = ox.x2c_polar(*_args(blk, tc), C, tc)
    s = np.abs(h).max()
    assert np.abs(h - h2).max() <= 1e-12 * s
    assert np.abs(h - h3).max() <= 1e-12 * s
    assert np.abs(eps - e2).max() <= 1e-12 * np.abs(eps).max()


# ---------------------------------------------------------------- P8 Hermiticity

@pytest.mark.parametrize("which", ["neon", "silver"])
def test_P8_hermitian(which, neon, silver):
    blk, h, eps, _ = neon if which == "neon" else silver
    assert np.abs(h - h.conj().T).max() <= 1e-13 * np.abs(h).max()


# ---------------------------------------------------------------- P9 spin-free reduction

def test_P9_twocomp_without_spin_orbit_doubles_scalar_spectrum():
    blk = atom_block(17)
    W = blk.W.copy()
    W[1:] = 0.0
    h2, e2 = ox.x2c_direct(blk.S, blk.T, blk.V, W, C, True)
    h1, e1 = ox.x2c_direct(blk.S, blk.T, blk.V, W[0], C, False)
    ref = np.sort(np.concatenate([e1, e1]))
    assert np.abs(np.sort(e2) - ref).max() <= 1e-10 * np.abs(ref).max()
    N = blk.N
    # the 2c matrix is diag(h1, h1)
    assert np.abs(h2[:N, :N] - h1).max() <= 1e-11 * np.abs(h1).max()
    assert np.abs(h2[:N, N:]).max() <= 1e-11 * np.abs(h1).max()


# ---------------------------------------------------------------- P10 Kramers

def test_P10_kramers_pairs(silver):
    blk, h, eps, _ = silver
    e = np.sort(oracle.spectrum_of(h, blk.S, True))
    assert np.abs(e[0::2] - e[1::2]).max() <= 1e-12 * np.abs(e).max()


# ---------------------------------------------------------------- P11 DLU = full, uncoupled

def _combine(blocks, twocomp):
    """Molecular matrices of uncoupled atoms: block diagonal in the scalar
    basis (all atoms' functions, atom-major)."""
    Ns = [b.N for b in blocks]
    N = sum(Ns)
    S = np.zeros((N, N)); T = np.zeros((N, N)); V = np.zeros((N, N)); W = np.zeros((4, N, N))
    o = 0
    for b in blocks:
        n = b.N
        S[o:o + n, o:o + n] = b.S; T[o:o + n, o:o + n] = b.T; V[o:o + n, o:o + n] = b.V
        W[:, o:o + n, o:o + n] = b.W
        o += n
    return S, T, V, (W if twocomp else W[0]), Ns


@pytest.mark.parametrize("twocomp", [False, True])
def test_P11_block_diagonal_input_gives_block_h(twocomp):
    blocks = [atom_block(6), atom_block(8)]
    S, T, V, W, Ns = _combine(blocks, twocomp)
    H, _ = ox.x2c_direct(S, T, V, W, C, twocomp)
    N = sum(Ns)
    o = 0
    for b in blocks:
        hb, _ = ox.x2c_direct(*_args(b, twocomp), C, twocomp)
        n = b.N
        if twocomp:
            idx = np.r_[o:o + n, N + o:N + o + n]
        else:
            idx = np.arange(o, o + n)
        sub = H[np.ix_(idx, idx)]
        assert np.abs(sub - hb).max() <= 1e-12 * np.abs(hb).max()
        o += n
    # off-diagonal atom blocks vanish
    if not twocomp:
        assert np.abs(H[:Ns[0], Ns[0]:]).max() <= 1e-12 * np.abs(H).max()


# ---------------------------------------------------------------- P12 congruence covariance

@pytest.mark.parametrize("twocomp", [False, True])
def test_P12_congruence_covariance(twocomp):
    blk = atom_block(8)
    N = blk.N
    rng = np.random.default_rng(3)
    B = np.eye(N) + 0.05 * rng.standard_normal((N, N))
    tr = lambda M: B.T @ M @ B
    W2 = np.stack([tr(w) for w in blk.W])
    h, _ = ox.x2c_direct(*_args(blk, twocomp), C, twocomp)
    hB, _ = ox.x2c_direct(tr(blk.S), tr(blk.T), tr(blk.V), W2 if twocomp else W2[0], C, twocomp)
    Bx = oracle.spin_blockdiag(B) if twocomp else B
    ref = Bx.conj().T @ h @ Bx
    assert np.abs(hB - ref).max() <= 1e-11 * np.abs(ref).max()


# ---------------------------------------------------------------- P13 tiny brute force

@pytest.mark.parametrize("N,seed,twocomp", [(1, 0, False), (2, 1, False), (3, 2, True),
                                            (5, 4, True), (6, 5, False)])
def test_P13_tiny_random_brute_force(N, seed, twocomp):
    S, T, V, W = random_spd_problem(N, seed, twocomp)
    c = 7.0
    h, eps, parts = ox.x2c_direct(S, T, V, W, c, twocomp, return_parts=True)
    e4 = oracle.dirac_positive_spectrum(S, T, V, W, c, twocomp)
    e2 = oracle.spectrum_of(h, S, twocomp)
    sc = np.abs(e4).max()
    assert np.abs(e2 - e4).max() <= 1e-12 * sc
    h2, _ = ox.x2c_kbasis(S, T, V, W, c, twocomp)
    h3, _ = ox.x2c_polar(S, T, V, W, c, twocomp)
    assert np.abs(h - h2).max() <= 1e-12 * np.abs(h).max()
    assert np.abs(h - h3).max() <= 1e-12 * np.abs(h).max()
    Sx = oracle.spin_blockdiag(S) if twocomp else S
    R = parts["R"]
    assert np.abs(R.conj().T @ parts["St"] @ R - Sx).max() <= 1e-13 * np.abs(Sx).max()


def test_P13_one_by_one_closed_form():
    """N = 1 spin-free: the 2x2 pencil has a closed-form positive root and
    the 1x1 h (with S = 1) must equal it."""
    S = np.array([[1.0]]); T = np.array([[2.5]]); V = np.array([[-4.0]]); W = np.array([[-30.0]])
    c = 3.0
    h, eps = ox.x2c_direct(S, T, V, W, c, False)
    # det([[V - e, T], [T, W/4c^2 - T - e T/2c^2]]) = 0
    a = -T[0, 0] / (2 * c * c)
    wq = W[0, 0] / (4 * c * c) - T[0, 0]
    v = V[0, 0]; t = T[0, 0]
    # (v - e)(wq + a e) - t^2 = 0 -> -a e^2 + (v a - wq) e + v wq - t^2 = 0
    roots = np.roots([-a, v * a - wq, v * wq - t * t])
    e_pos = roots[roots + c * c > 0]
    assert e_pos.size == 1
    assert abs(h[0, 0] - e_pos[0]) < 1e-12 * abs(e_pos[0])
    assert abs(eps[0] - e_pos[0]) < 1e-12 * abs(e_pos[0])


# ---------------------------------------------------------------- errors

def test_positive_count_failure_raises():
    blk = atom_block(79)
    with pytest.raises(ox.X2CError):
        ox.x2c_direct(*_args(blk, False), 1.0, False)


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(twocomp):
    """A compact battery of the pins above; returns False if any fails."""
    blk = neon_s20() if not twocomp else atom_block(17)
    try:
        h, eps, parts = ox.x2c_direct(*_args(blk, twocomp), C, twocomp, return_parts=True)
        h2, _ = ox.x2c_kbasis(*_args(blk, twocomp), C, twocomp)
        h3, _ = ox.x2c_polar(*_args(blk, twocomp), C, twocomp)
    except Exception:
        return False
    s = np.abs(h).max()
    ok = np.abs(h - h2).max() <= 1e-12 * s and np.abs(h - h3).max() <= 1e-12 * s
    ok &= np.abs(h - h.conj().T).max() <= 1e-13 * s
    e4 = oracle.dirac_positive_spectrum(*_args(blk, twocomp), C, twocomp)
    e2 = oracle.spectrum_of(h, blk.S, twocomp)
    ok &= np.abs(e2 - e4).max() <= 1e-10 * np.abs(e4).max()
    if not twocomp:
        ok &= abs(eps[0] - dirac_1s(10.0, C) - 2.047e-3) < 5e-6
    else:
        e = np.sort(eps)
        Z = 17.0
        # the small Z=17 block is far from the basis limit for 2p; the
        # multiplet structure still pins the spin-orbit sign: 2p1/2 (pair)
        # below 2p3/2 (quartet)
        ok &= abs(e[0] - dirac_energy(Z, 1, -1, C)) < 0.2
        ok &= e[6] > e[5] + 1e-2 and abs(e[9] - e[6]) < 1e-9 * abs(e[6])
    return bool(ok)


MUTANTS = {
    "wx_sign_in_lower_block": ("assemble_w",
        lambda W0, Wx, Wy, Wz: _assemble_mut(W0, Wx, Wy, Wz, flip="wx_lower")),
    "spin_orbit_global_sign": ("assemble_w",
        lambda W0, Wx, Wy, Wz: _assemble_mut(W0, -Wx, -Wy, -Wz)),
    "kinetic_metric_factor": ("dirac_matrices", None),
    "positive_branch_threshold": ("positive_branch", None),
}


def _assemble_mut(W0, Wx, Wy, Wz, flip=None):
    W = ox.__dict__["_orig_assemble_w"](W0, Wx, Wy, Wz)
    N = W0.shape[0]
    if flip == "wx_lower":
        W[N:, :N] = -Wy - 1j * Wx
    return W


def _mut_dirac(S, T, V, W, c):
    D, M = _ORIG["dirac_matrices"](S, T, V, W, c)
    n = S.shape[0]
    M[n:, n:] = T / (c * c)            # planted: 1/c^2 instead of 1/2c^2
    return D, M


def _mut_branch(e, C_, c, n):
    keep = np.argsort(e)[:n]           # planted: keeps the lowest n
    return e[keep], C_[:, keep]


_ORIG = {}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_are_caught(name, monkeypatch):
    func, repl = MUTANTS[name]
    _ORIG["dirac_matrices"] = ox.dirac_matrices
    ox.__dict__["_orig_assemble_w"] = ox.assemble_w
    assert _pins_pass(twocomp=(func == "assemble_w"))
    if func == "dirac_matrices":
        repl = _mut_dirac
    elif func == "positive_branch":
        repl = _mut_branch
    monkeypatch.setattr(ox, func, repl)
    twocomp = func == "assemble_w"
    assert not _pins_pass(twocomp), f"mutant {name} survived the pins"


def test_golden_dirac_reference_table():
    """The stored Dirac-Coulomb table (written from the closed form) agrees
    with the formula and with the hand value for Z = 10 1s."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "dirac_reference.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 5
    for Z, n, k, E in rows:
        assert abs(dirac_energy(float(Z), int(n), int(k), C) - float(E)) < 1e-9
    z10 = [float(r[3]) for r in rows if r[:3] == ["10", "1", "-1"]][0]
    assert abs(z10 - (-50.066742016894)) < 1e-9
