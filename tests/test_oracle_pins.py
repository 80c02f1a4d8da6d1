"""Pins of the FP64 oracle against closed forms, exact invariants and brute
force (no GPU).  Each test names the property of the method or of the Yee
scheme it checks; none retypes the oracle's own formulas.
"""
import math

import numpy as np
import pytest

from oracle.oracle import OBJ_DFT, OBJ_TIME, OracleSim
from paper_2305_00234_amd import inputs as I
from tests.oracle_setup import oracle_from_workload

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C0 = 299792458.0


def _sim(n=(12, 12, 12), dx=5e-9, S=0.5, npml=0):
    return OracleSim(n[0], n[1], n[2], dx, S, npml)


# --------------------------------------------------------------------- P1
@pytest.mark.parametrize("rho", [0.0, 0.3, 1.0])
def test_p1_single_edge_response_is_ccpr_at_warped_frequency(rho):
    """Eq. CCPRModel with Eqs. eps_mixed/sigma_mixed/Poles_mixed: the impulse
    response of one edge with the curl switched off gives
    eps_meas(w) = -dt S(z)/(eps0 (z-1) E(z)), z = e^{jw dt}, which must equal
    the closed-form CCPR permittivity at the bilinear-warped frequency
    (2/dt) tan(w dt/2), for a mixture of Table-1 gold and a damped Lorentz
    dielectric with the conductivity damping gamma."""
    s = _sim()
    diel = I.lorentz(2.0, 1.5, 2 * math.pi * C0 / 300e-9, 3e14)
    for ax in range(3):
        s.set_material(1, ax, diel.eps_inf, diel.sigma, diel.a, diel.c)
        s.set_material(2, ax, I.GOLD_TABLE1.eps_inf, I.GOLD_TABLE1.sigma, I.GOLD_TABLE1.a,
                       I.GOLD_TABLE1.c)
    gamma = 5e4
    N = 120000
    src = np.zeros(N)
    src[0], src[1] = 1.0, -1.0  # zero net charge: E decays for any passive material
    E = s.edge_response(1, rho, gamma, src)
    assert abs(E[-1]) < 1e-14 * np.abs(E).max()  # decayed: the z-transform has converged
    dt = s.dt
    n = np.arange(E.size)
    for lam in (350e-9, 500e-9, 700e-9, 1000e-9):
        w = 2 * math.pi * C0 / lam
        z = np.exp(1j * w * dt)
        Ez = np.sum(E * z ** (-n))
        Sz = 1.0 - 1.0 / z
        eps_meas = -dt * Sz / (EPS0 * (z - 1) * Ez)
        wd = 2 / dt * math.tan(w * dt / 2)
        eps_exact = s.eps_ccpr(1, rho, gamma, wd)
        assert abs(eps_meas - eps_exact) <= 1e-9 * abs(eps_exact)
        # and it is close to the unwarped permittivity (second-order scheme)
        eps_unwarped = s.eps_ccpr(1, rho, gamma, w)
        assert abs(eps_meas - eps_unwarped) <= 2e-2 * abs(eps_unwarped)


# --------------------------------------------------------------------- P2
def test_p2_drude_lorentz_ccpr_mappings_match_textbook():
    """Drude eps_inf - wp^2/(w^2 - j w g) and Lorentz
    eps_inf + de w0^2/(w0^2 - w^2 + j w d), written in CCPR form, evaluate to
    the textbook formulas; Table-1 gold's first pair is Drude-like
    (sigma/eps0 close to -2 c_1)."""
    s = _sim()
    dr = I.drude(1.0, 1.37e16, 1e14)
    lo = I.lorentz(2.1, 1.0, 2 * math.pi * C0 / 150e-9, 1e14)
    s.set_material(1, 0, dr.eps_inf, dr.sigma, dr.a, dr.c)
    s.set_material(1, 1, lo.eps_inf, lo.sigma, lo.a, lo.c)
    for lam in (300e-9, 550e-9, 900e-9):
        w = 2 * math.pi * C0 / lam
        drude_tb = 1.0 - 1.37e16 ** 2 / (w ** 2 - 1j * w * 1e14)
        w0 = 2 * math.pi * C0 / 150e-9
        lor_tb = 2.1 + 1.0 * w0 ** 2 / (w0 ** 2 - w ** 2 + 1j * w * 1e14)
        assert abs(s.eps_ccpr(0, 0.0, 0.0, w) - drude_tb) <= 1e-12 * abs(drude_tb)
        assert abs(s.eps_ccpr(1, 0.0, 0.0, w) - lor_tb) <= 1e-12 * abs(lor_tb)
    g = I.GOLD_TABLE1
    assert abs(g.sigma / EPS0 - (-2 * g.c[0].real)) < 0.01 * abs(2 * g.c[0].real)


# --------------------------------------------------------------------- P3 / P5
def _tm_mode(sim, n, m, dx):
    """Ez = sin(kx x) sin(ky y), uniform in z (a PEC cavity eigenmode)."""
    nz, ny, nx = sim.shape
    i = np.arange(nx)[None, None, :]
    j = np.arange(ny)[None, :, None]
    kx, ky = m[0] * math.pi / nx, m[1] * math.pi / ny
    ez = np.sin(kx * i) * np.sin(ky * j) * np.ones((nz, 1, 1))
    return ez, (kx, ky, 0.0)


def _te_mode(sim, m):
    """E = curl(z psi), psi = cos(kx(i+1/2)) cos(ky(j+1/2)) sin(kz k) on the Hz
    points: divergence-free, zero tangential E on every wall."""
    nz, ny, nx = sim.shape
    kx, ky, kz = m[0] * math.pi / nx, m[1] * math.pi / ny, m[2] * math.pi / nz
    k = np.arange(nz)[:, None, None]
    j = np.arange(ny)[None, :, None]
    i = np.arange(nx)[None, None, :]

    def psi(ii, jj):
        return np.cos(kx * (ii + 0.5)) * np.cos(ky * (jj + 0.5)) * np.sin(kz * k)

    ex = psi(i, j) - psi(i, j - 1)
    ey = -(psi(i, j) - psi(i - 1, j))
    return ex, ey, (kx, ky, kz)


def _series(sim, comp, steps):
    vals = []
    for _ in range(steps + 1):
        vals.append(sim.field(comp))
        sim.run(1)
    return np.array(vals)


@pytest.mark.parametrize("mode", ["tm", "te"])
def test_p3_yee_vacuum_dispersion(mode):
    """A discrete PEC-cavity eigenmode obeys E^{n+1} + E^{n-1} = 2 cos(w dt) E^n
    with cos(w dt) = 1 - 2 S^2 sum_l sin^2(k_l dx/2) (Yee dispersion)."""
    S = 0.5
    sim = _sim(n=(10, 12, 14), S=S)
    if mode == "tm":
        ez, k = _tm_mode(sim, (2, 3), (2, 3), 5e-9)
        sim.set_field(2, ez)
        comp = 2
    else:
        ex, ey, k = _te_mode(sim, (2, 3, 4))
        sim.set_field(0, ex)
        sim.set_field(1, ey)
        comp = 1
    c = 1 - 2 * S ** 2 * sum(math.sin(kl / 2) ** 2 for kl in k)
    v = _series(sim, comp, 60)
    lhs = v[2:] + v[:-2]
    rhs = 2 * c * v[1:-1]
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(v))


def test_p5_cfl_nyquist_growth():
    """At S=0.5 the near-Nyquist mode stays bounded; at S=0.6 > 1/sqrt(3) it
    grows by |x - sqrt(x^2-1)| per step, x = 1 - 2 S^2 sum sin^2(k dx/2)."""
    for S, grows in ((0.5, False), (0.6, True)):
        sim = _sim(n=(8, 8, 8), S=S)
        ex, ey, k = _te_mode(sim, (7, 7, 7))
        sim.set_field(0, ex)
        sim.set_field(1, ey)
        x = 1 - 2 * S ** 2 * sum(math.sin(kl / 2) ** 2 for kl in k)
        v = np.linalg.norm(_series(sim, 1, 40).reshape(41, -1), axis=1)
        if grows:
            lam = abs(x - math.sqrt(x * x - 1))
            ratio = (v[40] / v[30]) ** (1 / 10)
            assert abs(ratio - lam) < 1e-6 * lam
        else:
            assert abs(x) <= 1
            assert np.max(v) <= 2.0 * v[0] and v[0] > 0


# --------------------------------------------------------------------- P4
def test_p4_energy_invariant_lossless_cavity():
    """Lossless PEC cavity with eps_inf(rho) only: the discrete Yee energy
    W^n = eps0/2 sum eps E^n.E^n + mu0/2 sum H^{n+1/2}.H^{n-1/2} is constant
    once the source is off."""
    sim = _sim(n=(12, 11, 10))
    for ax in range(3):
        sim.set_material(1, ax, 1.0)
        sim.set_material(2, ax, 4.0)
    rng = np.random.default_rng(5)
    rho = rng.random((4, 5, 6))
    lo = (3, 3, 3)
    sim.set_design(lo, rho, 0.0)
    t = (np.arange(30) + 0.5) * sim.dt
    sim.set_dipole((6, 5, 5), 2, I.gaussian_sine(t, 400e-9, 0.2e-15, 0.25e-15, amp=1e9))
    sim.run(40)
    eps = [np.ones(sim.shape) for _ in range(3)]
    for ax in range(3):
        eps[ax][3:7, 3:8, 3:9] = 1.0 + 3.0 * rho
    W = []
    for _ in range(400):
        E = [sim.field(c) for c in range(3)]
        Hm = [sim.field(3 + c) for c in range(3)]
        sim.run(1)
        Hp = [sim.field(3 + c) for c in range(3)]
        W.append(0.5 * EPS0 * sum(np.sum(eps[c] * E[c] ** 2) for c in range(3)) +
                 0.5 * MU0 * sum(np.sum(Hm[c] * Hp[c]) for c in range(3)))
    W = np.array(W)
    assert W[0] > 0
    assert np.max(np.abs(W - W[0])) <= 1e-11 * W[0]


def _stretch_lengths(N, npml, m, kmax):
    """Cell lengths (in units of dx) of the coordinate stretch that a lossless
    CPML (sigma = 0, alpha = 0) applies along one axis: kappa graded as
    1 + (kmax - 1) xi^m, xi the depth into a layer of npml cells over npml,
    at the integer nodes q (dual lengths D) and at q + 1/2 (primal lengths L)."""
    def kappa(pos):
        d = np.maximum(npml - pos, pos - (N - npml))
        xi = np.clip(d, 0.0, npml) / npml
        return 1.0 + (kmax - 1.0) * xi ** m
    q = np.arange(N, dtype=np.float64)
    return kappa(q), kappa(q + 0.5)


def test_p4_energy_invariant_kappa_stretched_cpml():
    """A CPML with sigma = 0 and alpha = 0 leaves only the kappa grading, a
    real, lossless stretch of the coordinates: the Yee scheme on cells of
    primal lengths L = kappa(q + 1/2) dx and dual lengths D = kappa(q) dx.
    That scheme conserves W = eps0/2 sum V_E E.E + mu0/2 sum V_H H+.H- with
    E_c weighted by L_c D_d1 D_d2 and H_c by D_c L_d1 L_d2 (summation by parts
    against the PEC walls), so once the source is off W is constant.  A kappa
    at the wrong staggered position, on the wrong derivative, multiplied
    instead of divided, or graded differently, breaks the invariant."""
    n = (14, 13, 12)
    npml, m, kmax = 4, 3.0, 5.0
    sim = OracleSim(n[0], n[1], n[2], 5e-9, 0.5, npml, m, kmax, 0.0, 0.0)
    t = (np.arange(30) + 0.5) * sim.dt
    sim.set_dipole((7, 6, 6), 2, I.gaussian_sine(t, 400e-9, 0.2e-15, 0.25e-15, amp=1e9))
    sim.run(40)
    D, L = zip(*(_stretch_lengths(n[a], npml, m, kmax) for a in range(3)))

    def vol(lengths):  # (x, y, z) length arrays -> (z, y, x) cell volumes
        return lengths[2][:, None, None] * lengths[1][None, :, None] * lengths[0][None, None, :]
    VE = [vol([L[0], D[1], D[2]]), vol([D[0], L[1], D[2]]), vol([D[0], D[1], L[2]])]
    VH = [vol([D[0], L[1], L[2]]), vol([L[0], D[1], L[2]]), vol([L[0], L[1], D[2]])]
    W = []
    for _ in range(300):
        E = [sim.field(c) for c in range(3)]
        Hm = [sim.field(3 + c) for c in range(3)]
        sim.run(1)
        Hp = [sim.field(3 + c) for c in range(3)]
        W.append(0.5 * EPS0 * sum(np.sum(VE[c] * E[c] ** 2) for c in range(3)) +
                 0.5 * MU0 * sum(np.sum(VH[c] * Hm[c] * Hp[c]) for c in range(3)))
    W = np.array(W)
    assert W[0] > 0
    assert np.max(np.abs(W - W[0])) <= 1e-11 * W[0]
    # the uniform-grid weights do not make it an invariant: the stretch is real
    W1 = []
    sim2 = OracleSim(n[0], n[1], n[2], 5e-9, 0.5, npml, m, kmax, 0.0, 0.0)
    sim2.set_dipole((7, 6, 6), 2, I.gaussian_sine(t, 400e-9, 0.2e-15, 0.25e-15, amp=1e9))
    sim2.run(40)
    for _ in range(300):
        E = [sim2.field(c) for c in range(3)]
        Hm = [sim2.field(3 + c) for c in range(3)]
        sim2.run(1)
        Hp = [sim2.field(3 + c) for c in range(3)]
        W1.append(0.5 * EPS0 * sum(np.sum(E[c] ** 2) for c in range(3)) +
                  0.5 * MU0 * sum(np.sum(Hm[c] * Hp[c]) for c in range(3)))
    W1 = np.array(W1)
    assert np.max(np.abs(W1 - W1[0])) > 1e-6 * W1[0]


def test_p14_cpml_static_limit_is_a_stretched_electrostatic_field():
    """The static limit of the CFS-CPML recursion.  In steady state the
    memory of a constant derivative d settles at psi = a d / (1 - b), so every
    derivative along an axis is scaled by 1/kappa + a/(1 - b), which the
    CFS stretch s(w) = kappa + sigma/(alpha + j w eps0) fixes at w = 0:
    1/s0 = alpha / (sigma + kappa alpha), at each field's staggered position.
    A current pulse with a nonzero time integral leaves a static charge pair,
    so once the radiation has died out E must be the discrete electrostatic
    field of that pair on the grid stretched by s0: E = -grad phi with
    eps0 div grad phi = dt div S (S = the summed source on its edge), the
    gradient along c at half-integer positions, the divergence at the nodes,
    phi = 0 on the PEC walls.  Checked against a sparse solve of that Poisson
    problem.  A wrong sigma, kappa or alpha profile, a wrong a or b, or a
    half-cell shift of the CPML coefficients changes the field."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    N, npml, m, kmax, amax, dx = 16, 4, 3.0, 3.0, 2e4, 5e-9
    sim = OracleSim(N, N, N, dx, 0.5, npml, m, kmax, amax, 1.0)
    dt = sim.dt
    t = (np.arange(60) + 0.5) * dt
    wave = 1e9 * np.exp(-((t - 30 * dt) / (8 * dt)) ** 2)   # nonzero time integral
    src = (7, 6, 6)
    sim.set_dipole(src, 2, wave)
    sim.run(8000)

    # the static stretch 1/s0 of the CFS profile (sigma_max = 0.8 (m + 1) / (eta0 dx))
    def inv_s0(pos):
        xi = np.clip(np.maximum(npml - pos, pos - (N - npml)), 0.0, npml) / npml
        smax = 0.8 * (m + 1.0) / (math.sqrt(MU0 / EPS0) * dx)
        sig, kap, al = smax * xi ** m, 1.0 + (kmax - 1.0) * xi ** m, amax * (1.0 - xi)
        return al / (sig + kap * al)
    q = np.arange(N + 1, dtype=np.float64)
    h, g = inv_s0(q), inv_s0(q + 0.5)   # nodes; edges (half-integer)
    n1 = N - 1                           # unknown nodes 1 .. N-1 per axis

    def nid(p):
        return ((p[2] - 1) * n1 + (p[1] - 1)) * n1 + (p[0] - 1)
    rows, cols, vals = [], [], []
    for p in np.ndindex(n1, n1, n1):
        p = (p[0] + 1, p[1] + 1, p[2] + 1)
        r, diag = nid(p), 0.0
        for c in range(3):
            for sgn in (1, -1):
                w = h[p[c]] * g[p[c] if sgn > 0 else p[c] - 1] / dx ** 2
                diag -= w
                nb = list(p)
                nb[c] += sgn
                if 1 <= nb[c] <= N - 1:
                    rows.append(r)
                    cols.append(nid(nb))
                    vals.append(w)
        rows.append(r)
        cols.append(r)
        vals.append(diag)
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n1 ** 3, n1 ** 3))
    b = np.zeros(n1 ** 3)
    Ssum = dt / EPS0 * wave.sum()
    b[nid(src)] += Ssum * h[src[2]] / dx
    b[nid((src[0], src[1], src[2] + 1))] -= Ssum * h[src[2] + 1] / dx
    phi = np.zeros((N + 1, N + 1, N + 1))   # [i, j, k]; zero on the walls
    phi[1:N, 1:N, 1:N] = spl.spsolve(A, b).reshape(n1, n1, n1).transpose(2, 1, 0)
    num = den = 0.0
    for c in range(3):
        sl = [slice(0, N)] * 3
        up = [slice(0, N)] * 3
        up[c] = slice(1, N + 1)
        shape = [1, 1, 1]
        shape[c] = N
        Ec = -(phi[tuple(up)] - phi[tuple(sl)]) * g[:N].reshape(shape) / dx   # [i, j, k]
        Ec = Ec.transpose(2, 1, 0)                                           # (z, y, x)
        num += np.sum((sim.field(c) - Ec) ** 2)
        den += np.sum(Ec ** 2)
    err = math.sqrt(num / den)
    assert den > 0 and err <= 1e-9, err


def test_p14_cpml_recursion_integrates_the_cfs_kernel_exactly():
    """The CFS stretch s(w) = kappa + sigma/(alpha + j w eps0) turns a
    derivative into d/kappa + zeta * d with the causal kernel
    zeta(t) = -sigma/(eps0 kappa^2) exp(-(sigma/kappa + alpha) t/eps0).  The
    recursion psi^n = b psi^{n-1} + a d^n convolves d with the taps a b^m, and
    for a derivative held over each step these taps must be the kernel's
    integrals over [m dt, (m+1) dt]: checked for m = 0, 1, 10, 100 at every
    staggered position of a graded CPML (which also fixes the decay per step
    b, a quantity the static-limit pin does not see)."""
    n, npml, m, kmax, amax, dx = 20, 6, 3.0, 4.0, 0.3, 5e-9
    sim = OracleSim(n, n, n, dx, 0.5, npml, m, kmax, amax, 1.2)
    dt = sim.dt
    smax = 1.2 * 0.8 * (m + 1.0) / (math.sqrt(MU0 / EPS0) * dx)
    checked = 0
    for axis in range(3):
        for half in (False, True):
            b, a, kap = sim.pml_coefficients(axis, half)
            pos = np.arange(n) + (0.5 if half else 0.0)
            xi = np.clip(np.maximum(npml - pos, pos - (n - npml)), 0.0, npml) / npml
            sig, k_ref, al = smax * xi ** m, 1.0 + (kmax - 1.0) * xi ** m, amax * (1.0 - xi)
            assert np.allclose(kap, k_ref, rtol=1e-14, atol=0)
            rate = (sig / k_ref + al) / EPS0
            for q in range(n):
                if sig[q] == 0.0:
                    assert a[q] == 0.0
                    continue
                for mm in (0, 1, 10, 100):
                    tap = a[q] * b[q] ** mm
                    integral = -sig[q] / (EPS0 * k_ref[q] ** 2) * (
                        math.exp(-rate[q] * mm * dt) - math.exp(-rate[q] * (mm + 1) * dt)) / rate[q]
                    assert tap == pytest.approx(integral, rel=1e-10, abs=0), (axis, half, q, mm)
                checked += 1
    assert checked >= 3 * 2 * 2 * (npml - 1)


# --------------------------------------------------------------------- P6
def test_p6_reciprocity_with_dispersive_inclusion():
    """Reciprocal medium: E_x at B driven by J_x at A equals E_x at A driven by
    J_x at B (same waveform), with a lossy Drude / gold inclusion."""
    A, B = (3, 4, 5), (8, 6, 4)

    def run(src, rec):
        sim = _sim(n=(12, 11, 10))
        for ax in range(3):
            sim.set_material(2, ax, I.GOLD_TABLE1.eps_inf, I.GOLD_TABLE1.sigma,
                             I.GOLD_TABLE1.a, I.GOLD_TABLE1.c)
        rng = np.random.default_rng(9)
        sim.set_design((4, 3, 3), rng.random((4, 5, 4)), 5e4)
        t = (np.arange(200) + 0.5) * sim.dt
        sim.set_dipole(src, 0, I.gaussian_sine(t, 500e-9, 0.5e-15, 0.8e-15, amp=1e9))
        out = []
        for _ in range(200):
            sim.run(1)
            out.append(sim.field(0)[rec[2], rec[1], rec[0]])
        return np.array(out)

    ab = run(A, B)
    ba = run(B, A)
    assert np.max(np.abs(ab)) > 0
    assert np.max(np.abs(ab - ba)) <= 1e-11 * np.max(np.abs(ab))


# --------------------------------------------------------------------- P7
def test_p7_objective_quadratic_in_amplitude():
    w = I.drude_dipole_32(steps=60, n=20, npml=4)
    f1 = oracle_from_workload(w).objective(60, OBJ_DFT, w.gap_lo, w.gap_dims, w.omega)
    w.wave = 3.0 * w.wave
    f3 = oracle_from_workload(w).objective(60, OBJ_DFT, w.gap_lo, w.gap_dims, w.omega)
    assert f1 > 0
    assert abs(f3 / f1 - 9.0) < 1e-12


# --------------------------------------------------------------------- P8 / P9
def _fd_check(w, kind, voxels, h=1e-4):
    s = oracle_from_workload(w)
    F, g = s.gradient(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], w.window_end)
    rho0 = w.rho.astype(np.float64)
    fd = []
    for (z, y, x) in voxels:
        vals = []
        for sgn in (+1, -1):
            r = rho0.copy()
            r[z, y, x] += sgn * h
            s2 = oracle_from_workload(w)
            s2.set_design(w.design_lo, r, w.gamma)
            vals.append(s2.objective(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0],
                                     w.window_end))
        fd.append((vals[0] - vals[1]) / (2 * h))
    fd = np.array(fd)
    ad = np.array([g[v] for v in voxels])
    return F, ad, fd


def _small_pec(objective, gamma=5e4, nondispersive=False, steps=160):
    w = I.drude_dipole_32(steps=steps, n=14, npml=0, gamma=gamma)
    rng = np.random.default_rng(11)
    w.design_lo = (4, 4, 4)
    w.rho = rng.random((5, 6, 5)).astype(np.float32)
    w.gap_lo, w.gap_dims = (6, 6, 6), (2, 2, 2)
    w.rho[2:4, 2:4, 2:4] = 0.0
    w.dipole_cell = (2, 7, 7)
    if nondispersive:
        w.mat1 = (I.CCPRMaterial(1.0),) * 3
        w.mat2 = (I.CCPRMaterial(3.5),) * 3
    else:
        diel = I.lorentz(2.0, 1.2, 2 * math.pi * C0 / 250e-9, 2e14)
        w.mat1 = (diel, diel, diel)
        w.mat2 = (I.GOLD_TABLE1, I.ALUMINIUM_TABLE1, I.GOLD_TABLE1)
    w.objective = objective
    if objective == "time":
        w.window = (20, steps - 10)
    return w


@pytest.mark.parametrize("objective", ["dft", "time"])
def test_p8_adjoint_gradient_matches_central_fd_pec(objective):
    """Brute force: the time-exact adjoint gradient equals central finite
    differences of the objective (PEC box, two dispersive materials with
    diagonal anisotropy, conductivity damping gamma)."""
    w = _small_pec(objective)
    kind = OBJ_DFT if objective == "dft" else OBJ_TIME
    rng = np.random.default_rng(12)
    vox = [tuple(int(rng.integers(0, s)) for s in w.rho.shape) for _ in range(10)]
    F, ad, fd = _fd_check(w, kind, vox)
    assert F > 0
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    assert err < 1e-6, (err, ad, fd)


def test_p9_nondispersive_special_case():
    """Only eps_inf differs between the materials (no sigma, no poles): the
    gradient still matches finite differences (it reduces to the first term of
    Eq. Gradient_analytic)."""
    w = _small_pec("dft", gamma=0.0, nondispersive=True)
    vox = [(0, 0, 0), (1, 2, 3), (4, 5, 4), (2, 1, 0)]
    F, ad, fd = _fd_check(w, OBJ_DFT, vox)
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    assert err < 1e-6, (err, ad, fd)


@pytest.mark.slow
def test_p8_cpml_gradient_vs_fd_reported():
    """With the CPML the forward update is reused for the adjoint (as the paper
    does), which is not its exact transpose inside the absorbing layer: the
    gradient matches finite differences only up to that mismatch."""
    w = I.drude_dipole_32(steps=400)
    rng = np.random.default_rng(100)
    vox = [tuple(int(rng.integers(0, 8)) for _ in range(3)) for _ in range(8)]
    F, ad, fd = _fd_check(w, OBJ_DFT, vox)
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    print("cpml gradient vs fd rel err", err)
    assert err < 1e-5


# --------------------------------------------------------------------- P11
def test_p11_tfsf_leakage_empty_grid():
    """Axis-aligned TF/SF with an exact 1-D incident line: the scattered-field
    region of an empty grid stays at round-off."""
    for prop, sign, pol in ((2, 1, 0), (0, -1, 1), (1, 1, 2)):
        sim = _sim(n=(24, 22, 26))
        t = np.arange(200) * sim.dt
        sim.set_planewave(prop, sign, pol, (5, 6, 5), (18, 16, 20),
                          I.gaussian_sine(t, 300e-9, 0.4e-15, 1.0e-15))
        sim.run(150)
        inside = np.zeros(sim.shape, dtype=bool)
        inside[4:22, 5:18, 4:20] = True  # generous total-field box incl. its faces
        peak = max(np.max(np.abs(sim.field(c))) for c in range(3))
        leak = max(np.max(np.abs(sim.field(c)[~inside])) for c in range(3))
        assert peak > 0.1
        assert leak <= 1e-12 * peak, (prop, sign, pol, leak, peak)


# --------------------------------------------------------------------- P14
def test_p14_cpml_reflection_below_40db():
    """Bound only: a dipole pulse in a grid with an 8-cell CPML versus the same
    region cut from a grid large enough that nothing returns in time."""
    steps = 140
    t = (np.arange(steps) + 0.5) * 5e-9 * 0.5 / C0
    wave = I.gaussian_sine(t, 200e-9, 0.3e-15, 0.45e-15, amp=1e9)

    def probe(n, npml):
        sim = OracleSim(n, n, n, 5e-9, 0.5, npml)
        c = n // 2
        sim.set_dipole((c, c, c), 2, wave)
        out = []
        for _ in range(steps):
            sim.run(1)
            out.append(sim.field(2)[c, c, c + 10])
        return np.array(out)

    small = probe(36, 8)
    big = probe(96, 8)
    refl = np.max(np.abs(small - big)) / np.max(np.abs(big))
    print("cpml reflection", 20 * math.log10(refl), "dB")
    assert refl < 1e-2


# --------------------------------------------------------------------- P13
def _short_pulse_dipole(M, n=24, npml=5, lam=500e-9, fwhm=2e-15, t0=4e-15):
    w = I.drude_dipole_32(steps=M, n=n, npml=npml)
    t = (np.arange(M) + 0.5) * w.dt
    w.wave = I.gaussian_sine(t, lam, fwhm, t0)
    w.omega = 2 * math.pi * C0 / lam
    return w


def test_p13_dft_mode_gradient_tends_to_time_exact():
    """The single-frequency (DFT-mode) gradient estimator replaces the adjoint
    field by its steady state Re{A e^{j w dt m}}.  With a 2 fs pulse that has
    left the domain, the estimate must converge to the exact discrete gradient
    as the run lengthens (the adjoint transient overlaps less and less of the
    forward response): the relative error falls at every doubling and ends
    below 1e-4.  A wrong phase convention, window or pairing (e.g. an
    off-by-one step, about 6% at w dt = 0.063) cannot converge."""
    errs = []
    for M in (2000, 4000, 8000):
        w = _short_pulse_dipole(M)
        s = oracle_from_workload(w)
        F1, g_exact = s.gradient(M, OBJ_DFT, w.gap_lo, w.gap_dims, w.omega)
        F2, g_dft = s.gradient_dft(M, w.gap_lo, w.gap_dims, w.omega)
        assert F1 == F2
        errs.append(float(np.linalg.norm(g_dft - g_exact) / np.linalg.norm(g_exact)))
    print("P13 DFT-mode vs time-exact, M = 2000, 4000, 8000:", errs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4


def test_p13_dft_window_whole_periods():
    """Fit window: the whole periods that fit in half the run."""
    dt = 1e-17
    w = 2 * math.pi / (100 * dt)        # 100 steps per period
    assert OracleSim.dft_window(1000, w, dt) == 500
    assert OracleSim.dft_window(1099, w, dt) == 500
    assert OracleSim.dft_window(1250, w, dt) == 600
    assert OracleSim.dft_window(150, w, dt) == 75   # under one period: half the run


# ------------------------------------------------ per-edge design variables
def _edge_fd_check(w, kind, edges, h=1e-4):
    """Adjoint gradient of a per-edge design against central differences at
    the given (component, z, y, x) edges."""
    s = oracle_from_workload(w)
    F, g = s.gradient(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], w.window_end)
    base = [r.astype(np.float64) for r in w.rho_edges]
    fd = []
    for (c, z, y, x) in edges:
        vals = []
        for sgn in (+1, -1):
            r = [b.copy() for b in base]
            r[c][z, y, x] += sgn * h
            s2 = oracle_from_workload(w)
            s2.set_design_edges(w.design_lo, w.design_dims, r, w.gamma)
            vals.append(s2.objective(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0],
                                     w.window_end))
        fd.append((vals[0] - vals[1]) / (2 * h))
    return F, np.array([g[c][z, y, x] for (c, z, y, x) in edges]), np.array(fd)


@pytest.mark.parametrize("objective", ["dft", "time"])
def test_p8_edge_gradient_matches_central_fd_pec(objective):
    """Brute force for one density per E edge (Sec. "FDTD implementation and
    design export"): the adjoint gradient equals central differences, also on
    the extra edges of the box's far faces (N_l + 1 along the transverse
    axes), which a per-voxel layout does not have."""
    w = _small_pec(objective)
    dims = w.design_dims
    w.rho_edges = I.random_edge_densities(dims, seed=21)
    for r in w.rho_edges:   # the gap cells stay air
        r[2:4, 2:4, 2:4] = 0.0
    nx, ny, nz = dims
    edges = [(0, nz, ny, 1), (0, 0, ny, 3), (0, nz, 2, 4),      # x edges on the far y / z faces
             (1, nz, 3, nx), (1, 2, 0, nx),                      # y edges on the far x / z faces
             (2, 1, ny, nx), (2, 4, ny, 0),                      # z edges on the far x / y faces
             (0, 1, 1, 1), (1, 3, 2, 2), (2, 2, 4, 3)]           # interior edges
    F, ad, fd = _edge_fd_check(w, OBJ_DFT if objective == "dft" else OBJ_TIME, edges)
    assert F > 0
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    assert err < 1e-6, (err, ad, fd)


def test_edge_design_reduces_to_voxel_design():
    """Per-edge densities equal to a per-voxel design on the edges each voxel
    owns, and 0 on the far-face edges with a vacuum rho=0 material, give the
    same fields: the objective agrees and each voxel's gradient is the sum of
    its three edges' gradients (the voxel density drives all three)."""
    w = _small_pec("dft")
    w.mat1 = (I.CCPRMaterial(1.0),) * 3
    s = oracle_from_workload(w)
    F_v, g_v = s.gradient(w.steps, OBJ_DFT, w.gap_lo, w.gap_dims, w.omega)
    w.rho_edges = I.voxel_edge_densities(w.rho, fill=0.0)
    s = oracle_from_workload(w)
    F_e, g_e = s.gradient(w.steps, OBJ_DFT, w.gap_lo, w.gap_dims, w.omega)
    nz, ny, nx = w.rho.shape
    summed = sum(g[:nz, :ny, :nx] for g in g_e)
    assert F_e == pytest.approx(F_v, rel=1e-13, abs=0)
    assert np.max(np.abs(summed - g_v)) <= 1e-12 * np.max(np.abs(g_v))


# --------------------------------------------------------------------- P10
def _diag_symmetric_case(per_edge, objective):
    """Problem invariant under the mirror x <-> y (the plane x = y): square
    grid and CPML, design and gap boxes on the diagonal, identical x and y
    materials (z differs), a z dipole on the diagonal.  The mirror maps the
    Yee lattice onto itself, E_x edges onto E_y edges and E_z onto E_z."""
    w = I.drude_dipole_32(steps=150, n=16, npml=3, gamma=5e4)
    w.shape = (16, 16, 14)
    diel = I.lorentz(2.0, 1.2, 2 * math.pi * C0 / 250e-9, 2e14)
    w.mat1 = (diel, diel, diel)
    w.mat2 = (I.GOLD_TABLE1, I.GOLD_TABLE1, I.ALUMINIUM_TABLE1)
    w.design_lo = (5, 5, 4)
    dims = (6, 6, 5)
    rng = np.random.default_rng(31)
    a = rng.random((dims[2], dims[1], dims[0]))
    w.rho = (0.5 * (a + a.transpose(0, 2, 1))).astype(np.float32)
    w.gap_lo, w.gap_dims = (7, 7, 5), (2, 2, 2)
    w.dipole_cell, w.dipole_axis = (3, 3, 6), 2
    if per_edge:
        ex, _, ez = I.random_edge_densities(dims, seed=32)
        ey = np.ascontiguousarray(ex.transpose(0, 2, 1))
        ez = (0.5 * (ez + ez.transpose(0, 2, 1))).astype(np.float32)
        w.rho_edges = (ex, ey, ez)
    w.objective = objective
    if objective == "time":
        w.window = (10, 140)
    return w


@pytest.mark.parametrize("per_edge", [False, True])
@pytest.mark.parametrize("objective", ["dft", "time"])
def test_p10_mirror_symmetric_problem_has_mirror_symmetric_gradient(per_edge, objective):
    """Invariant: with a design, sources, gap and materials symmetric under
    x <-> y, the objective is symmetric, so its gradient is too: per voxel
    g(k, j, i) = g(k, i, j); per edge g_x(k, j, i) = g_y(k, i, j) and g_z
    symmetric.  An index or sign slip on one transverse axis (a curl term, a
    CPML coefficient, an edge box extent) breaks it."""
    w = _diag_symmetric_case(per_edge, objective)
    s = oracle_from_workload(w)
    kind = OBJ_DFT if objective == "dft" else OBJ_TIME
    F, g = s.gradient(w.steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], w.window_end)
    assert F > 0
    if per_edge:
        gx, gy, gz = g
        scale = max(np.max(np.abs(x)) for x in g)
        assert np.max(np.abs(gx - gy.transpose(0, 2, 1))) <= 1e-10 * scale
        assert np.max(np.abs(gz - gz.transpose(0, 2, 1))) <= 1e-10 * scale
    else:
        assert np.max(np.abs(g - g.transpose(0, 2, 1))) <= 1e-10 * np.max(np.abs(g))


# ------------------------------------------------------- objectives (Eq. 2)
def _gap_dipole_case(M=47):
    """Small CPML grid, Drude design, dipole beside it, 2^3 gap."""
    w = I.drude_dipole_32(steps=M, n=16, npml=3)
    t = (np.arange(M) + 0.5) * w.dt
    w.wave = I.gaussian_sine(t, 300e-9, 0.8e-15, 1.0e-15, amp=1e9)
    return w


def test_objectives_parseval_identity():
    """The single-frequency objective F_dft(w) = sum_e |dt sum_{n=0..M} E_e^n
    e^{-j w n dt}|^2 and the time-domain objective of Eq. 2 (rectangle rule,
    eps_inf = 1 in the gap) over the whole run [0, M+1) are tied by
    Parseval's identity for the DFT of length M+1: at the M+1 frequencies
    w_k = 2 pi k / ((M+1) dt),
        sum_k F_dft(w_k) = 2 (M+1) dt F_time / (eps0 dx^3).
    A dropped or extra sample in either sum, a missing dt in the transform, a
    wrong eps0/2, dx^3 or dt in Eq. 2 or a shifted time window breaks it."""
    M = 47
    w = _gap_dipole_case(M)
    dt = w.dt
    ft = oracle_from_workload(w).objective(M, OBJ_TIME, w.gap_lo, w.gap_dims, 0.0, 0, M + 1)
    assert ft > 0
    tot = 0.0
    for k in range(M + 1):
        wk = 2 * math.pi * k / ((M + 1) * dt)
        tot += oracle_from_workload(w).objective(M, OBJ_DFT, w.gap_lo, w.gap_dims, wk)
    expect = 2 * (M + 1) * dt * ft / (EPS0 * w.dx ** 3)
    assert abs(tot - expect) <= 1e-11 * expect, (tot, expect)


def test_time_objective_window_samples_the_state_after_n_steps():
    """Eq. 2's window [n_begin, n_end) samples E^n, the field after n steps
    (n = 0 is the zero initial state, n = M the last one): a one-sample
    window [n, n+1) equals (eps0/2) dx^3 dt sum over the gap edges of
    (E^n)^2 taken from the field state after n steps, and the windows
    partition the run (additivity)."""
    M = 47
    w = _gap_dipole_case(M)
    sim = oracle_from_workload(w)
    lo, dims = w.gap_lo, w.gap_dims
    wgt = 0.5 * EPS0 * w.dx ** 3 * w.dt

    def window(a, b):
        return oracle_from_workload(w).objective(M, OBJ_TIME, lo, dims, 0.0, a, b)

    sl = (slice(lo[2], lo[2] + dims[2]), slice(lo[1], lo[1] + dims[1]), slice(lo[0], lo[0] + dims[0]))
    for n in (20, 33, M):
        sim.reset()
        sim.run(n)
        e2 = sum(float(np.sum(sim.field(c)[sl] ** 2)) for c in range(3))
        assert e2 > 0
        assert window(n, n + 1) == pytest.approx(wgt * e2, rel=1e-12, abs=0)
    assert window(0, 1) == 0.0
    whole = window(0, M + 1)
    for a in (1, 17, 30, M):
        assert window(0, a) + window(a, M + 1) == pytest.approx(whole, rel=1e-12, abs=0)


# ------------------------------------------------ TF/SF incident amplitude
def _line_1d(wave, steps, L, S):
    """Textbook 1-D Yee line in SI units with the same dx, dt (Courant S):
    E at integer points u, H at u + 1/2, hard source E[0]^n = wave[n];
    eps0 dE/dt = -dH/du, mu0 dH/dt = -dE/du, so a wave moving to +u has
    H = E / eta0.  Returns E^n[u] and H^{n+1/2}[u] for n = 0..steps."""
    eta0 = math.sqrt(MU0 / EPS0)
    E = np.zeros(L + 1)
    H = np.zeros(L)
    E[0] = wave[0]
    Es, Hs = [E.copy()], []
    for n in range(steps):
        H -= (S / eta0) * (E[1:] - E[:-1])
        E[1:-1] -= (S * eta0) * (H[1:] - H[:-1])
        E[0] = wave[n + 1] if n + 1 < len(wave) else 0.0
        Hs.append(H.copy())
        Es.append(E.copy())
    return np.array(Es), np.array(Hs)


@pytest.mark.parametrize("prop,sign,pol", [(2, 1, 0), (0, -1, 1), (1, 1, 2), (2, -1, 1)])
def test_tfsf_total_field_equals_incident_wave(prop, sign, pol):
    """In an empty grid the total field inside the TF/SF box is the incident
    plane wave alone.  Its amplitude, sign and timing are fixed by the
    source's definition -- wave[n] is E_pol at the launch point two cells
    before the box (along the direction of travel) at t = n dt -- and by
    Maxwell's equations: E_pol(x_d) is the 1-D Yee line's E at distance
    sign*(x_d - x_launch) and H_t = sign * levi(pol, t, prop) * H_line (the
    Poynting vector points along sign * prop).  The line here is this test's
    own.  A scaled, sign-flipped, shifted or mis-polarised incident wave
    fails; the leakage pin (P11) alone would not see those."""
    n3 = (26, 22, 28)
    lo, hi = (5, 6, 5), (19, 15, 21)
    sim = _sim(n=n3)
    steps = 110
    t = np.arange(steps + 1) * sim.dt
    wave = I.gaussian_sine(t, 300e-9, 0.5e-15, 1.2e-15)
    sim.set_planewave(prop, sign, pol, lo, hi, wave)
    tr = 3 - prop - pol
    lev = 1 if (pol, tr, prop) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1
    launch = lo[prop] - 2 if sign > 0 else hi[prop] + 2
    Es, Hs = _line_1d(wave, steps, 80, 0.5)
    c0 = [(lo[a] + hi[a]) // 2 for a in range(3)]
    peakE = np.max(np.abs(Es))
    peakH = np.max(np.abs(Hs))
    seen = 0.0
    for n in (40, 70, steps):
        sim.reset()
        sim.run(n)
        Ef = sim.field(pol)
        Hf = sim.field(3 + tr)
        for q in range(lo[prop] + 1, hi[prop]):
            cell = list(c0)
            cell[prop] = q
            z, y, x = cell[2], cell[1], cell[0]
            # E_pol (pol != prop) sits at the integer coordinate q along prop;
            # H_t at q + 1/2
            uE = sign * (q - launch)
            assert abs(Ef[z, y, x] - Es[n, uE]) <= 1e-12 * peakE, (n, q, Ef[z, y, x], Es[n, uE])
            seen = max(seen, abs(Es[n, uE]))
            uH = q - launch if sign > 0 else launch - q - 1   # H_line[u] sits at u + 1/2
            h_ref = sign * lev * Hs[n - 1, uH]
            assert abs(Hf[z, y, x] - h_ref) <= 1e-12 * peakH, (n, q, Hf[z, y, x], h_ref)
    assert seen > 0.5 * peakE   # the pulse crossed the compared points


# ---------------------------------------------- P14 with a stretched CPML
def test_p14_cpml_reflection_with_kappa_grading():
    """Bound only, with a non-default grading that exercises every CPML term:
    kappa_max = 5 (the 1/kappa scaling of the differences), alpha_max = 0.1,
    polynomial order 4 and a 1.2x conductivity: still below -40 dB against a
    grid large enough that nothing returns in time.  A kappa used as
    kappa instead of 1/kappa, or applied to the wrong axis, reflects far
    more."""
    steps = 140
    t = (np.arange(steps) + 0.5) * 5e-9 * 0.5 / C0
    wave = I.gaussian_sine(t, 200e-9, 0.3e-15, 0.45e-15, amp=1e9)

    def probe(n, npml):
        sim = OracleSim(n, n, n, 5e-9, 0.5, npml, 4.0, 5.0, 0.1, 1.2)
        c = n // 2
        sim.set_dipole((c, c, c), 2, wave)
        out = []
        for _ in range(steps):
            sim.run(1)
            out.append(np.array([sim.field(2)[c, c, c + 10], sim.field(2)[c + 9, c - 9, c]]))
        return np.array(out)

    small = probe(36, 8)
    big = probe(96, 8)
    refl = np.max(np.abs(small - big)) / np.max(np.abs(big))
    print("cpml (kappa 5, alpha 0.1, m 4) reflection", 20 * math.log10(refl), "dB")
    assert refl < 1e-2
