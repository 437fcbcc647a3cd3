"""Pins of the oracle's solvent: D3Q19 lattice, BGK collision with Guo forcing,
streaming.  Each check compares against something the lattice-Boltzmann
theory or plain mechanics fixes, not against the oracle's own formulas."""
import math

import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I

EPS = np.finfo(np.float64).eps


def test_d3q19_isotropy():
    # moments of the discrete velocity set up to fourth order equal those of
    # the Maxwellian with c_s^2 = 1/3 (textbook D3Q19 property)
    c, w = oracle.lattice()
    c = c.astype(np.float64)
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    assert np.allclose(w @ c, 0.0, atol=1e-15)
    M2 = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(M2, np.eye(3) / 3.0, atol=1e-15)
    M3 = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.allclose(M3, 0.0, atol=1e-15)
    M4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(M4, iso, atol=1e-15)
    # numbering: 0 at rest, (odd i, i+1) opposite pairs, 6 faces then 12 edges
    assert np.all(c[0] == 0)
    for i in range(1, 19, 2):
        assert np.all(c[i] == -c[i + 1])
    assert np.all(np.abs(c[1:7]).sum(axis=1) == 1)
    assert np.all(np.abs(c[7:]).sum(axis=1) == 2)


def _single_phase(shape, **kw):
    return oracle.Oracle(shape, **kw)


def test_rest_state_is_fixed_point():
    shape = (6, 5, 4)
    N = 120
    o = _single_phase(shape)
    o.init_fields(np.zeros(N), np.zeros(N))
    f0 = o.populations().copy()
    o.step(20)
    assert np.abs(o.populations() - f0).max() <= 4 * EPS


def test_uniform_flow_is_fixed_point():
    # Galilean-invariant uniform state of BGK with the equilibrium as initial
    # condition and no force: it must stay put
    shape = (5, 4, 6)
    N = 120
    u0 = np.array([0.03, -0.02, 0.01])
    u = np.repeat(u0[:, None], N, axis=1)
    o = _single_phase(shape, tau=0.8)
    o.init_fields(np.zeros(N), np.zeros(N), None, u)
    f0 = o.populations().copy()
    o.step(25)
    assert np.abs(o.populations() - f0).max() <= 16 * EPS
    assert np.allclose(o.fields()["u"], u, atol=1e-15)


@pytest.mark.parametrize("tau", [1.0, 0.7])
def test_uniform_force_closed_form(tau):
    # uniform body force on a uniform periodic fluid: the momentum grows by F
    # per node per step exactly, and the forcing-corrected velocity after t
    # steps is (t + 1/2) F / rho
    shape = (4, 3, 5)
    N = 60
    F = np.array([1e-5, -2e-5, 3e-6])
    o = _single_phase(shape, tau=tau, ext_force=F)
    o.init_fields(np.zeros(N), np.zeros(N))
    for t in range(1, 11):
        o.step(1)
        tot, _ = o.observables()
        # rounding bound: a sum of 19 N populations of size <= 1/3, t steps
        assert np.allclose(tot["mom"], N * t * F, rtol=0, atol=19 * N * t * EPS)
        uf = o.aux()["u"]  # velocity used in step t (state at t-1)
        assert np.allclose(uf, ((t - 1) + 0.5) * F[:, None], rtol=0, atol=19 * t * EPS)
        assert abs(tot["mass"] - N) < 1e-12


@pytest.mark.parametrize("tau", [1.0, 0.8])
@pytest.mark.parametrize("axes", [(0, 2), (1, 0), (2, 1)])
def test_shear_wave_decay(tau, axes):
    # u_a = U0 sin(2 pi s / L) along axis s decays as exp(-nu k^2 t) with
    # nu = (tau - 1/2)/3 (BGK viscosity; tau = 1 gives the paper's nu = 1/6)
    a, s = axes
    L = 32
    shape = [2, 2, 2]
    shape[s] = L
    shape = tuple(shape)
    N = int(np.prod(shape))
    xs = I.coords(shape)[s]
    U0 = 1e-6
    u = np.zeros((3, N))
    u[a] = U0 * np.sin(2 * np.pi * xs / L)
    o = _single_phase(shape, tau=tau)
    o.init_fields(np.zeros(N), np.zeros(N), None, u)
    nst = 300
    o.step(nst)
    ua = o.fields()["u"][a]
    amp = 2.0 * np.mean(ua * np.sin(2 * np.pi * xs / L))
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / L
    assert abs(amp / U0 / math.exp(-nu * k * k * nst) - 1.0) < 0.01


def _exact_totals(o):
    """Exactly rounded sums (math.fsum) of the state over fluid nodes, so that
    the balance checks below see the update's rounding and not the
    summation's."""
    f = o.populations()
    flds = o.fields()
    c, _ = oracle.lattice()
    fluid = o.owner() < 0
    ff = f[:, fluid]
    mass = math.fsum(ff.ravel())
    mom = np.array([math.fsum((ff * c[:, a][:, None]).ravel()) for a in range(3)])
    return mass, mom, math.fsum(flds["psi"][fluid]), math.fsum(flds["c"][fluid])


def test_mass_and_momentum_balance_with_free_energy_force():
    # no particles: mass exact; momentum changes by the summed body force each
    # step (Guo forcing injects exactly F per node); sum of psi exact; the sum
    # of c changes by the sink only (Eq. 3a with no source)
    shape = (12, 10, 8)
    N = int(np.prod(shape))
    psi = I.slab(shape, I.WIDTH, amp=0.05, seed=11)
    c = 0.2 + I.noise(12, N, 0.05)
    p = dict(I.FREE_ENERGY)
    p["E"] = -0.2
    o = oracle.Oracle(shape, **p)
    o.init_fields(psi, c)
    m0, _, s0, _ = _exact_totals(o)
    # per-node rounding of one update is a few ulps of O(1) quantities
    tol = 32 * N * EPS
    for _ in range(15):
        mb, pb, sb, cb = _exact_totals(o)
        o.step(1)
        ma, pa, sa, ca = _exact_totals(o)
        dg = o.step_diag()
        assert abs(ma - m0) <= tol
        assert np.allclose(pa - pb, dg["sum_force"], rtol=0, atol=tol)
        assert abs(sa - s0) <= tol
        assert abs((ca - cb) - (dg["sum_src"] - p["k_d"] * dg["sum_chi"])) <= tol


@pytest.mark.parametrize("M_psi,nsub", [(0.1, 1), (0.4, 2)])
def test_linearised_update_has_no_growing_mode(M_psi, nsub):
    # Jacobian of one oracle step around the ordered state (psi = 1, rest
    # fluid) on a 4^3 box, by finite differences: every eigenvalue must lie in
    # the unit disk.  (With the central two-point gradient in the body force
    # instead of the isotropic lattice gradient, the explicit coupling of the
    # force with the advection of psi has modes growing by ~8% per step at
    # kappa = 0.04; the fix is the reading documented with the oracle.)  The
    # paper's mobility M_psi = 0.4 is stable with two psi/c sub-steps.
    FE = dict(rho0=1.0, tau=1.0, a=-0.0625, b=0.0625, kappa=0.04, M_psi=M_psi,
              ch_substeps=nsub)
    shape = (4, 4, 4)
    N = 64
    _, w = oracle.lattice()
    f0 = np.repeat(w[:, None], N, axis=1)
    psi0 = np.ones(N)

    def step(f, psi):
        o = oracle.Oracle(shape, **FE)
        o.init_fields(psi, np.zeros(N))
        o.set_populations(f)
        o.step(1)
        return np.concatenate([o.populations().ravel(), o.fields()["psi"]])

    base = step(f0, psi0)
    h = 1e-7
    J = np.zeros((20 * N, 20 * N))
    for j in range(20 * N):
        f = f0.copy().ravel()
        p = psi0.copy()
        if j < 19 * N:
            f[j] += h
        else:
            p[j - 19 * N] += h
        J[:, j] = (step(f.reshape(19, N), p) - base) / h
    assert np.abs(np.linalg.eigvals(J)).max() <= 1.0 + 1e-6


def test_solute_force_option_closed_form():
    # option OR_SOLUTE_FORCE: the solvent also feels -c grad(mu_c), mu_c =
    # C chi.  With psi = 0 (no psi force, tanh psi = 0: chi = c - c_b0) and
    # c = c0 + A sin(kx), the isotropic stencil reduces to the central
    # difference along x, grad_x chi = A sin(k) cos(kx) exactly, so
    # F = (-C c(x) A sin(k) cos(kx), 0, 0); without the option F = 0.
    shape = (32, 4, 3)
    N = int(np.prod(shape))
    x = I.coords(shape)[0]
    k = 2.0 * np.pi / shape[0]
    c0, A, C = 0.7, 0.2, 0.35
    c = c0 + A * np.sin(k * x)
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.0, C=C, E=-0.2, c_b0=0.5, D_c=0.0,
             k_d=0.0, tau=1.0)
    for flags, expect in ((0, np.zeros((3, N))),
                          (oracle.SOLUTE_FORCE,
                           np.stack([-C * c * A * np.sin(k) * np.cos(k * x), np.zeros(N), np.zeros(N)]))):
        o = oracle.Oracle(shape, flags=flags, **p)
        o.init_fields(np.zeros(N), c)
        o.step(1)
        F = o.aux()["force"]
        o.close()
        assert np.allclose(F, expect, rtol=0, atol=64 * EPS * C * A * c0)
    # the force pushes solute-rich fluid down its own gradient: F_x < 0 where c rises
    assert (expect[0][np.cos(k * x) > 0.1] < 0).all()


def test_option_flags_validated():
    with pytest.raises(RuntimeError):
        oracle.Oracle((4, 4, 4), flags=8)


def test_paper_mobility_needs_substeps():
    # M_psi = 0.4 (Sec. II.C) with a = -b = 0.0625, kappa = 0.04 puts the
    # explicit psi update beyond its stability bound M (12|a| + 36|b| +
    # 144 kappa) < 2 for a unit time step; two sub-steps of 1/2 satisfy it
    FE = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.4)
    with pytest.raises(RuntimeError):
        oracle.Oracle((8, 8, 8), **FE)
    with pytest.raises(RuntimeError):
        oracle.Oracle((8, 8, 8), ch_substeps=1, **FE)
    oracle.Oracle((8, 8, 8), ch_substeps=2, **FE).close()


def test_threads_do_not_change_results():
    # the per-node loops may run on several OpenMP threads; every sum is taken
    # in node or link order afterwards, so one thread and many give the same
    # bits (32^3 workload with a moving Janus sphere, 6 steps)
    from paper_2202_01631_amd import inputs as I
    w = I.workload_small()
    out = []
    for nt in (1, 4):
        assert oracle.set_threads(nt) == nt
        o = oracle.from_spec(w)
        o.step(6)
        f = o.populations()
        fl = o.fields()
        _, cols = o.observables()
        out.append((f, fl["psi"], fl["c"], o.links(), o.owner(), cols[0]["pos"], cols[0]["vel"]))
        o.close()
    oracle.set_threads(1)
    for a, b in zip(*out):
        assert np.array_equal(a, b)
