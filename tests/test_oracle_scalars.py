"""Pins of the oracle's order-parameter and solute updates (Eqs. 1-3):
exact discrete Fourier-mode evolution of the linear solute scheme, the
discrete free energy of Eq. 1 (+ Eq. 8) and its minimisers, the equilibrium
partition of the solute (Fig. 1 closed form) and the screened field around
an emitting sphere."""
import math

import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I

EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("kvec,u0", [
    ((1, 0, 0), (0.0, 0.0, 0.0)),
    ((0, 2, 0), (0.0, 0.0, 0.0)),
    ((0, 0, 1), (0.0, 0.0, 0.02)),
    ((1, 1, 2), (0.01, -0.015, 0.02)),
])
def test_solute_fourier_mode_exact(kvec, u0):
    # psi = 1 and E = 0: mu_psi = a + b = 0 exactly, no force, the uniform flow
    # u0 persists, and c - c_b0 obeys a linear constant-coefficient scheme
    # whose Fourier factor per step is
    #   G = 1 - i sum_a u_a sin k_a - D sum_a 4 sin^2(k_a/2) - k_d
    shape = (8, 6, 10)
    N = int(np.prod(shape))
    x = I.coords(shape)
    k = [2 * np.pi * kvec[a] / shape[a] for a in range(3)]
    phase = sum(k[a] * x[a] for a in range(3))
    D, kd, cb0, eps = 0.1, 0.01, 0.5, 1e-3
    o = oracle.Oracle(shape, a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0625, E=0.0,
                      c_b0=cb0, D_c=D, k_d=kd, tau=0.9)
    u = np.repeat(np.array(u0)[:, None], N, axis=1)
    o.init_fields(np.ones(N), cb0 + eps * np.cos(phase), None, u)
    G = (1.0 - 1j * sum(u0[a] * math.sin(k[a]) for a in range(3))
         - D * sum(4 * math.sin(k[a] / 2) ** 2 for a in range(3)) - kd)
    for t in (1, 10, 40):
        o.step(t - o.observables()[0]["step"])
        want = cb0 + eps * np.real(G ** t * np.exp(1j * phase))
        assert np.abs(o.fields()["c"] - want).max() <= 8 * t * EPS
        assert np.abs(o.fields()["psi"] - 1.0).max() == 0.0


@pytest.mark.parametrize("nsub", [2, 3])
def test_solute_fourier_mode_exact_substeps(nsub):
    # the same linear scheme advanced in n psi/c sub-steps of length 1/n per
    # LB step (u held, chi recomputed): the factor per LB step is
    #   G = (1 - (i sum_a u_a sin k_a + D sum_a 4 sin^2(k_a/2) + k_d) / n)^n
    kvec, u0 = (1, 2, 1), (0.03, -0.02, 0.01)
    shape = (8, 6, 10)
    N = int(np.prod(shape))
    x = I.coords(shape)
    k = [2 * np.pi * kvec[a] / shape[a] for a in range(3)]
    phase = sum(k[a] * x[a] for a in range(3))
    D, kd, cb0, eps = 0.1, 0.01, 0.5, 1e-3
    o = oracle.Oracle(shape, a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0625, E=0.0,
                      c_b0=cb0, D_c=D, k_d=kd, tau=0.9, ch_substeps=nsub)
    u = np.repeat(np.array(u0)[:, None], N, axis=1)
    o.init_fields(np.ones(N), cb0 + eps * np.cos(phase), None, u)
    g = 1.0 - (1j * sum(u0[a] * math.sin(k[a]) for a in range(3))
               + D * sum(4 * math.sin(k[a] / 2) ** 2 for a in range(3)) + kd) / nsub
    G = g ** nsub
    for t in (1, 10, 40):
        o.step(t - o.observables()[0]["step"])
        want = cb0 + eps * np.real(G ** t * np.exp(1j * phase))
        assert np.abs(o.fields()["c"] - want).max() <= 8 * nsub * t * EPS
        assert np.abs(o.fields()["psi"] - 1.0).max() == 0.0


def _iso_gradient_symbol(k):
    """Fourier symbol g of the D3Q19 isotropic gradient 3 sum_i w_i c_i f(x + c_i):
    for f = exp(i k.x) it returns i g(k) exp(i k.x).  Worked out by hand from
    the weights 1/18 (faces) and 1/36 (edges):
    g_x = sin(k_x) (1 + cos k_y + cos k_z) / 3, and cyclically."""
    s = [math.sin(v) for v in k]
    c = [math.cos(v) for v in k]
    return [s[0] * (1 + c[1] + c[2]) / 3, s[1] * (1 + c[2] + c[0]) / 3,
            s[2] * (1 + c[0] + c[1]) / 3]


@pytest.mark.parametrize("kvec,u0", [
    ((1, 0, 0), (0.0, 0.0, 0.0)),
    ((1, 1, 2), (0.0, 0.0, 0.0)),
    ((2, 1, 3), (0.0, 0.0, 0.0)),
    ((1, 2, 1), (0.03, -0.02, 0.01)),
])
def test_psi_update_one_step_fourier_mode(kvec, u0):
    # Eq. 3b linearised about psi = 1 (with a = -b, mu(1) = 0) for one small
    # Fourier mode psi = 1 + eps cos(k.x), E = 0 (no solute coupling), rest
    # populations at density 1 and uniform velocity u0.  One step of the
    # method then gives, to first order in eps:
    #   mu   = eps m_k cos(k.x),  m_k = a + 3b + kappa lam,  lam = sum_a 4 sin^2(k_a/2)
    #          (Eq. 2 with the 7-point Laplacian);
    #   F    = -psi grad(mu) = eps m_k g(k) sin(k.x) (isotropic gradient symbol g);
    #   u    = u0 + F/2 (first moment plus half the force, density 1);
    #   psi' = 1 + eps Re(G exp(i k.x)) with
    #   G    = 1 - i sum_a u0_a sin k_a - m_k (M_psi lam + 1/2 sum_a sin(k_a) g_a),
    #          the three terms being the central-flux advection by u0, the
    #          diffusion M_psi lap(mu) and the central-flux divergence of F/2.
    # The second-order remainder is ~eps^2 = 1e-14; a wrong factor on M_psi,
    # on the flux, on F/2 or on the gradient stencil moves psi' by >= 1e-10.
    shape = (8, 6, 10)
    N = int(np.prod(shape))
    x = I.coords(shape)
    k = [2 * np.pi * kvec[a] / shape[a] for a in range(3)]
    phase = sum(k[a] * x[a] for a in range(3))
    a, b, kap, M, eps = -0.0625, 0.0625, 0.04, 0.1, 1e-7
    o = oracle.Oracle(shape, a=a, b=b, kappa=kap, M_psi=M, C=0.0625, E=0.0, c_b0=0.3,
                      D_c=0.1, k_d=1e-3, tau=0.9)
    u = np.repeat(np.array(u0)[:, None], N, axis=1)
    o.init_fields(1.0 + eps * np.cos(phase), np.full(N, 0.3), None, u)
    o.step(1)
    lam = sum(4 * math.sin(v / 2) ** 2 for v in k)
    mk = a + 3 * b + kap * lam
    g = _iso_gradient_symbol(k)
    aux = o.aux()
    # first-order fields; the remainder is the eps^2 term (3 b eps^2 = 2e-15 in mu)
    assert np.abs(aux["mu"] - eps * mk * np.cos(phase)).max() <= 1e-14
    for ax in range(3):
        F = eps * mk * g[ax] * np.sin(phase)
        assert np.abs(aux["force"][ax] - F).max() <= 1e-14
        assert np.abs(aux["u"][ax] - (u0[ax] + F / 2)).max() <= 1e-14
    G = (1.0 - 1j * sum(u0[ax] * math.sin(k[ax]) for ax in range(3))
         - mk * (M * lam + 0.5 * sum(math.sin(k[ax]) * g[ax] for ax in range(3))))
    want = 1.0 + eps * np.real(G * np.exp(1j * phase))
    err = np.abs(o.fields()["psi"] - want).max()
    assert err <= 2e-13, err
    # the mode really moved: the first-order change is far above the bound
    assert eps * abs(1.0 - G) >= 1e-3 * eps
    o.close()


# ------------------------------------------------------ discrete free energy
def _free_energy(psi, c, shape, p, owner=None, surf=None):
    """Eq. 1 on the lattice (torch, FP64): sum over fluid nodes of
    a/2 psi^2 + b/4 psi^4 + C/2 (c - c_b0 - E tanh psi)^2, plus
    kappa/2 (psi(x+e) - psi(x))^2 for each pair of fluid face neighbours, plus
    the wetting term of Eq. 8 as sum over boundary faces of H |e.n| psi(x)
    (surf holds H|e.n| summed per node)."""
    import torch
    sh = tuple(shape[::-1])
    P = psi.reshape(sh)
    Cc = c.reshape(sh)
    fl = torch.ones(sh, dtype=torch.bool) if owner is None else \
        torch.from_numpy(owner.reshape(sh) < 0)
    chi = Cc - p["c_b0"] - p["E"] * torch.tanh(P)
    e = (p["a"] / 2 * P ** 2 + p["b"] / 4 * P ** 4 + p["C"] / 2 * chi ** 2)[fl].sum()
    for ax in range(3):
        Pn = torch.roll(P, -1, dims=2 - ax)
        fn = torch.roll(fl, -1, dims=2 - ax)
        e = e + (p["kappa"] / 2 * (Pn - P) ** 2)[fl & fn].sum()
    if surf is not None:
        e = e + (torch.from_numpy(surf.reshape(sh)) * P)[fl].sum()
    return e


def _minimise(psi0, c0, shape, p, owner=None, surf=None, fix_c_total=True, iters=40):
    """Stationary point of the discrete free energy at fixed total psi (and
    total c when the sink is off) over the fluid nodes: Newton iterations on
    the Lagrangian with gradient and Hessian of the energy taken by automatic
    differentiation (no hand-written derivative), started from (psi0, c0).
    When C = 0 the solute does not enter the energy and is left as given."""
    import torch
    N = psi0.size
    fl = np.ones(N, dtype=bool) if owner is None else owner < 0
    idx = torch.from_numpy(np.where(fl)[0])
    n = idx.numel()
    with_c = p["C"] != 0.0
    nv = 2 * n if with_c else n
    base_p = torch.from_numpy(psi0.astype(np.float64))
    base_c = torch.from_numpy(c0.astype(np.float64))

    def energy(v):
        ps = base_p.clone().index_put((idx,), v[:n])
        cc = base_c.clone().index_put((idx,), v[n:]) if with_c else base_c
        return _free_energy(ps, cc, shape, p, owner, surf)

    v = torch.cat([base_p[idx], base_c[idx]]).clone() if with_c else base_p[idx].clone()
    rows = [torch.cat([torch.ones(n), torch.zeros(nv - n)]).double()]
    if with_c and fix_c_total:
        rows.append(torch.cat([torch.zeros(n), torch.ones(n)]).double())
    A = torch.stack(rows)
    target = A @ v
    m = A.shape[0]
    for _ in range(iters):
        g = torch.autograd.functional.jacobian(energy, v)
        Hs = torch.autograd.functional.hessian(energy, v)
        K = torch.zeros(nv + m, nv + m, dtype=torch.float64)
        K[:nv, :nv] = Hs
        K[:nv, nv:] = A.T
        K[nv:, :nv] = A
        rhs = torch.cat([-g, target - A @ v])
        d = torch.linalg.solve(K, rhs)
        v = v + d[:nv]
        if d[:nv].abs().max() < 1e-15:
            break
    ps, cc = psi0.copy(), c0.copy()
    ps[fl] = v[:n].numpy()
    if with_c:
        cc[fl] = v[n:].numpy()
    return ps, cc


def test_flat_interface_minimiser_is_fixed_point():
    # the discrete minimiser of Eq. 1 (ordered phase, interfaces between nodes)
    # has uniform mu_psi, hence no force and no flux: it must not move
    shape = (1, 1, 32)
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0, E=0.0, c_b0=0.0,
             D_c=0.0, k_d=0.0)
    psi0 = I.slab(shape, I.WIDTH, offset=0.5)
    ps, cc = _minimise(psi0, np.zeros(32), shape, p)
    o = oracle.Oracle(shape, **p)
    o.init_fields(ps, cc)
    o.step(50)
    assert np.abs(o.fields()["psi"] - ps).max() < 1e-9
    assert np.abs(o.fields()["u"]).max() < 1e-12
    # and the continuum tanh width sqrt(2 kappa/|a|) within the lattice
    # discretisation error of a one-node-wide interface (the lattice profile
    # is about 12% sharper at w = 1.13)
    from scipy.optimize import curve_fit
    z = np.arange(32.0)

    def prof(z, z1, z2, w, amp):
        return -amp * np.tanh((z - z1) / w) * np.tanh((z - z2) / w)

    fit, _ = curve_fit(prof, z, ps, p0=[8.5, 23.5, 1.0, 1.0])
    assert abs(fit[2] / math.sqrt(2 * 0.04 / 0.0625) - 1.0) < 0.15
    assert abs(ps.max() - 1.0) < 1e-3 and abs(ps.min() + 1.0) < 1e-3


def test_coupled_minimiser_is_fixed_point():
    # psi and c together, E != 0, no sink: the joint minimiser of Eq. 1 at
    # fixed totals has uniform mu_psi and uniform chi -- a fixed point.  A
    # wrong sign or factor in the coupling term of Eq. 2 moves it.
    shape = (1, 1, 24)
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0625, E=-0.3, c_b0=0.5,
             D_c=0.1, k_d=0.0)
    psi0 = I.slab(shape, I.WIDTH, offset=0.5)
    c0 = 0.6 + 0.3 * np.tanh(psi0)
    ps, cc = _minimise(psi0, c0, shape, p)
    o = oracle.Oracle(shape, **p)
    o.init_fields(ps, cc)
    o.step(40)
    f = o.fields()
    assert np.abs(f["psi"] - ps).max() < 1e-8
    assert np.abs(f["c"] - cc).max() < 1e-8
    # the same fields with the coupling sign flipped in the functional are
    # not stationary for the oracle
    q = dict(p, E=+0.3)
    ps2, cc2 = _minimise(psi0, 0.6 - 0.3 * np.tanh(psi0), shape, q)
    o2 = oracle.Oracle(shape, **p)
    o2.init_fields(ps2, cc2)
    o2.step(40)
    assert np.abs(o2.fields()["psi"] - ps2).max() > 1e-5


def test_wetting_minimiser_is_fixed_point():
    # a fixed sphere with wetting H != 0 in an ordered fluid: the minimiser of
    # Eq. 1 plus the wetting energy of Eq. 8 (sum over boundary faces of
    # H |e.n| psi) is stationary under the oracle, whose Laplacian uses the
    # ghost value of Eq. 9.  Checks sign and size of the wetting condition.
    shape = (10, 10, 10)
    N = 1000
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0, E=0.0, c_b0=0.0,
             D_c=0.0, k_d=0.0)
    H = 0.02
    col = dict(pos=(4.6, 5.2, 4.9), m=(0, 0, 1), radius=2.6, H=H, fixed=1)
    probe = oracle.Oracle(shape, **p)
    probe.init_fields(np.ones(N), np.zeros(N))
    probe.add_colloids([col])
    owner = probe.owner()
    # H |e.n| per fluid node, summed over its solid faces (n from the centre
    # through the face midpoint), computed here independently
    x = np.stack(I.coords(shape))
    surf = np.zeros(N)
    L = np.array(shape, dtype=float)[:, None]
    R = np.array(col["pos"])[:, None]
    for ax in range(3):
        for sgn in (1, -1):
            e = np.zeros((3, 1))
            e[ax] = sgn
            nb = (x + e) % L
            nb_idx = (nb[0] + shape[0] * (nb[1] + shape[1] * nb[2])).astype(int)
            solid_face = (owner < 0) & (owner[nb_idx] >= 0)
            r = x + 0.5 * e - R
            r -= L * np.round(r / L)
            en = np.abs(r[ax]) / np.linalg.norm(r, axis=0)
            surf += np.where(solid_face, H * en, 0.0)
    assert surf.max() > 0
    ps, _ = _minimise(np.ones(N), np.zeros(N), shape, p, owner, surf, fix_c_total=True)
    assert ps[owner < 0].min() < 0.99  # H > 0 pulls psi towards the oil value
    o = oracle.Oracle(shape, **p)
    o.init_fields(ps, np.zeros(N))
    o.add_colloids([col])
    o.step(30)
    fl = owner < 0
    assert np.abs(o.fields()["psi"][fl] - ps[fl]).max() < 1e-7


def test_solute_partition_fig1():
    # no particles, sink on: c relaxes to c0(psi) = c_b0 + E tanh(psi)
    # pointwise (Eq. 2 with mu_c = 0), and with c_b0 = 0 the phase averages
    # are +E tanh 1 in water (psi > 0) and -E tanh 1 in oil, up to O(w/L).
    # psi starts at its discrete equilibrium and C is tiny, so that the
    # order parameter stays put while c relaxes at the rate k_d.
    L = 128
    shape = (1, 1, L)
    E = -0.4
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=1e-9, E=E, c_b0=0.0,
             D_c=0.1, k_d=0.05)
    psi0, _ = _minimise(I.slab(shape, I.WIDTH, offset=0.5), np.zeros(L), shape, dict(p, C=0.0))
    o = oracle.Oracle(shape, **p)
    o.init_fields(psi0, np.zeros(L))
    o.step(800)
    f = o.fields()
    assert np.abs(f["c"] - E * np.tanh(f["psi"])).max() < 1e-10
    water = f["psi"] > 0
    oil = ~water
    th = math.tanh(1.0)
    assert abs(f["c"][water].mean() / (E * th) - 1.0) < 0.03
    assert abs(f["c"][oil].mean() / (-E * th) - 1.0) < 0.03


def test_screened_solute_field():
    # a fixed sphere emitting on both hemispheres in a single-phase fluid
    # (A = E = kappa = 0, Sec. III.A): at steady state emission balances the
    # sink globally (sum alpha per link = k_d sum chi), and away from the
    # sphere the field is the screened kernel of D lap - k_d (continuum
    # exp(-r/l)/r, l = sqrt(D/k_d)) applied to the emitted sources.  The
    # kernel is the textbook periodic lattice Green's function, built here by
    # FFT; its amplitude absorbs the no-flux hole left by the particle.
    L = 20
    shape = (L, L, L)
    N = L ** 3
    D, kd, alpha = 0.1, 0.02, 1e-3
    h = L // 2
    p = dict(a=0.0, b=0.0, kappa=0.0, M_psi=0.0, C=0.0625, E=0.0, c_b0=0.0, D_c=D, k_d=kd)
    o = oracle.Oracle(shape, **p)
    o.init_fields(np.zeros(N), np.zeros(N))
    o.add_colloids([dict(pos=(h, h, h), m=(0, 0, 1), radius=2.5, alpha_minus=alpha,
                         alpha_plus=alpha, fixed=1)])
    o.step(700)  # 14 e-folds of the slowest rate k_d
    dg = o.step_diag()
    assert abs(dg["sum_src"] - kd * dg["sum_chi"]) < 1e-5 * dg["sum_src"]
    src = np.zeros(N)
    for _, n, _, _ in o.links():
        src[n] += alpha
    k = 2 * np.pi * np.fft.fftfreq(L)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    Gh = 1.0 / (kd + D * (4 * np.sin(KX / 2) ** 2 + 4 * np.sin(KY / 2) ** 2
                          + 4 * np.sin(KZ / 2) ** 2))
    S = np.fft.fftn(src.reshape(L, L, L).transpose(2, 1, 0))
    model = np.real(np.fft.ifftn(S * Gh)).transpose(2, 1, 0).ravel()
    c = o.fields()["c"]
    r = np.linalg.norm(np.stack(I.coords(shape)) - h, axis=0)
    far = (r >= 5) & (r <= 9)
    A = (c[far] @ model[far]) / (model[far] @ model[far])
    assert 1.0 <= A <= 1.3
    assert np.abs(c[far] / (A * model[far]) - 1.0).max() < 0.03
    # the lattice kernel's decay length along an axis, 1/acosh(1 + k_d/2D),
    # is the continuum l = sqrt(D/k_d) up to O(1/l^2)
    ell_h = 1.0 / math.acosh(1.0 + kd / (2 * D))
    assert abs(ell_h / math.sqrt(D / kd) - 1.0) < 0.01
