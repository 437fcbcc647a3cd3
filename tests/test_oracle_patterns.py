"""Pins of the oracle's surface patterns (the inhomogeneous surface patterns
of Sec. IV, a generalisation of the Janus caps of Eqs. 5-6): cells of polar
bands in m.n and azimuthal sectors about m, each with its own production,
phoretic mobility and wetting parameter.

Pinned here against what the geometry and the physics fix: the cell of every
link against an independent classification by angles (acos and atan2 of the
link midpoint in the body frame) and against each cell's share of the
sphere's surface; a two-band pattern cut at the equator reproduces the Janus
particle bit for bit; a uniform pattern does not swim, nor does a pattern
mirror-symmetric about the equator along the axis; the second body axis turns
with the particle; a wetting pattern's minimiser of Eq. 1 plus the Eq. 8
surface energy is a fixed point."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2202_01631_amd import inputs as I
from test_oracle_colloids import CVEC, _min_image
from test_oracle_scalars import _minimise

FE0 = dict(a=0.0, b=0.0, kappa=0.0, M_psi=0.0, C=0.0625, E=0.0, c_b0=0.0, D_c=0.05, k_d=1e-3,
           tau=1.0)


def pattern(bands, sectors, cuts=(), alpha=None, mu=None, H=None):
    n = bands * sectors
    return dict(bands=bands, sectors=sectors, cos=list(cuts),
                alpha=list(alpha if alpha is not None else [0.0] * n),
                mu=list(mu if mu is not None else [0.0] * n),
                H=list(H if H is not None else [0.0] * n))


def body_frame(m, e):
    m = np.asarray(m, float) / np.linalg.norm(m)
    e = np.asarray(e, float)
    e = e - (e @ m) * m
    e /= np.linalg.norm(e)
    return m, e, np.cross(m, e)


def cell_by_angles(r, m, e, w, cuts, sectors):
    """Cell of the direction r by its polar angle (acos of m.n against the
    cuts) and its azimuth (atan2 of the projections on w = m x e and e, in
    [0, 2 pi), sector width 2 pi / sectors); None within 1e-9 of a cut or of a
    sector edge, where only the half-open rule decides."""
    n = r / np.linalg.norm(r)
    th = math.acos(max(-1.0, min(1.0, float(n @ m))))
    band = 0
    for t in cuts:
        d = th - math.acos(t)
        if abs(d) < 1e-9:
            return None
        if d < 0:            # above the cut: m.n > t
            band += 1
    phi = math.atan2(float(n @ w), float(n @ e)) % (2 * math.pi)
    width = 2 * math.pi / sectors
    s = phi / width
    if sectors > 1 and abs(s - round(s)) < 1e-9 and np.linalg.norm(n - (n @ m) * m) > 1e-9:
        return None
    return band * sectors + int(s) % sectors


def test_pattern_cells_against_angles():
    # three spheres (random axes, ragged positions across the periodic wrap)
    # with patterns of 3 x 8, 1 x 4 and 5 x 2 cells: every link's cell equals
    # the angle classification, and each cell's share of the links follows its
    # share of the surface, (cos_hi - cos_lo)/2 / sectors, to 0.06
    shape = (30, 28, 26)
    N = int(np.prod(shape))
    ms = I.unit_vectors(91, 3)
    es = I.unit_vectors(92, 3)
    pats = [pattern(3, 8, (-0.3, 0.4)), pattern(1, 4), pattern(5, 2, (-0.7, -0.2, 0.1, 0.6))]
    cols = [dict(pos=(7.3, 7.9, 8.4), m=ms[0], e=es[0], radius=5.2, pattern=pats[0]),
            dict(pos=(21.6, 18.2, 16.1), m=ms[1], e=es[1], radius=5.7, pattern=pats[1]),
            dict(pos=(8.8, 21.1, 24.4), m=ms[2], e=es[2], radius=4.9, pattern=pats[2])]
    o = oracle.Oracle(shape, **FE0)
    o.init_fields(np.zeros(N), np.zeros(N))
    o.add_colloids(cols)
    links = o.links()
    _, got = o.observables()
    X = np.stack(I.coords(shape))
    Ls = np.array(shape, float)
    checked = 0
    for k, q in enumerate(cols):
        m, e, w = body_frame(q["m"], q["e"])
        assert np.allclose(got[k]["e"], e, atol=1e-15)
        rec = links[links[:, 0] == k]
        pat = q["pattern"]
        ncell = pat["bands"] * pat["sectors"]
        for _, n, d, cell in rec:
            r = np.array([_min_image((X[a, n] + 0.5 * CVEC[d][a]) - q["pos"][a], Ls[a])
                          for a in range(3)])
            want = cell_by_angles(r, m, e, w, pat["cos"], pat["sectors"])
            assert 0 <= cell < ncell
            if want is not None:
                assert cell == want, (k, n, d, cell, want)
                checked += 1
        cuts = [-1.0] + list(pat["cos"]) + [1.0]
        for c in range(ncell):
            b = c // pat["sectors"]
            area = (cuts[b + 1] - cuts[b]) / 2.0 / pat["sectors"]
            share = float(np.mean(rec[:, 3] == c))
            assert abs(share - area) <= 0.06, (k, c, share, area)
    assert checked > 0.99 * len(links)
    # bad patterns are refused
    for bad in (pattern(3, 3, (0.0, 0.5)), pattern(3, 4, (0.5, 0.0)),
                pattern(9, 1, [0.1 * i for i in range(7)]), pattern(2, 1, (1.0,))):
        with pytest.raises(RuntimeError):
            o2 = oracle.Oracle(shape, **FE0)
            o2.init_fields(np.zeros(N), np.zeros(N))
            o2.add_colloids([dict(cols[0], pattern=bad)])


def test_equator_pattern_is_the_janus_particle():
    # two bands cut at m.n = 0, one sector, with the Janus values: the same
    # step as the Janus particle of Eqs. 5-6, bit for bit (a moving, wetting,
    # emitting particle at an interface, 25 steps)
    w = I.workload_small()
    q = dict(w["colloids"][0], H=0.01, alpha_plus=2e-4, mu_minus=0.2, mu_plus=-0.1,
             omega=(0.0, 0.002, 0.001))
    pat = pattern(2, 1, (0.0,), alpha=(q["alpha_minus"], q["alpha_plus"]),
                  mu=(q["mu_minus"], q["mu_plus"]), H=(q["H"], q["H"]))
    out = []
    for col in (q, dict(q, pattern=pat, alpha_minus=0.0, alpha_plus=0.0, mu_minus=0.0,
                        mu_plus=0.0, H=0.0)):
        o = oracle.from_spec(dict(w, colloids=[col]))
        o.step(25)
        f = o.fields()
        _, c = o.observables()
        out.append((o.populations(), f["psi"], f["c"], c[0]["pos"], c[0]["vel"], c[0]["m"],
                    o.links()[:, :3]))
        o.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("which", ["uniform", "equatorial stripe", "polar cap",
                                   "polar mobility"])
def test_symmetric_patterns_do_not_swim(which):
    # a held sphere centred on a node (mirror-symmetric lattice sphere), axis
    # +x: a pattern that is the same everywhere, or symmetric about the
    # equator (an active equatorial stripe), takes no phoretic force along
    # the axis (round-off); a polar active cap does (Eq. 7's self-propulsion),
    # and so does a uniformly emitting sphere whose phoretic mobility is
    # nonzero on one polar band only (Eq. 4 with a patterned mobility)
    shape = (32, 32, 32)
    N = int(np.prod(shape))
    B, S = 4, 8
    cuts = (-0.5, 0.0, 0.5)
    if which == "uniform":
        alpha, mu = [1e-3] * (B * S), [0.2] * (B * S)
    elif which == "equatorial stripe":
        alpha = [0.0] * S + [1e-3] * (2 * S) + [0.0] * S
        mu = [0.2] * (B * S)
    elif which == "polar cap":
        alpha = [1e-3] * S + [0.0] * (3 * S)
        mu = [0.2] * (B * S)
    else:
        alpha = [1e-3] * (B * S)
        mu = [0.3] * S + [0.0] * (3 * S)
    o = oracle.Oracle(shape, **FE0)
    o.init_fields(np.zeros(N), np.zeros(N))
    o.add_colloids([dict(pos=(16.0, 16.0, 16.0), m=(1, 0, 0), e=(0, 1, 0), radius=5.0, fixed=1,
                         pattern=pattern(B, S, cuts, alpha=alpha, mu=mu))])
    o.step(150)
    F = o.colloid_diag(0)["F0"]
    o.close()
    if which in ("polar cap", "polar mobility"):
        assert abs(F[0]) > 1e-4
    else:
        assert abs(F[0]) <= 1e-12
        if which == "uniform":
            assert np.abs(F).max() <= 1e-12


def test_second_axis_turns_with_the_particle():
    # a free particle set spinning: after each step its axes (m, e) are the
    # previous ones turned by the rotation vector Omega' (Rodrigues), e stays
    # a unit vector orthogonal to m
    shape = (24, 24, 24)
    N = int(np.prod(shape))
    o = oracle.Oracle(shape, **FE0)
    o.init_fields(np.zeros(N), np.zeros(N))
    o.add_colloids([dict(pos=(11.3, 12.1, 12.6), m=(0.3, 0.5, 0.8), e=(1.0, 0.0, 0.0),
                         radius=4.0, omega=(0.01, -0.02, 0.015), rho_p=3.0,
                         pattern=pattern(2, 4, (0.0,), alpha=[1e-3] * 8, mu=[0.1] * 8))])
    _, c0 = o.observables()
    for _ in range(5):
        o.step(1)
        _, c1 = o.observables()
        R = Rotation.from_rotvec(c1[0]["omega"])
        assert np.allclose(R.apply(c0[0]["m"]), c1[0]["m"], atol=1e-13)
        assert np.allclose(R.apply(c0[0]["e"]), c1[0]["e"], atol=1e-13)
        assert abs(c1[0]["m"] @ c1[0]["e"]) <= 1e-15 and abs(np.linalg.norm(c1[0]["e"]) - 1) <= 1e-15
        c0 = c1
    o.close()


def test_wetting_pattern_minimiser_is_fixed_point():
    # a fixed sphere whose two hemispheres wet differently (H = +0.02 on the
    # m.n <= 0 half, -0.01 on the other): the minimiser of Eq. 1 plus the
    # Eq. 8 energy summed over boundary faces with the H of each face's cell
    # (classified here by angles) is stationary under the oracle
    shape = (10, 10, 10)
    N = 1000
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0, E=0.0, c_b0=0.0,
             D_c=0.0, k_d=0.0)
    Hs = (0.02, -0.01)
    col = dict(pos=(4.6, 5.2, 4.9), m=(0.0, 0.6, 0.8), e=(1.0, 0.0, 0.0), radius=2.6, fixed=1,
               pattern=pattern(2, 1, (0.0,), H=Hs))
    probe = oracle.Oracle(shape, **p)
    probe.init_fields(np.ones(N), np.zeros(N))
    probe.add_colloids([col])
    owner = probe.owner()
    m, e, w = body_frame(col["m"], col["e"])
    x = np.stack(I.coords(shape))
    surf = np.zeros(N)
    L = np.array(shape, dtype=float)[:, None]
    R = np.array(col["pos"])[:, None]
    for ax in range(3):
        for sgn in (1, -1):
            ev = np.zeros((3, 1))
            ev[ax] = sgn
            nb = (x + ev) % L
            nb_idx = (nb[0] + shape[0] * (nb[1] + shape[1] * nb[2])).astype(int)
            solid_face = (owner < 0) & (owner[nb_idx] >= 0)
            r = x + 0.5 * ev - R
            r -= L * np.round(r / L)
            en = np.abs(r[ax]) / np.linalg.norm(r, axis=0)
            for i in np.where(solid_face)[0]:
                cell = cell_by_angles(r[:, i], m, e, w, (0.0,), 1)
                assert cell is not None
                surf[i] += Hs[cell] * en[i]
    assert surf.max() > 0 > surf.min()
    ps, _ = _minimise(np.ones(N), np.zeros(N), shape, p, owner, surf, fix_c_total=True)
    fl = owner < 0
    # H > 0 pulls psi towards oil next to its half, H < 0 towards water
    assert ps[fl].min() < 0.99 and ps[fl].max() > 1.0
    o = oracle.Oracle(shape, **p)
    o.init_fields(ps, np.zeros(N))
    o.add_colloids([col])
    o.step(30)
    assert np.abs(o.fields()["psi"][fl] - ps[fl]).max() < 1e-7
