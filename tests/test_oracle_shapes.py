"""Pins of the oracle's spheroidal particles: a reading of Sec. IV, where the
local rules of the model (inside test and links of Sec. II.B, slip of Eq. 4
along the surface normal, wetting of Eqs. 8-9) carry over to particles of
other shapes.  A spheroid has semi-axis a (`axial`) along its axis m and b
(`radius`) across it.

Independent checks: solid nodes and links against a classification in the
body frame of the spheroid (its own arithmetic); the lattice volume against
4 pi a b^2 / 3; the rigid-body update against the textbook mass and inertia
tensor of a spheroid; symmetry (a uniformly coated spheroid does not swim);
the wetting ghost against a surface energy whose normal is the
finite-difference gradient of the spheroid's implicit function."""
import math

import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I
from test_oracle_colloids import CVEC, _min_image
from test_oracle_scalars import _minimise

EPS = np.finfo(np.float64).eps


def body_axes(m):
    m = np.asarray(m, float) / np.linalg.norm(m)
    j = int(np.argmin(np.abs(m)))
    t = np.zeros(3)
    t[j] = 1.0
    u = np.cross(m, t)
    u /= np.linalg.norm(u)
    return u, np.cross(m, u), m


def shape_function(q, r):
    """(x^2 + y^2)/b^2 + z^2/a^2 in the body frame (z along m), for
    displacements r (3, n)."""
    u, v, m = body_axes(q["m"])
    a = q.get("axial") or q["radius"]
    b = q["radius"]
    x, y, z = u @ r, v @ r, m @ r
    return (x * x + y * y) / (b * b) + z * z / (a * a)


def displacements(shape, pos, half=None):
    X = np.stack(I.coords(shape)).astype(float)
    if half is not None:
        X = X + 0.5 * half[:, None]
    L = np.array(shape, dtype=float)
    return np.stack([_min_image(X[a] - pos[a], L[a]) for a in range(3)])


def _oracle(shape, cols, **kw):
    N = int(np.prod(shape))
    p = dict(C=0.0625, D_c=0.1, k_d=0.01)
    p.update(kw)
    o = oracle.Oracle(shape, **p)
    o.init_fields(np.zeros(N), np.zeros(N))
    o.add_colloids(cols)
    return o


@pytest.mark.parametrize("a,b", [(6.3, 3.7), (2.9, 5.4)])
def test_solid_nodes_against_the_body_frame(a, b):
    # prolate and oblate spheroids at non-integer positions with random axes,
    # one across the periodic boundary: solid exactly where the body-frame
    # shape function is below 1 (nodes within 1e-9 of the surface excluded)
    shape = (30, 28, 26)
    cols = [dict(pos=(7.3, 9.1, 13.4), m=I.unit_vectors(5, 1)[0], radius=b, axial=a),
            dict(pos=(22.6, 26.2, 3.1), m=I.unit_vectors(6, 1)[0], radius=b, axial=a)]
    o = _oracle(shape, cols)
    own = o.owner()
    checked = 0
    for k, q in enumerate(cols):
        f = shape_function(q, displacements(shape, q["pos"]))
        clear = np.abs(f - 1.0) > 1e-9
        assert np.array_equal(own[clear & (f < 1.0)], np.full(int((clear & (f < 1.0)).sum()), k))
        assert not np.any(own[clear & (f > 1.0)] == k)
        checked += int(clear.sum())
    assert checked > 0.99 * 2 * own.size


def test_lattice_volume_of_a_spheroid():
    # solid node counts of a prolate (9, 6) and an oblate (4, 7) spheroid,
    # averaged over random positions and axes, within 1% of 4 pi a b^2 / 3
    shape = (28, 28, 28)
    for a, b in ((9.0, 6.0), (4.0, 7.0)):
        u = I.uniform(90 + int(a), 3 * 8).reshape(8, 3)
        counts = []
        for i in range(8):
            q = dict(pos=tuple(14.0 + u[i]), m=I.unit_vectors(40 + i, 1)[0], radius=b, axial=a)
            o = _oracle(shape, [q])
            counts.append(int((o.owner() == 0).sum()))
            o.close()
        vol = 4.0 * math.pi * a * b * b / 3.0
        assert abs(np.mean(counts) / vol - 1.0) < 0.01, (a, b, np.mean(counts), vol)


def test_links_against_brute_force():
    # links (fluid node, direction into the spheroid) and their cap bits
    # (m.r <= 0 at the link midpoint) by enumeration over the body-frame
    # classification, for a prolate and an oblate spheroid
    shape = (26, 24, 22)
    cols = [dict(pos=(6.6, 7.2, 10.9), m=I.unit_vectors(11, 1)[0], radius=3.1, axial=5.2),
            dict(pos=(18.4, 16.3, 11.7), m=I.unit_vectors(12, 1)[0], radius=4.6, axial=2.8)]
    o = _oracle(shape, cols)
    nx, ny, nz = shape
    N = nx * ny * nz
    owner = -np.ones(N, dtype=np.int64)
    for k, q in enumerate(cols):
        f = shape_function(q, displacements(shape, q["pos"]))
        assert np.abs(f - 1.0).min() > 1e-9  # no node on a surface
        owner[f < 1.0] = k
    assert np.array_equal(owner, o.owner())
    X = np.stack(I.coords(shape))
    recs = []
    for k, q in enumerate(cols):
        for n in np.where(owner < 0)[0]:
            for d in range(1, 19):
                y = (X[:, n] + CVEC[d]) % np.array(shape)
                if owner[int(y[0] + nx * (y[1] + ny * y[2]))] != k:
                    continue
                r = np.array([_min_image((X[a, n] + 0.5 * CVEC[d][a]) - q["pos"][a], shape[a])
                              for a in range(3)])
                mm = np.asarray(q["m"]) / np.linalg.norm(q["m"])
                recs.append((k, n, d, int(mm @ r <= 0.0)))
    want = np.array(sorted(recs), dtype=np.int64)
    got = o.links()
    assert len(want) > 300 and np.array_equal(got, want)


def test_axial_equal_to_radius_is_the_sphere():
    # axial 0 or equal to the radius: the sphere's own arithmetic, same bits
    shape = (20, 18, 16)
    base = dict(pos=(8.3, 9.1, 7.7), m=(0.3, 0.5, 0.8), radius=4.1, vel=(0.02, -0.01, 0.01),
                omega=(0.01, 0.0, -0.02), alpha_minus=1e-3, mu_minus=0.2, mu_plus=-0.1, H=0.003)
    out = []
    for extra in ({}, dict(axial=0.0), dict(axial=4.1)):
        o = _oracle(shape, [dict(base, **extra)], kappa=0.04)
        o.step(12)
        out.append((o.populations(), o.links(), o.observables()[1][0]["pos"]))
        o.close()
    for x in out[1:]:
        assert np.array_equal(x[0], out[0][0]) and np.array_equal(x[1], out[0][1])
        assert np.array_equal(x[2], out[0][2])


@pytest.mark.parametrize("explicit", [False, True])
def test_rigid_body_update_uses_the_spheroid_inertia(explicit):
    # a free prolate spheroid launched with V and Omega (not along its axis)
    # through fluid at rest, cover/uncover included: every step, with the
    # force F and torque T the oracle reports as acting,
    #   m (V' - V) = F  and  I (Omega' - Omega) = T,
    # m = rho_p 4 pi a b^2 / 3 and I = I_perp 1 + (I_par - I_perp) m m^T
    # (I_par = 2 m b^2 / 5 about the axis, I_perp = m (a^2 + b^2) / 5
    # across it) at the axis of the start of the step
    shape = (24, 22, 22)
    a, b, rho = 6.0, 3.5, 1.3
    q = dict(pos=(8.2, 10.9, 11.3), m=(0.6, 0.0, 0.8), radius=b, axial=a, rho_p=rho,
             vel=(0.03, 0.01, -0.01), omega=(0.004, -0.006, 0.003), alpha_minus=1e-3,
             mu_minus=0.1, mu_plus=0.1)
    o = _oracle(shape, [q], flags=2 if explicit else 0)
    mass = rho * 4.0 * math.pi * a * b * b / 3.0
    ipar, iperp = 0.4 * mass * b * b, 0.2 * mass * (a * a + b * b)
    changed = 0
    for _ in range(12):
        _, c0 = o.observables()
        own0 = o.owner()
        o.step(1)
        _, c1 = o.observables()
        d = o.colloid_diag(0)
        m0 = c0[0]["m"]
        Iten = iperp * np.eye(3) + (ipar - iperp) * np.outer(m0, m0)
        assert np.allclose(mass * (c1[0]["vel"] - c0[0]["vel"]), d["F"], rtol=0, atol=1e-12)
        assert np.allclose(Iten @ (c1[0]["omega"] - c0[0]["omega"]), d["T"], rtol=0, atol=1e-11)
        changed += int((o.owner() != own0).sum())
    assert changed > 0
    assert abs(np.linalg.norm(c1[0]["m"]) - 1.0) < 1e-14


def test_uniformly_coated_spheroid_does_not_swim():
    # a held prolate spheroid along x centred on a node (mirror symmetric on
    # the lattice), emitting on its whole surface with one mobility: no
    # phoretic force (round-off); the Janus spheroid (active half m.n <= 0,
    # m = +x) is pushed along +x, and an oblate one too
    shape = (36, 30, 30)
    N = int(np.prod(shape))
    F = {}
    for name, a, b, cc in (("uniform", 7.0, 4.0, 1.0), ("janus", 7.0, 4.0, 0.0),
                           ("oblate janus", 3.0, 5.5, 0.0)):
        o = oracle.Oracle(shape, a=0.0, b=0.0, kappa=0.0, M_psi=0.0, C=0.0625, E=0.0, c_b0=0.0,
                          D_c=0.05, k_d=1e-3, tau=1.0)
        o.init_fields(np.zeros(N), np.zeros(N))
        o.add_colloids([dict(pos=(18.0, 15.0, 15.0), m=(1, 0, 0), radius=b, axial=a,
                             alpha_minus=1e-3, alpha_plus=0.0, mu_minus=0.2, mu_plus=0.2,
                             fixed=1, cap_cos=cc)])
        o.step(120)
        F[name] = o.colloid_diag(0)["F0"].copy()
        o.close()
    assert np.abs(F["uniform"]).max() <= 1e-12
    assert F["janus"][0] > 0.005 and abs(F["janus"][1]) < 1e-12 and abs(F["janus"][2]) < 1e-12
    assert F["oblate janus"][0] > 0.005


def test_wetting_minimiser_with_the_spheroid_normal_is_fixed_point():
    # a fixed tilted prolate spheroid with wetting H in an ordered fluid: the
    # minimiser of Eq. 1 plus the Eq. 8 energy, sum over boundary faces of
    # H |e.n| psi with n the normalised finite-difference gradient of the
    # body-frame shape function at the face midpoint, is stationary under
    # the oracle, whose Laplacian takes the ghost of Eq. 9
    shape = (12, 12, 12)
    N = 12 ** 3
    p = dict(a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1, C=0.0, E=0.0, c_b0=0.0,
             D_c=0.0, k_d=0.0)
    H = 0.02
    col = dict(pos=(5.6, 6.2, 5.9), m=(0.0, 0.6, 0.8), radius=2.4, axial=3.6, H=H, fixed=1)
    probe = oracle.Oracle(shape, **p)
    probe.init_fields(np.ones(N), np.zeros(N))
    probe.add_colloids([col])
    owner = probe.owner()
    x = np.stack(I.coords(shape))
    L = np.array(shape, dtype=float)[:, None]
    R = np.array(col["pos"])[:, None]
    surf = np.zeros(N)
    h = 1e-5
    for ax in range(3):
        for sgn in (1, -1):
            e = np.zeros((3, 1))
            e[ax] = sgn
            nb = (x + e) % L
            nb_idx = (nb[0] + shape[0] * (nb[1] + shape[1] * nb[2])).astype(int)
            solid_face = (owner < 0) & (owner[nb_idx] >= 0)
            r = x + 0.5 * e - R
            r -= L * np.round(r / L)
            g = np.zeros_like(r)
            for j in range(3):
                dj = np.zeros((3, 1))
                dj[j] = h
                g[j] = (shape_function(col, r + dj) - shape_function(col, r - dj)) / (2 * h)
            en = np.abs(g[ax]) / np.linalg.norm(g, axis=0)
            surf += np.where(solid_face, H * en, 0.0)
    assert surf.max() > 0
    ps, _ = _minimise(np.ones(N), np.zeros(N), shape, p, owner, surf, fix_c_total=True)
    fl = owner < 0
    assert ps[fl].min() < 0.99
    o = oracle.Oracle(shape, **p)
    o.init_fields(ps, np.zeros(N))
    o.add_colloids([col])
    o.step(30)
    # the finite-difference normal carries ~1e-10 of error into the energy
    assert np.abs(o.fields()["psi"][fl] - ps[fl]).max() < 1e-7


def test_spheroid_options_validated():
    shape = (24, 24, 24)
    N = 24 ** 3
    q = dict(pos=(12.0, 12.0, 12.0), m=(0, 0, 1), radius=3.0, axial=5.0)
    for kw, col in ((dict(soft_eps=0.05, soft_sigma=1.0, soft_nu=1.0, soft_hc=1.0), q),
                    (dict(lub_hc=2.0), q), ({}, dict(q, axial=-1.0)), ({}, dict(q, axial=10.5))):
        o = oracle.Oracle(shape, C=0.0625, D_c=0.1, k_d=0.01, **kw)
        o.init_fields(np.zeros(N), np.zeros(N))
        with pytest.raises(oracle.OracleError):
            o.add_colloids([col])
        o.close()
