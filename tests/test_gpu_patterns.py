"""GPU parity of particles with surface patterns (polar bands times azimuthal
sectors, each cell with its own production, phoretic mobility and wetting
parameter; the inhomogeneous surfaces of Sec. IV, the Janus split of
Eqs. 5-6 generalised) against the FP64 oracle.

Bars as for the Janus particle: link tables (with the cell of every link)
and owner maps bit-exact, FP64 fields within 1e-12, particle states within
1e-11; the boundary fix-up launches that carry the cell arithmetic give the
bits of the inline forms where a pattern reduces to the Janus split."""
import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb
from parity_util import U_FLOOR_FP32, field_errors, flush_print, run_pair

pytestmark = pytest.mark.gpu


def _pattern(bands, sectors, cuts, alpha, mu, H):
    n = bands * sectors
    assert len(alpha) == len(mu) == len(H) == n and len(cuts) == bands - 1
    return dict(bands=bands, sectors=sectors, cos=list(cuts), alpha=list(alpha), mu=list(mu),
                H=list(H))


def _spec(shape, seed, colloids, precision="fp64", E=-0.2):
    N = int(np.prod(shape))
    p = dict(I.FREE_ENERGY)
    p["E"] = E
    return dict(name="pattern%s" % (shape,), shape=shape, precision=precision, params=p,
                psi=I.slab(shape, I.WIDTH, amp=0.05, seed=seed),
                c=0.3 + I.noise(seed + 1, N, 0.05), colloids=list(colloids))


def _patterned(shape):
    """Three moving spheres: 3 bands x 8 sectors (random cells), 2 bands x
    4 sectors with a zero second axis (the fallback axis), 4 bands x 1
    sector; productions, mobilities and wetting differing per cell."""
    u = I.uniform(77, 3 * 64).reshape(3, 64)
    pats = [
        _pattern(3, 8, (-0.45, 0.3), 2e-3 * u[0, :24], 0.4 * (u[1, :24] - 0.5),
                 0.01 * (u[2, :24] - 0.5)),
        _pattern(2, 4, (0.1,), [1e-3, 0.0, 3e-3, 0.0, 0.0, 2e-3, 0.0, 1e-3],
                 [0.2, -0.1, 0.05, 0.3, -0.2, 0.0, 0.1, 0.15],
                 [0.004, -0.003, 0.0, 0.002, -0.001, 0.003, 0.0, -0.004]),
        _pattern(4, 1, (-0.6, 0.0, 0.55), [0.0, 2e-3, 0.0, 1e-3], [0.1, -0.2, 0.25, 0.0],
                 [0.002, 0.0, -0.002, 0.001]),
    ]
    pos = [(10.2, 10.3, 9.1), (31.4, 12.7, 20.2), (15.9, 26.1, 24.3)]
    es = [I.unit_vectors(90, 1)[0], np.zeros(3), (1.0, 0.5, -0.25)]
    cols = []
    for k in range(3):
        c = I.janus(pos[k], I.unit_vectors(80 + k, 1)[0], 4.6, alpha=0.0, mu=0.0, theta=90.0)
        c["e"] = np.asarray(es[k], dtype=np.float64)
        c["pattern"] = pats[k]
        c["vel"] = np.array([0.01, -0.006, 0.004]) * (k - 1)
        c["omega"] = np.array([0.002, 0.003, -0.001]) * (k + 1)
        cols.append(c)
    return cols


def test_patterns_match_oracle():
    # 30 steps of three patterned, moving, turning spheres: links with their
    # cells and owner maps bit-exact after every 10 steps, FP64 fields within
    # 1e-12, positions, axes (m and e) and velocities within 1e-11, the count
    # of producing links equal
    shape = (46, 38, 34)
    cols = _patterned(shape)
    g, o = run_pair(_spec(shape, 41, cols), 0)
    assert np.array_equal(g.owner(), o.owner())
    assert np.array_equal(g.links(), o.links())
    assert g.links()[:, 3].max() > 8  # cells beyond the Janus bit are in the table
    for _ in range(3):
        g.step(10)
        o.step(10)
        assert np.array_equal(g.owner(), o.owner())
        assert np.array_equal(g.links(), o.links())
    e = field_errors(g.fields(), o.fields(), o.owner() < 0)
    flush_print("[patterns] fp64 errors %s" % e)
    assert max(e.values()) <= 1e-12
    tg, cg = g.observables()
    to, co = o.observables()
    assert tg["n_active"] == to["n_active"] and tg["n_links"] == to["n_links"]
    for k in range(3):
        for a in ("vel", "omega", "pos", "m", "e"):
            assert np.abs(cg[k][a] - co[k][a]).max() <= 1e-11, (k, a)
        assert abs(float(cg[k]["e"] @ cg[k]["m"])) <= 1e-14
        assert cg[k]["pattern"]["bands"] == cols[k]["pattern"]["bands"]
        assert cg[k]["pattern"]["alpha"] == list(cols[k]["pattern"]["alpha"])


def test_equatorial_pattern_gives_the_janus_bits():
    # a pattern of two bands cut at m.n = 0, one sector, with the Janus
    # values on the cells, steps bit for bit like the Janus particle (the
    # pattern box takes the boundary fix-up launches, the Janus box the
    # inline forms), FP32 and FP64; the link tags differ only in naming
    # (cell 0 is the active cap, tag 1 of the Janus table)
    shape = (40, 36, 34)
    base = I.janus((17.3, 15.8, 16.4), I.unit_vectors(5, 1)[0], 4.7, alpha=2e-3, mu_minus=0.25,
                   mu_plus=-0.1, theta=90.0)
    base["vel"] = np.array([0.012, -0.004, 0.006])
    base["H"] = 0.003
    pat = dict(base, pattern=_pattern(2, 1, (0.0,), [2e-3, 0.0], [0.25, -0.1], [0.003, 0.003]))
    pat.pop("contact_angle")
    base.pop("contact_angle")
    for prec in ("fp64", "fp32"):
        a = lb.from_spec(_spec(shape, 12, [base], precision=prec))
        b = lb.from_spec(_spec(shape, 12, [pat], precision=prec))
        a.step(25)
        b.step(25)
        assert np.array_equal(a.populations(), b.populations()), prec
        assert np.array_equal(a.fields()["psi"], b.fields()["psi"]), prec
        la, lb_ = a.links(), b.links()
        assert np.array_equal(la[:, :3], lb_[:, :3])
        assert np.array_equal(la[:, 3], 1 - lb_[:, 3])
        _, ca = a.observables()
        _, cb = b.observables()
        for key in ("pos", "vel", "omega", "m"):
            assert np.array_equal(ca[0][key], cb[0][key]), (prec, key)
        a.close()
        b.close()


def test_pattern_fp32_alone_batched_and_graph():
    # FP32: a patterned box stepped alone, in a batch beside a Janus box
    # (the whole batch takes the fix-up launches) and graph-replayed gives
    # the same bits; against the oracle within the FP32 bar after 100 steps
    import torch
    shape = (46, 38, 34)
    cols = _patterned(shape)
    spec = _spec(shape, 43, cols, precision="fp32")
    other = _spec((40, 36, 34), 44, [I.janus((18.2, 17.1, 16.9), (0.0, 0.6, 0.8), 4.4)],
                  precision="fp32")
    s = torch.cuda.Stream()
    a = lb.from_spec(spec, stream=s)
    a.step(100)
    b = lb.from_spec(spec, stream=s)
    c = lb.from_spec(other, stream=s)
    lb.batch_step([b, c], 100)
    d = lb.from_spec(other, stream=s)
    d.step(100)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(c.populations(), d.populations())
    assert np.array_equal(a.links(), b.links())
    o = oracle.from_spec(dict(spec, precision="fp64"))
    o.step(100)
    assert np.array_equal(a.owner(), o.owner())
    assert np.array_equal(a.links(), o.links())
    e = field_errors(a.fields(), o.fields(), o.owner() < 0, u_floor=U_FLOOR_FP32)
    flush_print("[patterns] fp32 100 steps errors %s" % e)
    assert max(e.values()) <= 2e-5
    for x in (a, b, c, d):
        x.close()


def test_pattern_validation():
    shape = (32, 32, 32)
    N = int(np.prod(shape))
    ok = _pattern(2, 2, (0.2,), [1e-3] * 4, [0.1] * 4, [0.0] * 4)
    bad = [
        dict(ok, bands=9),
        dict(ok, sectors=3),
        dict(ok, bands=8, sectors=16),
        dict(ok, cos=[1.0]),
        dict(_pattern(3, 1, (0.3, -0.2), [0.0] * 3, [0.0] * 3, [0.0] * 3)),
    ]
    for pat in bad:
        box = lb.Box(shape, "fp64", **I.FREE_ENERGY)
        box.init_fields(np.zeros(N), np.zeros(N))
        with pytest.raises(lb.LBError):
            box.add_colloids([dict(pos=(16.0, 16.0, 16.0), m=(0.0, 0.0, 1.0), radius=4.0,
                                   rho_p=1.0, pattern=pat)])
        box.close()
    p0 = dict(I.FREE_ENERGY, kappa=0.0)
    box = lb.Box(shape, "fp64", **p0)
    box.init_fields(np.zeros(N), np.zeros(N))
    with pytest.raises(lb.LBError):
        box.add_colloids([dict(pos=(16.0, 16.0, 16.0), m=(0.0, 0.0, 1.0), radius=4.0, rho_p=1.0,
                               pattern=dict(ok, H=[0.0, 0.01, 0.0, 0.0]))])
    box.add_colloids([dict(pos=(16.0, 16.0, 16.0), m=(0.0, 0.0, 1.0), radius=4.0, rho_p=1.0,
                           pattern=ok)])
    _, c = box.observables()
    assert c[0]["pattern"]["sectors"] == 2
    # zero second axis, m = z: the least aligned lattice axis x, made orthogonal to m
    assert np.array_equal(c[0]["e"], (1.0, 0.0, 0.0))
    box.close()
