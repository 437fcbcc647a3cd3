"""The paper's printed parameter values (tests/golden/paper_values.json,
each entry citing its section) against the model's closed forms and the
oracle's free energy."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I
from test_oracle_scalars import _free_energy, _minimise

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def v(k):
    return G[k]["value"]


def test_printed_closed_forms():
    # sigma = (2/3) sqrt(2 kappa A) ~ 0.047 (Sec. II.C)
    assert (2.0 / 3.0) * math.sqrt(2 * v("kappa") * v("A")) == pytest.approx(v("sigma"), abs=5e-4)
    # D_psi = A M_psi, D_phi = C M_phi (definitions after Eq. 3)
    assert v("A") * v("M_psi") == pytest.approx(v("D_psi"), rel=1e-12)
    assert v("C") * v("M_phi") == pytest.approx(v("D_phi"), rel=1e-12)
    # BGK viscosity (tau - 1/2)/3 = 1/6 at tau = 1 (the oracle's shear-wave
    # test measures this relation)
    assert (1.0 - 0.5) / 3.0 == pytest.approx(v("nu"), rel=1e-15)
    # l = sqrt(D_phi/k_d) "approximately one diameter"
    ell = math.sqrt(v("D_phi") / v("k_d"))
    assert 0.7 < ell / (v("screening_length_over_R") * v("R")) < 1.1


def test_surface_tension_of_the_lattice_free_energy():
    # excess free energy per unit area of the discrete flat interface (two
    # interfaces in a periodic column), with the paper's A and kappa, is the
    # printed sigma ~ 0.047 up to the lattice error of a one-node-wide
    # interface (below 5%)
    A, kap = v("A"), v("kappa")
    p = dict(a=-A, b=A, kappa=kap, M_psi=0.1, C=0.0, E=0.0, c_b0=0.0, D_c=0.0, k_d=0.0)
    shape = (1, 1, 32)
    ps, _ = _minimise(I.slab(shape, I.WIDTH, offset=0.5), np.zeros(32), shape, p)
    import torch
    F = _free_energy(torch.from_numpy(ps), torch.zeros(32), shape, p).item()
    bulk = -A / 2 + A / 4
    sigma = (F - 32 * bulk) / 2.0
    assert abs(sigma / v("sigma") - 1.0) < 0.05
    # and the oracle holds this profile still
    o = oracle.Oracle(shape, **p)
    o.init_fields(ps, np.zeros(32))
    o.step(30)
    assert np.abs(o.fields()["psi"] - ps).max() < 1e-9


def test_printed_mobility_is_outside_explicit_stability():
    # the explicit Euler scheme used for psi needs
    # M_psi (12|a| + 36 b + 144 kappa) < 2; the printed M_psi = 0.4 violates
    # it (the paper's own scheme is not stated), so the oracle refuses it and
    # the workloads use M_psi = 0.1
    A, kap = v("A"), v("kappa")
    with pytest.raises(oracle.OracleError):
        oracle.Oracle((4, 4, 4), a=-A, b=A, kappa=kap, M_psi=v("M_psi"))
    oracle.Oracle((4, 4, 4), a=-A, b=A, kappa=kap, M_psi=0.1).close()


def _bulk_psi(mu, sign, a, b):
    """Bulk order parameter at chemical potential mu: the root of
    a psi + b psi^3 = mu (Eq. 2 without gradients) next to psi = sign."""
    p = float(sign)
    for _ in range(60):
        p -= (a * p + b * p ** 3 - mu) / (a + 3 * b * p * p)
    return p


@pytest.mark.slow
def test_laplace_law_of_a_droplet():
    # Laplace pressure of a droplet (Sec. II.C surface tension): a spherical
    # water droplet (psi = +1) in oil, relaxed by the oracle's own dynamics to
    # equilibrium, where mu is uniform.  Its bulk phases then sit at psi_in,
    # psi_out with a psi + b psi^3 = mu, and the pressure jump p = psi mu - f
    # across the interface is the Laplace pressure 2 sigma / R; for the
    # symmetric free energy (Delta psi = 2) this is mu R = sigma, with R the
    # equimolar radius from sum psi.  Two radii (R = 7 and 9 in boxes 24^3 and
    # 28^3; M_psi = 3.2 in 16 psi sub-steps so the exterior equilibrates in
    # 1000 steps): mu R within 4% of the printed sigma ~ 0.047 and mu ~ 1/R
    # (mu R equal within 2%).  Measured: mu R = 0.0462, 0.0467.
    A, kap = v("A"), v("kappa")
    a, b = -A, A
    oracle.set_threads(os.cpu_count() or 1)
    muR = []
    for R in (7, 9):
        L = 2 * R + 10
        shape = (L, L, L)
        N = L ** 3
        x = I.coords(shape)
        c0 = L / 2 - 0.5
        r = np.sqrt((x[0] - c0) ** 2 + (x[1] - c0) ** 2 + (x[2] - c0) ** 2)
        o = oracle.Oracle(shape, a=a, b=b, kappa=kap, M_psi=3.2, C=0.0, E=0.0, c_b0=0.0,
                          D_c=0.0, k_d=0.0, tau=1.0, ch_substeps=16)
        o.init_fields(-np.tanh((r - R) / I.WIDTH), np.zeros(N))
        o.step(1000)
        mu = o.aux()["mu"]
        ps = o.fields()["psi"]
        o.close()
        m = mu.mean()
        assert mu.max() - mu.min() <= 1e-2 * m          # equilibrated (measured 4e-3)
        pin, pout = _bulk_psi(m, 1.0, a, b), _bulk_psi(m, -1.0, a, b)
        Re = (3.0 * (ps.sum() - N * pout) / (pin - pout) / (4.0 * math.pi)) ** (1.0 / 3.0)
        muR.append(m * Re)
    oracle.set_threads(1)
    for s in muR:
        assert abs(s / v("sigma") - 1.0) <= 0.04, muR
    assert abs(muR[0] / muR[1] - 1.0) <= 0.02, muR
