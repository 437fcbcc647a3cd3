"""GPU checks of the divergence-form solvent force (LB_STRESS_FORM, with
LB_CAPILLARY_FORCE; the momentum exchange of Sec. II.B made exact for the
capillary coupling): FP32 and FP64 against the oracle on the paper's
regime box, batched beside a box without the option bit for bit as alone,
long runs that stay finite, and a particle settling at its contact angle."""
import numpy as np
import pytest

import oracle
from paper_2202_01631_amd import inputs as I
from paper_2202_01631_amd import lb
from parity_util import U_FLOOR_FP32, field_errors, flush_print

pytestmark = pytest.mark.gpu


def _trap_spec(mu=0.05, E=-0.25, flags=lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM, R=4.5,
               M_psi=0.1, nsub=1, precision="fp32"):
    # a tilted axis: no link midpoint lies exactly on the cap's equator, where
    # the cap bit would hang on round-off in the turning axis
    col = I.janus((16.0, 48.0, 48.0), (0.3, 0.9, 0.2), R, alpha=0.0, mu=mu, theta=90.0)
    w = I.workload_paper([col], E=E)
    w["params"].update(flags=flags, M_psi=M_psi, ch_substeps=nsub)
    w["c"] = w["params"]["c_b0"] + E * np.tanh(w["psi"])
    w["precision"] = precision
    return w


@pytest.mark.parametrize("precision,steps,tol", [("fp64", 20, 1e-12), ("fp32", 20, 2e-5)])
def test_paper_box_matches_oracle(precision, steps, tol):
    # the paper's box with the option, a sphere on the interface pushed
    # phoretically, 20 steps: owner maps and links exact, fields within the
    # precision's bar, the particle's state within 1e-11 (FP64)
    w = _trap_spec(precision=precision)
    g = lb.from_spec(w)
    o = oracle.from_spec(dict(w, precision="fp64"))
    g.step(steps)
    o.step(steps)
    assert np.array_equal(g.owner(), o.owner())
    assert np.array_equal(g.links(), o.links())
    e = field_errors(g.fields(), o.fields(), o.owner() < 0,
                     u_floor=None if precision == "fp64" else U_FLOOR_FP32)
    flush_print("[stress form] %s errors %s" % (precision, e))
    assert max(e.values()) <= tol
    if precision == "fp64":
        _, cg = g.observables()
        _, co = o.observables()
        for a in ("vel", "omega", "pos"):
            assert np.abs(cg[0][a] - co[0][a]).max() <= 1e-11, a
    g.close()
    o.close()


def test_batched_beside_a_box_without_the_option():
    # one launch per kernel for both boxes: the box with the option takes
    # the one-node forms and the fix-ups, the other its own path; each gives
    # the bits it gives alone
    import torch
    s = torch.cuda.Stream()
    a_spec = _trap_spec()
    b_spec = _trap_spec(flags=lb.LB_CAPILLARY_FORCE, mu=0.1)
    a = lb.from_spec(a_spec, stream=s)
    b = lb.from_spec(b_spec, stream=s)
    lb.batch_step([a, b], 40)
    a1 = lb.from_spec(a_spec, stream=s)
    b1 = lb.from_spec(b_spec, stream=s)
    a1.step(40)
    b1.step(40)
    assert np.array_equal(a.populations(), a1.populations())
    assert np.array_equal(b.populations(), b1.populations())
    for x in (a, b, a1, b1):
        x.close()


def test_option_validated():
    with pytest.raises(lb.LBError):
        lb.Box((32, 32, 32), "fp32", **dict(I.FREE_ENERGY, flags=lb.LB_STRESS_FORM))


def test_twice_the_radius_stays_stable_past_ten_thousand_steps():
    # the R = 9 displacement runs of the paper-regime tests (128 x 160 x
    # 160, E = -0.25, mu = 0.025 ... 0.2, M_psi = 0.4 in two sub-steps), with
    # the divergence-form force: where the capillary option alone grows a
    # slow instability (two of the four runs overflow near step 10^4), every
    # run stays finite for 12000 steps, the fluid calm (max |u| < 0.03), and
    # every particle sits on the side away from the solute-rich phase, the
    # strongest push furthest out (measured Delta X 1.01, 2.50, 2.46, 3.90:
    # the settled particles pin near lattice positions, so Delta X is not
    # proportional to mu E here and that is not asserted)
    import torch
    shape = (128, 160, 160)
    st = torch.cuda.Stream()
    boxes, mus = [], (0.025, 0.05, 0.1, 0.2)
    for mu in mus:
        col = I.janus((32.0, 80.0, 80.0), (0.0, 1.0, 0.0), 9.0, alpha=0.0, mu=mu, theta=90.0)
        w = I.workload_paper([col], E=-0.25, shape=shape)
        w["params"]["flags"] = lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM
        w["c"] = w["params"]["c_b0"] - 0.25 * np.tanh(w["psi"])
        boxes.append(lb.from_spec(w, stream=st))
    for k in range(4):
        lb.batch_step(boxes, 3000)
        flush_print("[stress form R=9] %d steps" % (3000 * (k + 1)))
    dxs = []
    for b, mu in zip(boxes, mus):
        t, c = b.observables()
        assert t["error_bits"] == 0, mu
        f = b.fields()
        assert np.abs(f["u"]).max() < 0.03, mu
        ps = f["psi"].reshape(shape[2], shape[1], shape[0])
        colm = ps[:, :40, :].reshape(-1, shape[0]).mean(axis=0)
        i = 24 + int(np.argmax((colm[24:40] < 0) & (colm[25:41] >= 0)))
        xint = i + colm[i] / (colm[i] - colm[i + 1])
        dxs.append(c[0]["pos"][0] - xint)
        flush_print("[stress form R=9] mu %s Delta X %.4f ratio %.1f max|u| %.4f"
                    % (mu, dxs[-1], dxs[-1] / (0.25 * mu), np.abs(f["u"]).max()))
        b.close()
    assert min(dxs) > 0 and dxs[3] == max(dxs) and dxs[3] > dxs[0] + 1.0


def test_trap_runs_at_one_psi_update_stay_stable():
    # the trap runs at M_psi = 0.1 with one psi/c update per step (R = 4.5,
    # E = -0.25, mu = 0.025 ... 0.2), where the capillary option alone lets
    # the total momentum grow until a run overflows near step 3200: with the
    # divergence form every run stays finite for 8000 steps with a calm fluid
    import torch
    st = torch.cuda.Stream()
    boxes = [lb.from_spec(_trap_spec(mu=mu), stream=st) for mu in (0.025, 0.05, 0.1, 0.2)]
    for k in range(4):
        lb.batch_step(boxes, 2000)
        flush_print("[stress form R=4.5] %d steps" % (2000 * (k + 1)))
    for b in boxes:
        t, _ = b.observables()
        assert t["error_bits"] == 0
        assert np.abs(b.fields()["u"]).max() < 0.03
        b.close()


def test_particle_settles_at_its_contact_angle():
    # Young's position (Sec. III.B; the wetting of Eqs. 8-10): a sphere of
    # radius 8 released on a flat interface (64^3, interfaces at x = 16 and
    # 48, the paper's free energy, no solute) settles with its centre R cos
    # theta into the phase it prefers -- oil (psi < 0, x < 16) for theta < 90
    # degrees.  With H from the lattice's own map (the angle a flat wall of
    # this lattice realises) and the capillary stress in divergence form,
    # after 8000 steps the offset is within 0.5 of -R cos theta (measured
    # -3.88 / +3.84 / 0.00 for 60 / 120 / 90 degrees).  With H from the
    # printed Eq. 10, the same 60 degrees realises about 43 on this lattice
    # and the particle sits beyond 4.8 (measured 5.53).
    import torch
    shape = (64, 64, 64)
    R = 8.0
    st = torch.cuda.Stream()
    cases = [("lattice", 60.0), ("lattice", 90.0), ("lattice", 120.0), ("eq10", 60.0)]
    boxes = []
    for wmap, th in cases:
        col = I.janus((16.0, 32.0, 32.0), (0.0, 1.0, 0.0), R, alpha=0.0, mu=0.0, theta=th)
        w = I.workload_paper([col], E=0.0, shape=shape)
        w["params"]["flags"] = lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM
        w["wetting_map"] = wmap
        boxes.append(lb.from_spec(w, stream=st))
    lb.batch_step(boxes, 8000)
    for b, (wmap, th) in zip(boxes, cases):
        t, c = b.observables()
        assert t["error_bits"] == 0
        f = b.fields()["psi"].reshape(shape[2], shape[1], shape[0])
        far = np.concatenate([f[:, :12, :].reshape(-1, shape[0]), f[:, 52:, :].reshape(-1, shape[0])])
        col = far.mean(axis=0)
        i = 4 + int(np.argmax((col[4:28] < 0) & (col[5:29] >= 0)))
        dx = c[0]["pos"][0] - (i + col[i] / (col[i] - col[i + 1]))
        want = -R * np.cos(np.radians(th))
        flush_print("[young] %s theta %.0f: offset %.3f (R cos theta %.3f)" % (wmap, th, dx, want))
        if wmap == "lattice":
            assert abs(dx - want) <= 0.5, (wmap, th, dx)
        else:
            assert dx < want - 0.8, (wmap, th, dx)
        b.close()


def test_active_particle_swims_along_the_interface():
    # Sec. III.C: an active Janus particle trapped at a neutral-wetting
    # interface moves along it, its axis settling towards the interface
    # plane.  Paper box (64 x 96 x 96, M_psi = 0.4 in two sub-steps), alpha =
    # 1e-3, mu = 0.1, no solubility contrast (E = 0), theta = 90 degrees, axis
    # 30 degrees out of the plane, capillary stress in divergence form.  Over
    # 12000 steps the particle stays within 1 of the plane (measured 0.41 at
    # step 6000, 0.30 at 12000), swims along the interface in the direction of
    # its in-plane axis (+6.4 between steps 6000 and 12000, 1.07e-3 per step)
    # and its axis turns into the plane (23.5 -> 16.9 degrees)
    import torch
    shape = (64, 96, 96)
    m = np.array([np.sin(np.radians(30.0)), np.cos(np.radians(30.0)), 0.0])
    col = I.janus((16.0, 48.0, 48.0), m, 4.5, alpha=1e-3, mu=0.1, theta=90.0)
    w = I.workload_paper([col], E=0.0)
    w["params"]["flags"] = lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM
    b = lb.from_spec(w, stream=torch.cuda.Stream())

    def sample():
        t, c = b.observables()
        assert t["error_bits"] == 0
        f = b.fields()["psi"].reshape(shape[2], shape[1], shape[0])
        far = np.concatenate([f[:24].reshape(-1, shape[0]), f[72:].reshape(-1, shape[0])])
        col = far.mean(axis=0)
        i = 8 + int(np.argmax((col[8:24] < 0) & (col[9:25] >= 0)))
        q = c[0]
        return (q["pos"][0] - (i + col[i] / (col[i] - col[i + 1])), q["pos"][1], q["pos"][2],
                np.degrees(np.arcsin(np.clip(q["m"][0], -1.0, 1.0))))

    b.step(6000)
    dx1, y1, z1, th1 = sample()
    b.step(6000)
    dx2, y2, z2, th2 = sample()
    flush_print("[active] offset %.3f -> %.3f, along %.3f -> %.3f, axis %.1f -> %.1f deg"
                % (dx1, dx2, y1, y2, th1, th2))
    assert abs(dx1) < 1.0 and abs(dx2) < 1.0
    assert y2 - y1 > 3.0 and abs(z2 - 48.0) < 0.5
    assert th2 < th1 < 30.0 and th2 < 20.0
    b.close()


def test_passive_offsets_grow_away_from_neutral_wetting():
    # Fig. 5A's passive points at the paper's radius: inactive particles
    # (R = 4.5, mu = 0) released on the interface of the paper box settle
    # further from the plane the more the contact angle departs from 90
    # degrees, into the phase they prefer, mirror-symmetric about 90 degrees.
    # Lattice map for H, capillary stress in divergence form, 12000 steps:
    # the offsets are ordered like -cos(theta), odd about 90 degrees to 0.02,
    # and between 0.55 and 1 of R cos(theta) (measured 0.63 at 75 and 105
    # degrees, 0.86 at 60 and 120, 0.76 at 45 and 135: a sphere of radius
    # 4.5 on this lattice sits short of the continuum Young position)
    import torch
    shape = (64, 96, 96)
    st = torch.cuda.Stream()
    ths = (45.0, 60.0, 75.0, 90.0, 105.0, 120.0, 135.0)
    boxes = []
    for th in ths:
        col = I.janus((16.0, 48.0, 48.0), (0.0, 1.0, 0.0), 4.5, alpha=0.0, mu=0.0, theta=th)
        w = I.workload_paper([col], E=0.0)
        w["params"]["flags"] = lb.LB_CAPILLARY_FORCE | lb.LB_STRESS_FORM
        w["wetting_map"] = "lattice"
        boxes.append(lb.from_spec(w, stream=st))
    lb.batch_step(boxes, 12000)
    dx = []
    for b in boxes:
        t, c = b.observables()
        assert t["error_bits"] == 0
        f = b.fields()["psi"].reshape(shape[2], shape[1], shape[0])
        far = np.concatenate([f[:24].reshape(-1, shape[0]), f[72:].reshape(-1, shape[0])])
        col = far.mean(axis=0)
        i = 8 + int(np.argmax((col[8:24] < 0) & (col[9:25] >= 0)))
        dx.append(c[0]["pos"][0] - (i + col[i] / (col[i] - col[i + 1])))
        b.close()
    flush_print("[fig5A] offsets %s" % np.round(dx, 3))
    assert all(dx[k] < dx[k + 1] for k in range(len(ths) - 1))
    for k in range(3):
        assert abs(dx[k] + dx[6 - k]) <= 0.02
        want = -4.5 * np.cos(np.radians(ths[k]))
        assert 0.55 <= dx[k] / want <= 1.0, (ths[k], dx[k])
    assert abs(dx[3]) <= 0.05
