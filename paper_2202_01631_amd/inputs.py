"""Seeded synthetic inputs for the lattice update.

This module only draws numbers and lays them out: SplitMix64 streams, uniform
noise, initial interface profiles and colloid placements.  It holds none of the
solver's arithmetic and is shared by the solver's tests and benchmark and by
the oracle's tests, which receive identical FP64 arrays from it.

Workload specifications are plain dicts.  Physical parameters that the paper
states through derived quantities (the contact angle of Eq. 10, the
solubility ratio that sets E in Eq. 1) are carried as those quantities
(``contact_angle`` in degrees, ``solubility_ratio``); each consumer maps them
to H and E itself.
"""
import math

import numpy as np

MASK64 = (1 << 64) - 1
BASE_SEED = 2202016310


def splitmix64(seed, n):
    """n successive outputs of SplitMix64 (Steele, Lea, Flood 2014) from `seed`."""
    out = np.empty(n, dtype=np.uint64)
    s = np.uint64(seed & MASK64)
    # vectorised: state_k = seed + (k+1) * golden, then the output mix
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = s + k * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        out[:] = z ^ (z >> np.uint64(31))
    return out


def uniform(seed, n):
    """U[0,1) doubles from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def noise(seed, n, amp):
    """amp * (2u - 1), x-fastest node order."""
    return amp * (2.0 * uniform(seed, n) - 1.0)


def gaussian(seed, n):
    """Standard normals by Box-Muller from one uniform stream."""
    u = uniform(seed, 2 * n)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def coords(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel().astype(np.float64), y.ravel().astype(np.float64), z.ravel().astype(np.float64)


def flat_interface(shape, z0, width, amp=0.0, seed=BASE_SEED):
    """psi = tanh((z - z0)/width) + amp*(2u-1): one flat interface (the periodic
    wrap leaves a second, sharp one)."""
    _, _, z = coords(shape)
    psi = np.tanh((z - z0) / width)
    if amp:
        psi = psi + noise(seed, psi.size, amp)
    return psi


def slab(shape, width, amp=0.0, seed=BASE_SEED, axis=2, offset=0.0):
    """Two smooth interfaces at L/4 + offset and 3L/4 - offset along `axis`:
    psi = -tanh((s - z1)/width) * tanh((s - z2)/width)  (+1 in the middle slab)."""
    s = coords(shape)[axis]
    L = shape[axis]
    z1, z2 = L / 4.0 + offset, 3.0 * L / 4.0 - offset
    psi = -np.tanh((s - z1) / width) * np.tanh((s - z2) / width)
    if amp:
        psi = psi + noise(seed, psi.size, amp)
    return psi


def unit_vectors(seed, n):
    g = gaussian(seed, 3 * n).reshape(n, 3)
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def place_spheres(shape, n, radius, z_choices, gap, seed, max_tries=200000):
    """Seeded non-overlapping sphere centres (minimum-image surface gap >= gap).
    z_choices(u) maps a uniform draw to a z coordinate."""
    L = np.array(shape, dtype=np.float64)
    u = uniform(seed, 4 * max_tries).reshape(max_tries, 4)
    centres = []
    for t in range(max_tries):
        if len(centres) == n:
            break
        c = np.array([u[t, 0] * L[0], u[t, 1] * L[1], z_choices(u[t, 2], u[t, 3])])
        ok = True
        for q in centres:
            d = c - q
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < 2 * radius + gap:
                ok = False
                break
        if ok:
            centres.append(c)
    if len(centres) < n:
        raise RuntimeError("could not place %d spheres" % n)
    return np.array(centres)


# ---------------------------------------------------------------- workloads
FREE_ENERGY = dict(rho0=1.0, tau=1.0, a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.1,
                   C=0.0625, c_b0=0.5, D_c=0.1, k_d=1e-3)
# equilibrium interface width sqrt(2 kappa/|a|) for the parameters above
WIDTH = math.sqrt(2.0 * 0.04 / 0.0625)


def janus(pos, m, radius, alpha=1e-3, mu=0.1, theta=90.0, rho_p=1.0, mu_minus=None,
          mu_plus=None, fixed=0):
    return dict(pos=np.asarray(pos, dtype=np.float64), m=np.asarray(m, dtype=np.float64),
                vel=np.zeros(3), omega=np.zeros(3), radius=float(radius),
                alpha_minus=float(alpha), alpha_plus=0.0,
                mu_minus=float(mu if mu_minus is None else mu_minus),
                mu_plus=float(mu if mu_plus is None else mu_plus),
                contact_angle=float(theta), rho_p=float(rho_p), fixed=int(fixed))


def workload_small(seed=BASE_SEED):
    """32^3 periodic box, 200 steps, FP64: flat interface at z = 16 with
    uniform noise +-0.01, c = 0, 2:1 solubility contrast, one Janus sphere of
    radius 4 at (16,16,12), axis +z, emitting 1e-3 per active link, 90 deg."""
    shape = (32, 32, 32)
    psi = flat_interface(shape, 16.0, WIDTH, 0.01, seed)
    return dict(name="box32_fp64", shape=shape, precision="fp64", steps=200,
                params=dict(FREE_ENERGY), solubility_ratio=2.0,
                psi=psi, c=np.zeros(psi.size),
                colloids=[janus((16.0, 16.0, 12.0), (0.0, 0.0, 1.0), 4.0)])


# the paper's own regime (Sec. II.C): A = C = 0.0625, kappa = 0.04,
# M_psi = 0.4 (two psi/c sub-steps per step), M_phi = 0.8 (D_c = C M_phi =
# 0.05), k_d = 1e-3, R = 4.5, 64 x 96 x 96 box, flat interfaces normal to x;
# particles feel the capillary stress (option flag 4)
PAPER_REGIME = dict(rho0=1.0, tau=1.0, a=-0.0625, b=0.0625, kappa=0.04, M_psi=0.4,
                    C=0.0625, c_b0=0.0, D_c=0.05, k_d=1e-3, ch_substeps=2, flags=4)


def workload_paper(particles, E=-0.25, shape=(64, 96, 96), single_phase=False):
    """Box of the paper's regime: psi = -tanh((x - L/4)/w) tanh((x - 3L/4)/w)
    (interfaces at x = 16 and 48 for L = 64, psi > 0 between them), c = 0, or
    with single_phase psi = 0 and A = kappa = E = 0.  `particles`: list of
    janus() dicts (radius 4.5 in the paper)."""
    p = dict(PAPER_REGIME, E=E)
    if single_phase:
        p.update(a=0.0, b=0.0, kappa=0.0, E=0.0)
        psi = np.zeros(int(np.prod(shape)))
    else:
        psi = slab(shape, WIDTH, axis=0)
    return dict(name="paper_%dx%dx%d" % shape, shape=shape, precision="fp32", params=p,
                psi=psi, c=np.zeros(psi.size), colloids=list(particles))


def workload_single(n=128, seed=BASE_SEED + 1, theta=None, ratio=None, mu=None):
    """n^3 FP32 box: flat interface at n/2, noise +-0.01, one Janus sphere of
    radius 8 centred on the interface; contact angle from {60, 90, 120},
    mobility +-0.1, solubility ratio 1..5 drawn from the seed."""
    u = uniform(seed, 8)
    theta = theta if theta is not None else (60.0, 90.0, 120.0)[int(u[0] * 3)]
    ratio = ratio if ratio is not None else 1.0 + 4.0 * u[1]
    mu = mu if mu is not None else (-0.1, 0.1)[int(u[2] * 2)]
    m = unit_vectors(seed + 7, 1)[0]
    shape = (n, n, n)
    psi = flat_interface(shape, n / 2.0, WIDTH, 0.01, seed)
    h = n / 2.0
    return dict(name="box%d_fp32" % n, shape=shape, precision="fp32", steps=10000,
                params=dict(FREE_ENERGY), solubility_ratio=ratio, psi=psi,
                c=np.zeros(psi.size),
                colloids=[janus((h + 0.37, h - 0.21, h + 0.13), m, 8.0, mu=mu, theta=theta)])


def workload_many(n=256, count=64, radius=6.0, precision="fp16", seed=BASE_SEED + 2):
    """n^3 box, planar interface at n/2, `count` Janus spheres of radius 6 at
    seeded non-overlapping positions (surface gap >= 2), uniformly random
    orientations; half centred on the interface, half near it
    (|z - z_int| in [radius+2, radius+6], either side)."""
    shape = (n, n, n)
    zi = n / 2.0
    half = count // 2
    at = place_spheres(shape, half, radius, lambda a, b: zi, 2.0, seed)

    def near(a, b):
        d = radius + 2.0 + 4.0 * a
        return zi + d if b < 0.5 else zi - d

    # the "near" set must also avoid the "at" set: place all together
    pts = list(at)
    L = np.array(shape, dtype=np.float64)
    u = uniform(seed + 11, 4 * 200000).reshape(-1, 4)
    t = 0
    while len(pts) < count:
        c = np.array([u[t, 0] * L[0], u[t, 1] * L[1], near(u[t, 2], u[t, 3])])
        t += 1
        ok = True
        for q in pts:
            d = c - q
            d -= L * np.round(d / L)
            if np.linalg.norm(d) < 2 * radius + 2.0:
                ok = False
                break
        if ok:
            pts.append(c)
    ms = unit_vectors(seed + 5, count)
    uu = uniform(seed + 6, 3 * count).reshape(count, 3)
    cols = []
    for k in range(count):
        theta = (60.0, 90.0, 120.0)[int(uu[k, 0] * 3)]
        mu = -0.1 + 0.2 * uu[k, 1]
        cols.append(janus(pts[k], ms[k], radius, mu=mu, theta=theta))
    psi = flat_interface(shape, zi, WIDTH, 0.01, seed)
    return dict(name="box%d_%dspheres_%s" % (n, count, precision), shape=shape,
                precision=precision, steps=5000, params=dict(FREE_ENERGY),
                solubility_ratio=2.0, psi=psi, c=np.zeros(psi.size), colloids=cols)


def batch_boxes(count=512, seed=BASE_SEED + 3, sides=(32, 48, 64), steps=2000):
    """`count` independent boxes: side uniform in `sides`, interface at L/2,
    one Janus sphere of radius 4.5 on it; mobility from {-0.2,...,0.2} step
    0.05, contact angle from {45,...,135} step 10, ratio from {1..5}."""
    u = uniform(seed, 8 * count).reshape(count, 8)
    mus = np.round(np.arange(-0.2, 0.2001, 0.05), 10)
    thetas = np.arange(45.0, 135.01, 10.0)
    out = []
    for b in range(count):
        L = sides[int(u[b, 0] * len(sides))]
        mu = float(mus[int(u[b, 1] * len(mus))])
        th = float(thetas[int(u[b, 2] * len(thetas))])
        ratio = float(1 + int(u[b, 3] * 5))
        m = unit_vectors(seed + 100 + b, 1)[0]
        shape = (L, L, L)
        h = L / 2.0
        psi = flat_interface(shape, h, WIDTH, 0.01, seed + 1000 + b)
        out.append(dict(name="batch%d" % b, shape=shape, precision="fp32", steps=steps,
                        params=dict(FREE_ENERGY), solubility_ratio=ratio, psi=psi,
                        c=np.zeros(psi.size),
                        colloids=[janus((h + u[b, 4] - 0.5, h + u[b, 5] - 0.5, h), m, 4.5,
                                        mu=mu, theta=th)]))
    return out


def serving_trace(n_requests=500, rate=50.0, seed=BASE_SEED + 4, sides=(32, 96),
                  steps=(2000, 20000)):
    """Poisson arrivals at `rate`/s of sweep requests: side uniform in
    [sides], 1-8 spheres of radius 4.5, steps uniform in [steps], accuracy
    class tight (FP32) or loose (FP16 storage) with equal odds.  Returns
    (arrival_time, spec-parameters) pairs; the fields are generated on
    admission by `serving_request`."""
    u = uniform(seed, 8 * n_requests).reshape(n_requests, 8)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += -math.log(1.0 - u[r, 0]) / rate
        L = int(sides[0] + int(u[r, 1] * (sides[1] - sides[0] + 1)))
        nsph = 1 + int(u[r, 2] * 8)
        st = int(steps[0] + int(u[r, 3] * (steps[1] - steps[0] + 1)))
        prec = "fp32" if u[r, 4] < 0.5 else "fp16"
        out.append(dict(t=t, side=L, spheres=nsph, steps=st, precision=prec,
                        seed=seed + 10000 + r, mu=-0.2 + 0.4 * u[r, 5],
                        theta=45.0 + 90.0 * u[r, 6], ratio=1.0 + 4.0 * u[r, 7]))
    return out


def serving_request(req):
    L = req["side"]
    shape = (L, L, L)
    n = req["spheres"]
    radius = 4.5
    # at most what fits: centres within +-(radius+4) of the interface
    zi = L / 2.0
    seed = req["seed"]
    pts = place_spheres(shape, n, radius,
                        lambda a, b: zi + (2.0 * a - 1.0) * (radius + 4.0), 2.0, seed)
    ms = unit_vectors(seed + 1, n)
    cols = [janus(pts[k], ms[k], radius, mu=req["mu"], theta=req["theta"]) for k in range(n)]
    psi = flat_interface(shape, zi, WIDTH, 0.01, seed + 2)
    return dict(name="req%d" % seed, shape=shape, precision=req["precision"],
                steps=req["steps"], params=dict(FREE_ENERGY),
                solubility_ratio=req["ratio"], psi=psi, c=np.zeros(psi.size),
                colloids=cols)
