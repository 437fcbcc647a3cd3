"""Python binding of the C ABI in include/lb.h (argument marshalling only).

Every step of the lattice update runs in the gfx950 HIP library
``csrc/liblbphoretic.so``; this module only converts arguments.  PyTorch, when
used, supplies the device arena and the stream.  There is no fallback: if the
library is absent, ``load()`` raises.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "csrc", "liblbphoretic.so")

LB_FP64, LB_FP32, LB_FP16_STORAGE = 0, 1, 2
LB_SOLUTE_FORCE, LB_EXPLICIT_COLLOID, LB_CAPILLARY_FORCE, LB_STRESS_FORM = 1, 2, 4, 8  # lb_params.flags
PRECISIONS = {"fp64": LB_FP64, "fp32": LB_FP32, "fp16": LB_FP16_STORAGE}
STATUS = {0: "LB_OK", -1: "LB_E_INVALID", -2: "LB_E_OOM", -3: "LB_E_DEVICE",
          -4: "LB_E_UNSTABLE", -5: "LB_E_STATE"}
ERR_NAN, ERR_FAST, ERR_CONTACT, ERR_LINKS = 1, 2, 4, 8
EXPORTS = ("lb_footprint_bytes", "lb_create", "lb_destroy", "lb_init_fields",
           "lb_add_colloids", "lb_step", "lb_observables", "lb_get_fields",
           "lb_get_populations", "lb_get_owner", "lb_get_links", "lb_colloid_forces",
           "lb_save_state", "lb_load_state", "lb_batch_step", "lb_batch_step_noalloc",
           "lb_set_launch_shapes",
           "lb_get_launch_shapes", "lb_timing_enable", "lb_timing_read",
           "lb_last_error", "lb_wetting_H", "lb_wetting_H_lattice", "lb_solubility_E")


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("precision", C.c_int32),
                ("rho0", C.c_double), ("tau", C.c_double),
                ("a", C.c_double), ("b", C.c_double), ("kappa", C.c_double),
                ("M_psi", C.c_double),
                ("C", C.c_double), ("E", C.c_double), ("c_b0", C.c_double),
                ("D_c", C.c_double), ("k_d", C.c_double),
                ("ext_force", C.c_double * 3), ("f16_scale", C.c_double),
                ("max_colloids", C.c_int32), ("flags", C.c_uint32),
                ("ch_substeps", C.c_int32), ("soft_eps", C.c_double), ("soft_sigma", C.c_double),
                ("soft_nu", C.c_double), ("soft_hc", C.c_double), ("lub_hc", C.c_double)]


PATTERN_MAX_BANDS, PATTERN_MAX_CELLS = 8, 64


class Colloid(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("m", C.c_double * 3),
                ("vel", C.c_double * 3), ("omega", C.c_double * 3),
                ("radius", C.c_double), ("alpha_minus", C.c_double),
                ("alpha_plus", C.c_double), ("mu_minus", C.c_double),
                ("mu_plus", C.c_double), ("H", C.c_double), ("rho_p", C.c_double),
                ("fixed", C.c_int32), ("cap_cos", C.c_double), ("e", C.c_double * 3),
                ("pattern_bands", C.c_int32), ("pattern_sectors", C.c_int32),
                ("pattern_cos", C.c_double * (PATTERN_MAX_BANDS - 1)),
                ("pattern_alpha", C.c_double * PATTERN_MAX_CELLS),
                ("pattern_mu", C.c_double * PATTERN_MAX_CELLS),
                ("pattern_H", C.c_double * PATTERN_MAX_CELLS), ("axial", C.c_double)]


class Totals(C.Structure):
    _fields_ = [("mass", C.c_double), ("mom", C.c_double * 3),
                ("sum_psi", C.c_double), ("sum_c", C.c_double),
                ("n_fluid", C.c_int64), ("n_links", C.c_int64),
                ("n_active", C.c_int64), ("step", C.c_int64),
                ("error_bits", C.c_int32)]


class LBError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


_lib = None


def load():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is missing: build it with "
                           "`python -m paper_2202_01631_amd.build`" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that copy, so the process holds one
    # HIP runtime (two runtimes in one process cannot both open the GPU)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp, dp, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)
    L.lb_footprint_bytes.argtypes = [C.POINTER(Params), C.POINTER(C.c_size_t)]
    L.lb_create.argtypes = [C.POINTER(Params), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.lb_destroy.argtypes = [vp]
    L.lb_init_fields.argtypes = [vp, dp, dp, dp, dp]
    L.lb_add_colloids.argtypes = [vp, C.POINTER(Colloid), C.c_int32]
    L.lb_step.argtypes = [vp, C.c_int64]
    L.lb_observables.argtypes = [vp, C.POINTER(Totals), C.POINTER(Colloid), C.c_int32]
    L.lb_get_fields.argtypes = [vp, dp, dp, dp, dp]
    L.lb_get_populations.argtypes = [vp, dp]
    L.lb_get_owner.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lb_get_links.argtypes = [vp, C.POINTER(C.c_int32), C.c_int64, i64p]
    L.lb_colloid_forces.argtypes = [vp, dp, C.c_int32]
    L.lb_save_state.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    L.lb_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lb_batch_step.argtypes = [C.POINTER(vp), C.c_int32, C.c_int64]
    L.lb_batch_step_noalloc.argtypes = [C.POINTER(vp), C.c_int32, C.c_int64]
    L.lb_set_launch_shapes.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lb_get_launch_shapes.argtypes = [vp, C.POINTER(C.c_int32)]
    L.lb_timing_enable.argtypes = [vp, C.c_int32]
    L.lb_timing_read.argtypes = [vp, dp, i64p]
    L.lb_last_error.argtypes = [vp]
    L.lb_last_error.restype = C.c_char_p
    L.lb_wetting_H.argtypes = [C.c_double, C.c_double, C.c_double]
    L.lb_wetting_H.restype = C.c_double
    L.lb_wetting_H_lattice.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double]
    L.lb_wetting_H_lattice.restype = C.c_double
    L.lb_solubility_E.argtypes = [C.c_double, C.c_double]
    L.lb_solubility_E.restype = C.c_double
    for name in EXPORTS:
        if name not in ("lb_last_error", "lb_wetting_H", "lb_wetting_H_lattice", "lb_solubility_E"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


PARAM_KEYS = ("rho0", "tau", "a", "b", "kappa", "M_psi", "C", "E", "c_b0", "D_c", "k_d")
COLLOID_SCALARS = ("radius", "alpha_minus", "alpha_plus", "mu_minus", "mu_plus", "H", "rho_p")


def make_params(shape, precision="fp64", **kw):
    p = Params()
    p.nx, p.ny, p.nz = (int(s) for s in shape)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    vals = dict(rho0=1.0, tau=1.0, a=0.0, b=0.0, kappa=0.0, M_psi=0.0, C=0.0, E=0.0,
                c_b0=0.0, D_c=0.0, k_d=0.0)
    vals.update({k: v for k, v in kw.items() if k in PARAM_KEYS})
    for k in PARAM_KEYS:
        setattr(p, k, float(vals[k]))
    ef = kw.get("ext_force", (0.0, 0.0, 0.0))
    for a in range(3):
        p.ext_force[a] = float(ef[a])
    p.f16_scale = float(kw.get("f16_scale", 0.0))
    p.max_colloids = int(kw.get("max_colloids", 0))
    p.ch_substeps = int(kw.get("ch_substeps", 0))
    for k in ("soft_eps", "soft_sigma", "soft_nu", "soft_hc", "lub_hc"):
        setattr(p, k, float(kw.get(k, 0.0)))
    p.flags = int(kw.get("flags", 0))
    return p


def make_colloid(d):
    q = Colloid()
    for key in ("pos", "m", "vel", "omega"):
        v = d.get(key, (0.0, 0.0, 1.0) if key == "m" else (0.0, 0.0, 0.0))
        for a in range(3):
            getattr(q, key)[a] = float(v[a])
    for key in COLLOID_SCALARS:
        setattr(q, key, float(d.get(key, 1.0 if key == "rho_p" else 0.0)))
    q.fixed = int(d.get("fixed", 0))
    q.cap_cos = float(d.get("cap_cos", 0.0))
    q.axial = float(d.get("axial", 0.0))  # spheroid semi-axis along m (0: sphere)
    e = d.get("e", (0.0, 0.0, 0.0))
    for a in range(3):
        q.e[a] = float(e[a])
    pat = d.get("pattern")
    if pat:
        # {"bands": B, "sectors": S, "cos": B-1 cuts, "alpha"/"mu"/"H": B*S values}
        q.pattern_bands, q.pattern_sectors = int(pat["bands"]), int(pat["sectors"])
        cuts = list(pat.get("cos", ()))
        if len(cuts) > PATTERN_MAX_BANDS - 1:
            raise ValueError(f"at most {PATTERN_MAX_BANDS - 1} pattern cuts")
        for i, v in enumerate(cuts):
            q.pattern_cos[i] = float(v)
        for key in ("alpha", "mu", "H"):
            vals = list(pat.get(key, ()))
            if len(vals) > PATTERN_MAX_CELLS:
                raise ValueError(f"at most {PATTERN_MAX_CELLS} pattern cells")
            for i, v in enumerate(vals):
                getattr(q, "pattern_" + key)[i] = float(v)
    return q


def colloid_dict(q):
    d = {k: np.array(getattr(q, k)[:]) for k in ("pos", "m", "vel", "omega")}
    for k in COLLOID_SCALARS:
        d[k] = getattr(q, k)
    d["fixed"] = q.fixed
    d["cap_cos"] = q.cap_cos
    d["e"] = np.array(q.e[:])
    d["axial"] = q.axial
    if q.pattern_bands > 0:
        nc = q.pattern_bands * q.pattern_sectors
        d["pattern"] = {"bands": q.pattern_bands, "sectors": q.pattern_sectors,
                        "cos": list(q.pattern_cos[:q.pattern_bands - 1]),
                        "alpha": list(q.pattern_alpha[:nc]), "mu": list(q.pattern_mu[:nc]),
                        "H": list(q.pattern_H[:nc])}
    return d


def footprint_bytes(shape, precision="fp32", **params):
    p = make_params(shape, precision, **params)
    n = C.c_size_t()
    rc = load().lb_footprint_bytes(C.byref(p), C.byref(n))
    if rc != 0:
        raise LBError(rc, load().lb_last_error(None).decode())
    return n.value


def wetting_H(theta_deg, kappa, b):
    return load().lb_wetting_H(float(theta_deg), float(kappa), float(b))


def wetting_H_lattice(theta_deg, a, b, kappa):
    return load().lb_wetting_H_lattice(float(theta_deg), float(a), float(b), float(kappa))


def solubility_E(ratio, c_b0):
    return load().lb_solubility_E(float(ratio), float(c_b0))


class Box:
    """One periodic box on the GPU.  ``arena``: optional device buffer (e.g. a
    torch uint8 CUDA tensor of at least ``footprint_bytes``) that the context
    borrows; ``stream``: optional hipStream_t handle (int) or torch stream."""

    def __init__(self, shape, precision="fp64", arena=None, stream=None, **params):
        L = load()
        self.shape = tuple(int(s) for s in shape)
        self.N = self.shape[0] * self.shape[1] * self.shape[2]
        self.precision = precision
        self.params = dict(params)
        self._arena = arena
        p = make_params(self.shape, precision, **params)
        aptr, abytes = None, 0
        if arena is not None:
            aptr = C.c_void_p(arena.data_ptr())
            abytes = arena.numel() * arena.element_size()
        sptr = None
        if stream is not None:
            sptr = C.c_void_p(getattr(stream, "cuda_stream", stream))
        self._ctx = C.c_void_p()
        rc = L.lb_create(C.byref(p), aptr, abytes, sptr, C.byref(self._ctx))
        if rc != 0:
            raise LBError(rc, L.lb_last_error(None).decode())
        self.ncol = 0

    def _check(self, rc):
        if rc != 0:
            raise LBError(rc, load().lb_last_error(self._ctx).decode())

    def close(self):
        if self._ctx:
            load().lb_destroy(self._ctx)
            self._ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, psi, c, rho=None, u=None):
        a = [np.ascontiguousarray(x, dtype=np.float64).ravel() if x is not None else None
             for x in (psi, c, rho, u)]
        self._check(load().lb_init_fields(self._ctx, *[_dp(x) for x in a]))
        self.ncol = 0

    def add_colloids(self, cols):
        arr = (Colloid * max(1, len(cols)))(*[make_colloid(d) for d in cols])
        self._check(load().lb_add_colloids(self._ctx, arr, len(cols)))
        self.ncol = len(cols)

    def step(self, n=1):
        self._check(load().lb_step(self._ctx, int(n)))

    def observables(self, check=True):
        t = Totals()
        out = (Colloid * max(1, self.ncol))()
        rc = load().lb_observables(self._ctx, C.byref(t), out, self.ncol)
        if check:
            self._check(rc)
        tot = dict(mass=t.mass, mom=np.array(t.mom[:]), sum_psi=t.sum_psi, sum_c=t.sum_c,
                   n_fluid=t.n_fluid, n_links=t.n_links, n_active=t.n_active, step=t.step,
                   error_bits=t.error_bits)
        return tot, [colloid_dict(out[k]) for k in range(self.ncol)]

    def fields(self):
        N = self.N
        rho, u, psi, c = np.empty(N), np.empty(3 * N), np.empty(N), np.empty(N)
        self._check(load().lb_get_fields(self._ctx, _dp(rho), _dp(u), _dp(psi), _dp(c)))
        return dict(rho=rho, u=u.reshape(3, N), psi=psi, c=c)

    def populations(self):
        f = np.empty(19 * self.N)
        self._check(load().lb_get_populations(self._ctx, _dp(f)))
        return f.reshape(19, self.N)

    def owner(self):
        o = np.empty(self.N, dtype=np.int32)
        self._check(load().lb_get_owner(self._ctx, o.ctypes.data_as(C.POINTER(C.c_int32))))
        return o

    def links(self):
        n = C.c_int64()
        self._check(load().lb_get_links(self._ctx, None, 0, C.byref(n)))
        rec = np.empty((max(1, n.value), 4), dtype=np.int32)
        self._check(load().lb_get_links(self._ctx, rec.ctypes.data_as(C.POINTER(C.c_int32)),
                                        n.value, C.byref(n)))
        return rec[:n.value]

    def colloid_forces(self):
        o = np.zeros(12 * max(1, self.ncol))
        self._check(load().lb_colloid_forces(self._ctx, _dp(o), self.ncol))
        o = o.reshape(-1, 12)[:self.ncol]
        return dict(F=o[:, 0:3], T=o[:, 3:6], F0=o[:, 6:9], T0=o[:, 9:12])

    def save_state(self):
        n = C.c_size_t()
        self._check(load().lb_save_state(self._ctx, None, 0, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(load().lb_save_state(self._ctx, buf, n.value, C.byref(n)))
        return buf.raw

    def load_state(self, data):
        buf = C.create_string_buffer(data, len(data))
        self._check(load().lb_load_state(self._ctx, buf, len(data)))
        self.ncol = int(np.frombuffer(data[:40], dtype=np.int32)[6])

    def set_launch_shapes(self, shapes):
        """shapes: 3 x (bx, by, remap) for the mu, collide and scalar kernels."""
        a = (C.c_int32 * 9)(*[int(v) for t in shapes for v in t])
        self._check(load().lb_set_launch_shapes(self._ctx, a))

    def launch_shapes(self):
        a = (C.c_int32 * 9)()
        self._check(load().lb_get_launch_shapes(self._ctx, a))
        return [tuple(a[3 * k:3 * k + 3]) for k in range(3)]

    def timing_enable(self, on=True):
        self._check(load().lb_timing_enable(self._ctx, 1 if on else 0))

    def timing_read(self):
        ms = (C.c_double * 6)()
        calls = (C.c_int64 * 6)()
        self._check(load().lb_timing_read(self._ctx, ms, calls))
        return np.array(ms[:]), np.array(calls[:])


def batch_step(boxes, nsteps):
    """Advance several boxes together with batched launches (one launch per
    kernel over all boxes, graph-replayed step pairs)."""
    if not boxes:
        return
    arr = (C.c_void_p * len(boxes))(*[b._ctx.value for b in boxes])
    rc = load().lb_batch_step(arr, len(boxes), int(nsteps))
    if rc != 0:
        raise LBError(rc, load().lb_last_error(boxes[0]._ctx).decode())


def batch_step_noalloc(boxes, nsteps):
    """batch_step without device allocation: the batch tables live in the
    library's fixed device array, launches go one by one (no graph)."""
    if not boxes:
        return
    arr = (C.c_void_p * len(boxes))(*[b._ctx.value for b in boxes])
    rc = load().lb_batch_step_noalloc(arr, len(boxes), int(nsteps))
    if rc != 0:
        raise LBError(rc, load().lb_last_error(boxes[0]._ctx).decode())


def spec_params(spec, **override):
    """Box parameters of a workload spec: its free-energy parameters, with E
    from the solubility ratio through the library's host helper."""
    p = dict(spec["params"])
    p.update(override)
    if "E" not in p:
        p["E"] = solubility_E(spec.get("solubility_ratio", 1.0), p.get("c_b0", 0.0))
    return p


def from_spec(spec, precision=None, arena=None, stream=None, **override):
    """Box built from a workload spec of paper_2202_01631_amd.inputs; the
    contact angle maps to H (Eq. 10, or with ``wetting_map: "lattice"`` the H
    whose flat wall this lattice wets at that angle) and the solubility ratio
    to E through the library's own host helpers."""
    p = spec_params(spec, **override)
    prec = precision or spec.get("precision", "fp64")
    b = Box(spec["shape"], prec, arena=arena, stream=stream, **p)
    b.init_fields(spec["psi"], spec["c"], spec.get("rho"), spec.get("u"))
    cols = []
    for d in spec.get("colloids", []):
        q = dict(d)
        if "H" not in q:
            th = q.get("contact_angle", 90.0)
            # Eq. 10 by default; "lattice": the angle this lattice realises
            q["H"] = (wetting_H_lattice(th, p["a"], p["b"], p["kappa"])
                      if spec.get("wetting_map") == "lattice" else wetting_H(th, p["kappa"], p["b"]))
        cols.append(q)
    if cols:
        b.add_colloids(cols)
    return b
