"""FP64 CPU oracle of the lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_2506_09242_amd``) and never imports it.

The lattice part is plain C (``lbm_oracle.c``, two-population push scheme,
FP64, OpenMP over z); this module only marshals numpy arrays through ctypes.
The learned-closure part (MLP forward/backward, Adam, box filter and SGS
targets) is plain numpy in FP64 (``oracle.mlp``).
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TAG_SOLID, TAG_BGK, TAG_TRT, TAG_SMAG, TAG_MLP, TAG_REG, TAG_WALL0 = 0, 1, 2, 3, 4, 5, 16
TAG_VIN, TAG_POUT, TAG_PIN, TAG_VOUT = 6, 7, 8, 9  # open boundaries on the x planes
TAG_RR = 10
MLP_PARAMS = 1359


class OrcConfig(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("q", C.c_int32),
                ("rho0", C.c_double), ("tau", C.c_double), ("trt_lambda", C.c_double),
                ("smag_cs", C.c_double), ("force", C.c_double * 3),
                ("wall_u", (C.c_double * 3) * 16), ("bc_u", C.c_double * 3), ("bc_rho", C.c_double * 2),
                ("flags", C.c_int32), ("pad", C.c_int32),
                ("mlp", C.POINTER(C.c_float))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        L.orc_velocity.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.orc_velocity.restype = C.c_int
        L.orc_equilibrium.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_equilibrium.restype = None
        L.orc_equilibrium3.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_equilibrium3.restype = None
        L.orc_collide_node.argtypes = [C.POINTER(OrcConfig), C.c_int, dp, dp, C.POINTER(C.c_double)]
        L.orc_collide_node.restype = C.c_int
        L.orc_init.argtypes = [C.POINTER(OrcConfig), u8, C.c_void_p, C.c_void_p, dp]
        L.orc_init.restype = None
        L.orc_run.argtypes = [C.POINTER(OrcConfig), u8, dp, C.c_int64]
        L.orc_run.restype = C.c_int
        L.orc_moments.argtypes = [C.POINTER(OrcConfig), u8, dp, dp]
        L.orc_moments.restype = None
        L.orc_fields.argtypes = [C.POINTER(OrcConfig), u8, dp, dp, dp]
        L.orc_fields.restype = None
        L.orc_bf16.argtypes = [C.c_double]
        L.orc_bf16.restype = C.c_double
        L.orc_mlp_eddy_viscosity.argtypes = [C.POINTER(C.c_float), dp, C.c_double]
        L.orc_mlp_eddy_viscosity.restype = C.c_double
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def velocity(q, i):
    """(c, w, opposite) of velocity i in the canonical order."""
    c = (C.c_int * 3)()
    w = C.c_double()
    o = lib().orc_velocity(q, i, c, C.byref(w))
    if o < 0:
        raise ValueError("bad velocity index")
    return np.array(list(c), dtype=np.int64), w.value, o


def tables(q):
    cs, ws, op = [], [], []
    for i in range(q):
        c, w, o = velocity(q, i)
        cs.append(c); ws.append(w); op.append(o)
    return np.array(cs), np.array(ws), np.array(op)


class Oracle:
    """One lattice: unshifted FP64 populations f[Q][nz][ny][nx], tags uint8."""

    def __init__(self, nx, ny, nz, q=19, tau=0.8, rho0=1.0, trt_lambda=3.0 / 16.0, smag_cs=0.0,
                 force=(0.0, 0.0, 0.0), wall_velocity=None, tags=None, free_streaming=False,
                 mlp=None, bc_velocity=(0.0, 0.0, 0.0), bc_density=(1.0, 1.0)):
        self.cfg = OrcConfig()
        self.cfg.nx, self.cfg.ny, self.cfg.nz, self.cfg.q = nx, ny, nz, q
        self.cfg.rho0, self.cfg.tau, self.cfg.trt_lambda, self.cfg.smag_cs = rho0, tau, trt_lambda, smag_cs
        for a in range(3):
            self.cfg.force[a] = force[a]
        if wall_velocity is not None:
            for k, v in enumerate(wall_velocity):
                for a in range(3):
                    self.cfg.wall_u[k][a] = v[a]
        for a in range(3):
            self.cfg.bc_u[a] = bc_velocity[a]
        self.cfg.bc_rho[0], self.cfg.bc_rho[1] = bc_density
        self.cfg.flags = 1 if free_streaming else 0
        self._mlp = None
        if mlp is not None:
            self.set_mlp(mlp)
        self.shape = (nz, ny, nx)
        self.N = nx * ny * nz
        self.q = q
        if tags is None:
            tags = np.full(self.shape, TAG_BGK, dtype=np.uint8)
        self.tags = np.ascontiguousarray(tags, dtype=np.uint8).reshape(self.shape)
        self.f = np.zeros((q,) + self.shape, dtype=np.float64)

    def set_mlp(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == MLP_PARAMS
        self._mlp = p
        self.cfg.mlp = p.ctypes.data_as(C.POINTER(C.c_float))

    def init_equilibrium(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64).reshape(self.shape)
        v = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape((3,) + self.shape)
        lib().orc_init(C.byref(self.cfg), self.tags,
                       None if r is None else r.ctypes.data, None if v is None else v.ctypes.data,
                       self.f)
        self._keep = (r, v)

    def run(self, n_steps):
        rc = lib().orc_run(C.byref(self.cfg), self.tags, self.f, int(n_steps))
        if rc != 0:
            raise RuntimeError(f"orc_run failed ({rc})")

    def moments(self):
        out = np.zeros(11)
        lib().orc_moments(C.byref(self.cfg), self.tags, self.f, out)
        return {"mass_delta": out[0], "momentum": out[1:4].copy(), "sum_u": out[4:7].copy(),
                "ke_sum": out[7], "ke_rho_sum": out[8], "n_nonfinite": int(out[9]),
                "n_fluid": int(out[10])}

    def fields(self):
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        lib().orc_fields(C.byref(self.cfg), self.tags, self.f, rho, u)
        return rho, u

    def collide_node(self, tag, fin):
        fout = np.zeros(self.q)
        nut = C.c_double(0.0)
        rc = lib().orc_collide_node(C.byref(self.cfg), tag, np.ascontiguousarray(fin, dtype=np.float64),
                                    fout, C.byref(nut))
        if rc != 0:
            raise ValueError("non-fluid tag")
        return fout, nut.value


def equilibrium(q, rho, u):
    feq = np.zeros(q)
    lib().orc_equilibrium(q, rho, np.ascontiguousarray(u, dtype=np.float64), feq)
    return feq


def equilibrium3(q, rho, u):
    """Third-order Hermite equilibrium (the recursive regularized model's)."""
    feq = np.zeros(q)
    lib().orc_equilibrium3(q, rho, np.ascontiguousarray(u, dtype=np.float64), feq)
    return feq


def bf16(v):
    return lib().orc_bf16(float(v))


def mlp_eddy_viscosity(params, feat, nu0):
    p = np.ascontiguousarray(params, dtype=np.float32)
    return lib().orc_mlp_eddy_viscosity(p.ctypes.data_as(C.POINTER(C.c_float)),
                                        np.ascontiguousarray(feat, dtype=np.float64), nu0)


def enstrophy(u):
    """(1/N) sum |curl u|^2 / 2 over a periodic all-fluid lattice, u[3][z][y][x],
    each derivative by the eighth-order centred difference (Eq. 5)."""
    a = (4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0)

    def d(f, axis):  # axis in array order (0: z, 1: y, 2: x)
        return sum(a[j - 1] * (np.roll(f, -j, axis=axis) - np.roll(f, j, axis=axis)) for j in range(1, 5))

    ux, uy, uz = u
    wx = d(uz, 1) - d(uy, 0)
    wy = d(ux, 0) - d(uz, 2)
    wz = d(uy, 2) - d(ux, 1)
    return float(np.mean(0.5 * (wx * wx + wy * wy + wz * wz)))


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))
