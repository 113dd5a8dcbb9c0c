"""FP64 CPU oracle for the polyatomic ES-BGK lattice Boltzmann scheme
(Hu et al., arXiv:1611.02409).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports,
links or executes anything in this directory, and this directory never
touches the GPU library.

The arithmetic lives in ``esbgk_oracle.c`` (plain C, double precision,
OpenMP over cells); this module compiles it with gcc and exposes it with
ctypes and numpy arrays.  Every function cites, in the C source, the part
of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esbgk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int64_p = ctypes.POINTER(ctypes.c_int64)
_c_int_p = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-Wall", "-Wno-unused-function",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_lattice_export.argtypes = [ctypes.c_int, ctypes.c_int, _c_int_p, _c_double_p, _c_double_p, _c_int_p]
        L.orc_param_map.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int, _c_double_p]
        L.orc_hermite.argtypes = [ctypes.c_int, ctypes.c_int, _c_double_p, _c_double_p]
        L.orc_hermite.restype = None
        L.orc_coeff.argtypes = [ctypes.c_int, ctypes.c_int, _c_double_p, _c_double_p, _c_double_p]
        L.orc_coeff.restype = None
        L.orc_equilibrium_order.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, _c_double_p,
                                            _c_double_p, _c_double_p]
        L.orc_sim_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, _c_int64_p]
        L.orc_sim_create.restype = ctypes.c_void_p
        L.orc_sim_destroy.argtypes = [ctypes.c_void_p]
        L.orc_sim_destroy.restype = None
        L.orc_sim_init.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p]
        L.orc_sim_init.restype = None
        L.orc_sim_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.orc_sim_step.restype = None
        L.orc_sim_moments.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p]
        L.orc_sim_moments.restype = None
        L.orc_sim_totals.argtypes = [ctypes.c_void_p, _c_double_p]
        L.orc_sim_totals.restype = None
        L.orc_sim_get_pops.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p]
        L.orc_sim_get_pops.restype = None
        L.orc_sim_set_pops.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p]
        L.orc_sim_set_pops.restype = None
        L.orc_sim_steps.argtypes = [ctypes.c_void_p]
        L.orc_sim_steps.restype = ctypes.c_int64
        L.orc_sim_params.argtypes = [ctypes.c_void_p, _c_double_p]
        L.orc_sim_params.restype = None
        L.orc_sim_set_walls.argtypes = [ctypes.c_void_p, _c_double_p, _c_double_p]
        L.orc_sim_set_walls.restype = ctypes.c_int
        L.orc_sim_set_open_x.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_sim_set_open_x.restype = ctypes.c_int
        L.orc_collide_cells.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, ctypes.c_int64, _c_double_p, _c_double_p,
                                        _c_double_p, _c_double_p]
        L.orc_cell_moments_many.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                            ctypes.c_int64, _c_double_p, _c_double_p, _c_double_p]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_c_double_p)


def set_threads(n: int = 0) -> int:
    """Set (n > 0) and return the OpenMP thread count the oracle uses."""
    return lib().orc_set_threads(int(n))


class Lattice:
    """Velocity set solved from the moment conditions: c (Q x 3 int), w, r, opp."""

    def __init__(self, D: int, Q: int):
        c = np.zeros(3 * Q, dtype=np.int32)
        w = np.zeros(Q)
        r = ctypes.c_double()
        opp = np.zeros(Q, dtype=np.int32)
        rc = lib().orc_lattice_export(D, Q, c.ctypes.data_as(_c_int_p), _p(w), ctypes.byref(r),
                                      opp.ctypes.data_as(_c_int_p))
        if rc:
            raise ValueError(f"oracle: no lattice D{D}Q{Q} (code {rc})")
        self.D, self.Q = D, Q
        self.c = c.reshape(Q, 3)[:, :D].copy()
        self.w, self.r, self.opp = w, r.value, opp

    @property
    def xi(self) -> np.ndarray:
        return self.r * self.c


def param_map(D: int, Nf: int, Pr: float, tau: float, kappa: float = 0.2, reading: str = "B") -> dict:
    out = np.zeros(4)
    rc = lib().orc_param_map(D, Nf, Pr, tau, kappa, 0 if reading == "B" else 1, _p(out))
    if rc:
        raise ValueError("oracle: invalid parameters")
    return dict(omega=out[0], omega_s=out[1], nu=out[2], gamma=out[3])


def hermite(n: int, xi) -> np.ndarray:
    """Grad's Hermite tensor H^(n)(xi), shape (D,)*n (index order as numpy)."""
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    D = xi.shape[0]
    out = np.zeros(D ** n)
    lib().orc_hermite(n, D, _p(xi), _p(out))
    # C stores the first index fastest; numpy reshape with order='F' gives [i1, i2, ...]
    return out.reshape((D,) * n, order="F") if n else out.reshape(())


def coeff(n: int, u, A) -> np.ndarray:
    """General-term Hermite coefficient a^(n)(u, A = Lambda - delta), shape (D,)*n."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    D = u.shape[0]
    out = np.zeros(D ** n)
    lib().orc_coeff(n, D, _p(u), _p(A), _p(out))
    return out.reshape((D,) * n, order="F") if n else out.reshape(())


def equilibrium(D: int, Q: int, rho: float, u, A, order: int = 4) -> np.ndarray:
    """Discrete target G_i(rho, u, Lambda = A + delta) truncated at Hermite order `order`."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    G = np.zeros(Q)
    rc = lib().orc_equilibrium_order(D, Q, order, float(rho), _p(u), _p(A), _p(G))
    if rc:
        raise ValueError(f"oracle: equilibrium failed ({rc})")
    return G


def collide_cells(D, Q, Nf, Pr, tau, kappa, fin, gin=None, reading="B"):
    """Post-collision populations of independent cells; fin/gin shape (n, Q)."""
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    n = fin.shape[0]
    fout = np.zeros_like(fin)
    if Nf > 0:
        gin = np.ascontiguousarray(gin, dtype=np.float64)
        gout = np.zeros_like(gin)
    else:
        gin = gout = None
    rc = lib().orc_collide_cells(D, Q, Nf, Pr, tau, kappa, 0 if reading == "B" else 1, n, _p(fin), _p(gin),
                                 _p(fout), _p(gout))
    if rc:
        raise ValueError("oracle: collide failed")
    return fout, gout


def cell_moments(D, Q, Nf, fin, gin=None, kappa=0.2):
    """Moments of independent cells: dict rho, u (n, D), T (T_eq), P (n, D(D+1)/2)."""
    fin = np.ascontiguousarray(fin, dtype=np.float64)
    n = fin.shape[0]
    gin = np.ascontiguousarray(gin, dtype=np.float64) if Nf > 0 else None
    out = np.zeros((n, 11))
    lib().orc_cell_moments_many(D, Q, Nf, kappa, n, _p(fin), _p(gin), _p(out))
    npc = D * (D + 1) // 2
    return dict(rho=out[:, 0].copy(), u=out[:, 1:1 + D].copy(), T=out[:, 4].copy(), P=out[:, 5:5 + npc].copy())


class Sim:
    """FP64 simulation (two buffers, collide then pull-stream), periodic, or
    with diffusely reflecting walls normal to y (set_walls)."""

    def __init__(self, D, Q, Nf, Pr, tau, dims, kappa=0.2, reading="B"):
        self.D, self.Q, self.Nf = D, Q, Nf
        self.dims = tuple(int(d) for d in dims)
        assert len(self.dims) == D
        d = np.array(list(self.dims) + [1] * (3 - D), dtype=np.int64)
        h = lib().orc_sim_create(D, Q, Nf, Pr, tau, kappa, 0 if reading == "B" else 1,
                                 d.ctypes.data_as(_c_int64_p))
        if not h:
            raise ValueError("oracle: could not create simulation")
        self._h = h
        self.ncell = int(np.prod(self.dims))
        # fields are indexed [z][y][x] -> numpy shape reversed
        self.shape = tuple(reversed(self.dims))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_sim_destroy(h)
            self._h = None

    def init(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        assert rho.size == self.ncell and T.size == self.ncell and u.size == self.D * self.ncell
        lib().orc_sim_init(self._h, _p(rho), _p(u), _p(T))

    def step(self, n=1):
        lib().orc_sim_step(self._h, int(n))

    @property
    def steps(self):
        return lib().orc_sim_steps(self._h)

    def params(self):
        out = np.zeros(5)
        lib().orc_sim_params(self._h, _p(out))
        return dict(omega=out[0], omega_s=out[1], nu=out[2], gamma=out[3], kappa=out[4])

    def moments(self, with_P=False):
        rho = np.zeros(self.ncell)
        u = np.zeros(self.D * self.ncell)
        T = np.zeros(self.ncell)
        npc = self.D * (self.D + 1) // 2
        P = np.zeros(npc * self.ncell) if with_P else None
        lib().orc_sim_moments(self._h, _p(rho), _p(u), _p(T), _p(P))
        out = dict(rho=rho.reshape(self.shape), u=u.reshape((self.D,) + self.shape), T=T.reshape(self.shape))
        if with_P:
            out["P"] = P.reshape((npc,) + self.shape)
        return out

    def totals(self):
        out = np.zeros(2 + self.D)
        lib().orc_sim_totals(self._h, _p(out))
        return out

    def set_walls(self, bottom, top):
        """Diffusely reflecting walls normal to y: bottom/top = (u_x, u_y, T)
        (2D) or (u_x, u_y, u_z, T) (3D) of the wall at low / high y.  The
        first and last `reach` rows become ghost rows outside the gas."""
        def w(v):
            v = list(v)
            return np.array(v[:-1] + [0.0] * (3 - (len(v) - 1)) + [v[-1]], dtype=np.float64)
        b, t = w(bottom), w(top)
        if lib().orc_sim_set_walls(self._h, _p(b), _p(t)) != 0:
            raise ValueError("oracle: domain too short for walls")

    def set_open_x(self, on=True):
        """Open (zero-gradient) ends along x: the first and last `reach_x`
        columns become ghost columns that repeat the nearest gas column."""
        if lib().orc_sim_set_open_x(self._h, 1 if on else 0) != 0:
            raise ValueError("oracle: domain too narrow for open ends, or walls are set")

    def get_pops(self):
        f = np.zeros(self.Q * self.ncell)
        g = np.zeros(self.Q * self.ncell) if self.Nf > 0 else None
        lib().orc_sim_get_pops(self._h, _p(f), _p(g))
        f = f.reshape((self.Q,) + self.shape)
        return f, (g.reshape((self.Q,) + self.shape) if g is not None else None)

    def set_pops(self, f, g=None):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1) if self.Nf > 0 else None
        lib().orc_sim_set_pops(self._h, _p(f), _p(g))
