"""MI355X (gfx950) ES-BGK lattice Boltzmann stream-collide library.

Thin ctypes binding of the C ABI in ``include/esbgk.h``: every call marshals
numpy arrays and forwards to ``libesbgk.so``; all arithmetic of the scheme
runs in the library's HIP kernels.  PyTorch supplies device memory (the
population storage is a torch uint8 tensor) and the HIP stream.

The library must have been built (``python paper_1611_02409_amd/build.py``);
importing this package without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded first so that the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesbgk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1611_02409_amd/build.py`")

_lib = ctypes.CDLL(LIB_PATH)

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p

F32, F16_DEV, BF16_DEV = 0, 1, 2
STORAGE = {"f32": F32, "f16": F16_DEV, "bf16": BF16_DEV}
PULL = 0x10   # two-copy pull streaming (or-ed into the storage code)
STREAMING = {"aa": 0, "pull": PULL}


def _storage_code(storage: str, streaming: str = "aa", plane_pad: int = 0) -> int:
    """Storage argument of the C ABI; plane_pad is the padding after every
    plane in bytes (a multiple of 4096, at most 255 * 4096)."""
    if storage not in STORAGE:
        raise ValueError(f"storage must be one of {sorted(STORAGE)}")
    if streaming not in STREAMING:
        raise ValueError(f"streaming must be one of {sorted(STREAMING)}")
    if plane_pad % 4096 or not 0 <= plane_pad <= 255 * 4096:
        raise ValueError("plane_pad must be a multiple of 4096 bytes in [0, 255 * 4096]")
    return STORAGE[storage] | STREAMING[streaming] | ((plane_pad // 4096) << 8)


ERRORS = {-1: "EINVAL", -2: "EUNSUPPORTED", -3: "ENOMEM", -4: "EDEVICE", -5: "ESTATE", -6: "ENONFINITE", -7: "EIO"}


class EsbgkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def _sig(name, args, res=ctypes.c_int):
    fn = getattr(_lib, name)
    fn.argtypes = args
    fn.restype = res
    return fn


_sig("esbgk_last_error", [], ctypes.c_char_p)
_sig("esbgk_version", [], ctypes.c_char_p)
_sig("esbgk_lattice_info", [ctypes.c_int, ctypes.c_int, _ip, _dp, _dp, _ip])
_sig("esbgk_params", [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp])
_sig("esbgk_create", [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _i64p, ctypes.c_int,
                      ctypes.POINTER(_vp)])
_sig("esbgk_create_ex", [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _i64p,
                         ctypes.c_int, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)])
_sig("esbgk_storage_bytes", [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64p, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_size_t)])
_sig("esbgk_set_kappa", [_vp, ctypes.c_double])
_sig("esbgk_set_stream", [_vp, _vp])
_sig("esbgk_init_fields", [_vp, _dp, _dp, _dp])
_sig("esbgk_step", [_vp, ctypes.c_int64])
_sig("esbgk_set_walls", [_vp, _dp, _dp])
_sig("esbgk_set_open_x", [_vp, ctypes.c_int])
_sig("esbgk_step_count", [_vp, _i64p])
_sig("esbgk_plane_pad", [_vp, _i64p])
_sig("esbgk_read_moments", [_vp, _dp, _dp, _dp, _dp])
_sig("esbgk_totals", [_vp, _dp])
_sig("esbgk_read_cells", [_vp, ctypes.c_int64, _i64p, _dp, _dp])
_sig("esbgk_read_populations", [_vp, _dp, _dp])
_sig("esbgk_write_populations", [_vp, _dp, _dp])
_sig("esbgk_save", [_vp, ctypes.c_char_p])
_sig("esbgk_load", [_vp, ctypes.c_char_p])
_sig("esbgk_step_timed", [_vp, ctypes.c_int64, _dp, _dp])
_sig("esbgk_set_tile", [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int])
_sig("esbgk_get_tile", [_vp, ctypes.c_int, _ip, _ip, _ip, _ip])
_sig("esbgk_autotune", [_vp, ctypes.c_double, ctypes.c_char_p])
_sig("esbgk_destroy", [_vp], None)
_sig("esbgk_stream_ceiling", [ctypes.c_int64, ctypes.c_int, _dp])
_sig("esbgk_stream_ceiling_planes", [ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp])


def stream_ceiling(cells: int = 4096 * 4096, reps: int = 10, planes: int = 74, sets: int = 2) -> float:
    """GB/s (read plus written) of an arithmetic-free read and write of
    `planes` 4-byte planes (in `sets` sets) of `cells` cells: the best over
    buffer placements, occupancies, store cache policies and plane strides."""
    out = ctypes.c_double()
    _check(_lib.esbgk_stream_ceiling_planes(int(cells), int(planes), int(sets), int(reps), ctypes.byref(out)))
    return out.value


def _check(rc: int):
    if rc != 0:
        raise EsbgkError(rc, _lib.esbgk_last_error().decode())


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def version() -> str:
    return _lib.esbgk_version().decode()


def lattice_info(D: int, Q: int) -> dict:
    """Velocities c (Q x D), weights w, scale r and reach of a lattice, in the
    library's storage order."""
    c = np.zeros(3 * Q, dtype=np.int32)
    w = np.zeros(Q)
    r = ctypes.c_double()
    reach = ctypes.c_int()
    _check(_lib.esbgk_lattice_info(D, Q, c.ctypes.data_as(_ip), _p(w), ctypes.byref(r), ctypes.byref(reach)))
    return dict(c=c.reshape(Q, 3)[:, :D].copy(), w=w, r=r.value, reach=reach.value)


def params(D: int, Nf: int, Pr: float, tau: float, kappa: float = 0.2) -> dict:
    out = np.zeros(4)
    _check(_lib.esbgk_params(D, Nf, Pr, tau, kappa, _p(out)))
    return dict(omega=out[0], omega_s=out[1], nu=out[2], gamma=out[3])


def _dims(dims):
    return (ctypes.c_int64 * 3)(*(list(dims) + [1] * (3 - len(dims))))


def storage_bytes(D, Q, Nf, dims, storage="f32", streaming="aa", plane_pad=0) -> int:
    out = ctypes.c_size_t()
    _check(_lib.esbgk_storage_bytes(D, Q, Nf, _dims(dims), _storage_code(storage, streaming, plane_pad),
                                    ctypes.byref(out)))
    return out.value


class Lattice:
    """One periodic domain.  Fields use numpy shape (ny, nx) / (nz, ny, nx),
    velocity (D, ...).  streaming: "aa" (one copy, A-A in place) or "pull"
    (two copies, aligned stores; same results bit for bit).  plane_pad:
    unused bytes after every plane (a multiple of 4096), which moves the
    planes' address streams apart; results do not depend on it."""

    def __init__(self, D: int, Q: int, Nf: int, Pr: float, tau: float, dims, storage: str = "f32",
                 kappa: float = 0.2, device: int = 0, stream=None, streaming: str = "aa", plane_pad: int = 0,
                 owned: bool = False):
        self.D, self.Q, self.Nf, self.Pr, self.tau = D, Q, Nf, Pr, tau
        self.dims = tuple(int(d) for d in dims)
        if len(self.dims) != D:
            raise ValueError("dims must have D entries")
        self.storage = storage
        self.streaming = streaming
        code = _storage_code(storage, streaming, plane_pad)
        self.plane_pad = plane_pad
        self.ncell = int(np.prod(self.dims))
        self.shape = tuple(reversed(self.dims))
        self._h = None
        nbytes = storage_bytes(D, Q, Nf, self.dims, storage, streaming, plane_pad)
        self.device = torch.device("cuda", device)
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = _vp()
        if owned:
            # the library allocates (and may move, see autotune) the storage
            self._buf = None
            with torch.cuda.device(self.device):
                _check(_lib.esbgk_create(D, Q, Nf, Pr, tau, _dims(self.dims), code, ctypes.byref(h)))
            self._h = h
            _check(_lib.esbgk_set_stream(h, self._stream.cuda_stream))
        else:
            self._buf = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            _check(_lib.esbgk_create_ex(D, Q, Nf, Pr, tau, _dims(self.dims), code, self._buf.data_ptr(),
                                        nbytes, self._stream.cuda_stream, ctypes.byref(h)))
            self._h = h
        if kappa != 0.2:
            self.set_kappa(kappa)

    # the destroy function is bound at definition: module globals may already
    # be cleared when the interpreter collects handles at exit
    def __del__(self, _destroy=_lib.esbgk_destroy):
        h = getattr(self, "_h", None)
        if h:
            _destroy(h)
            self._h = None

    @property
    def stream(self):
        return self._stream

    @property
    def storage_tensor(self) -> torch.Tensor:
        """The caller-owned storage (None when the library owns it)."""
        return self._buf

    @property
    def plane_pad_bytes(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.esbgk_plane_pad(self._h, ctypes.byref(v)))
        return v.value

    def set_kappa(self, kappa: float):
        _check(_lib.esbgk_set_kappa(self._h, kappa))

    def set_stream(self, stream):
        self._stream = stream
        _check(_lib.esbgk_set_stream(self._h, stream.cuda_stream))

    def set_walls(self, bottom, top):
        """Diffusely reflecting walls at low and high y (the thermal Couette
        flow of Sec. VI.A): bottom/top = (u_x, u_y, T) in 2D or
        (u_x, u_y, u_z, T) in 3D; None, None removes them.  The first and last
        `reach` rows become ghost rows outside the gas; needs streaming="pull"."""
        if bottom is None and top is None:
            _check(_lib.esbgk_set_walls(self._h, None, None))
            return

        def wall(v):
            v = _f64(v, self.D + 1)
            out = np.zeros(4)
            out[:self.D], out[3] = v[:self.D], v[self.D]
            return out

        b, t = wall(bottom), wall(top)
        _check(_lib.esbgk_set_walls(self._h, _p(b), _p(t)))

    def set_open_x(self, on: bool = True):
        """Open (zero-gradient) ends along x (the shock tube of Sec. VI.B): the
        first and last `reach_x` columns become ghost columns repeating the
        nearest gas column; needs streaming="pull"."""
        _check(_lib.esbgk_set_open_x(self._h, 1 if on else 0))

    def init_fields(self, rho, u, T):
        n = self.ncell
        _check(_lib.esbgk_init_fields(self._h, _p(_f64(rho, n)), _p(_f64(u, self.D * n)), _p(_f64(T, n))))

    def step(self, n: int = 1):
        _check(_lib.esbgk_step(self._h, int(n)))

    @property
    def steps(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.esbgk_step_count(self._h, ctypes.byref(v)))
        return v.value

    def read_moments(self, with_P: bool = False) -> dict:
        n = self.ncell
        rho, u, T = np.zeros(n), np.zeros(self.D * n), np.zeros(n)
        npc = self.D * (self.D + 1) // 2
        P = np.zeros(npc * n) if with_P else None
        _check(_lib.esbgk_read_moments(self._h, _p(rho), _p(u), _p(T), _p(P)))
        out = dict(rho=rho.reshape(self.shape), u=u.reshape((self.D,) + self.shape), T=T.reshape(self.shape))
        if with_P:
            out["P"] = P.reshape((npc,) + self.shape)
        return out

    def totals(self) -> np.ndarray:
        out = np.zeros(2 + self.D)
        _check(_lib.esbgk_totals(self._h, _p(out)))
        return out

    def read_cells(self, cells):
        cells = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
        f = np.zeros((cells.size, self.Q))
        g = np.zeros((cells.size, self.Q)) if self.Nf > 0 else None
        _check(_lib.esbgk_read_cells(self._h, cells.size, cells.ctypes.data_as(_i64p), _p(f), _p(g)))
        return f, g

    def read_populations(self):
        f = np.zeros(self.Q * self.ncell)
        g = np.zeros(self.Q * self.ncell) if self.Nf > 0 else None
        _check(_lib.esbgk_read_populations(self._h, _p(f), _p(g)))
        f = f.reshape((self.Q,) + self.shape)
        return f, (g.reshape((self.Q,) + self.shape) if g is not None else None)

    def write_populations(self, f, g=None):
        n = self.Q * self.ncell
        _check(_lib.esbgk_write_populations(self._h, _p(_f64(f, n)), _p(_f64(g, n)) if self.Nf > 0 else None))

    def save(self, path: str):
        _check(_lib.esbgk_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        _check(_lib.esbgk_load(self._h, os.fsencode(path)))

    def step_timed(self, n: int):
        tot = ctypes.c_double()
        per = np.zeros(int(n))
        _check(_lib.esbgk_step_timed(self._h, int(n), ctypes.byref(tot), _p(per)))
        return tot.value, per

    def set_tile(self, block: int = 0, order: int = 0, policy: int = 0, cells_per_item: int = 0, parity: int = -1):
        _check(_lib.esbgk_set_tile(self._h, parity, block, order, policy, cells_per_item))

    def get_tile(self, parity: int | None = None):
        """(block, order, policy, cells_per_item) of one parity's kernel, or
        a pair (even, odd) when parity is None."""
        if parity is None:
            return self.get_tile(0), self.get_tile(1)
        b, o, p, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.esbgk_get_tile(self._h, parity, ctypes.byref(b), ctypes.byref(o), ctypes.byref(p),
                                   ctypes.byref(k)))
        return b.value, o.value, p.value, k.value

    def autotune(self, budget_ms: float = 0.0, cache_path: str | None = None):
        """Pick (and optionally cache) the fastest launch shape; returns it."""
        _check(_lib.esbgk_autotune(self._h, budget_ms, os.fsencode(cache_path) if cache_path else None))
        return self.get_tile()


class DomainDesc(ctypes.Structure):
    _fields_ = [("N_f", ctypes.c_int), ("Pr", ctypes.c_double), ("tau", ctypes.c_double),
                ("kappa", ctypes.c_double), ("dims", ctypes.c_int64 * 3)]


_sig("esbgk_batch_create", [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(DomainDesc), ctypes.c_int,
                            ctypes.POINTER(_vp)])
_sig("esbgk_batch_set_stream", [_vp, _vp])
_sig("esbgk_batch_init_fields", [_vp, ctypes.c_int, _dp, _dp, _dp])
_sig("esbgk_batch_set_tile", [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double])
_sig("esbgk_batch_step", [_vp, ctypes.c_int64, ctypes.c_int])
_sig("esbgk_batch_step_timed", [_vp, ctypes.c_int64, ctypes.c_int, _dp])
_sig("esbgk_batch_sync", [_vp])
_sig("esbgk_batch_status", [_vp, _ip])
_sig("esbgk_batch_info", [_vp, _i64p, _dp])
_sig("esbgk_batch_read_moments", [_vp, ctypes.c_int, _dp, _dp, _dp, _dp])
_sig("esbgk_batch_totals", [_vp, ctypes.c_int, _dp])
_sig("esbgk_batch_read_populations", [_vp, ctypes.c_int, _dp, _dp])
_sig("esbgk_batch_autotune", [_vp, ctypes.c_double, ctypes.c_char_p])
_sig("esbgk_batch_get_tile", [_vp, _ip, _ip])
_sig("esbgk_batch_destroy", [_vp], None)

PERSISTENT, PER_STEP, PER_DOMAIN = 0, 1, 2


class Batch:
    """Independent periodic domains of one lattice and storage mode, stepped
    together.  `domains` is a list of dicts with keys dims, Nf, Pr, tau and
    optionally kappa; streaming "aa" (in place) or "pull" (two copies)."""

    def __init__(self, D: int, Q: int, domains, storage: str = "f32", streaming: str = "aa", plane_pad: int = 0):
        self.D, self.Q, self.storage, self.streaming = D, Q, storage, streaming
        self.domains = [dict(d) for d in domains]
        arr = (DomainDesc * len(domains))()
        for i, d in enumerate(domains):
            dims = list(d["dims"]) + [1] * (3 - len(d["dims"]))
            arr[i] = DomainDesc(int(d["Nf"]), float(d["Pr"]), float(d["tau"]), float(d.get("kappa", 0.2)),
                                (ctypes.c_int64 * 3)(*dims))
        h = _vp()
        self._h = None
        _check(_lib.esbgk_batch_create(D, Q, len(domains), arr, _storage_code(storage, streaming, plane_pad),
                                       ctypes.byref(h)))
        self._h = h

    def __del__(self, _destroy=_lib.esbgk_batch_destroy):
        h = getattr(self, "_h", None)
        if h:
            _destroy(h)
            self._h = None

    def _shape(self, k):
        return tuple(reversed(self.domains[k]["dims"]))

    def _ncell(self, k):
        return int(np.prod(self.domains[k]["dims"]))

    def init_fields(self, k, rho, u, T):
        n = self._ncell(k)
        _check(_lib.esbgk_batch_init_fields(self._h, k, _p(_f64(rho, n)), _p(_f64(u, self.D * n)), _p(_f64(T, n))))

    def set_tile(self, block=0, policy=0, window=0, group_bytes=0.0):
        _check(_lib.esbgk_batch_set_tile(self._h, block, policy, window, group_bytes))

    def autotune(self, budget_ms: float = 0.0, cache_path: str | None = None):
        """Pick (and optionally cache) the fastest work-group size and cache
        policy of the persistent launch; returns (block, policy)."""
        _check(_lib.esbgk_batch_autotune(self._h, budget_ms, os.fsencode(cache_path) if cache_path else None))
        return self.get_tile()

    def get_tile(self):
        blk, pol = ctypes.c_int(), ctypes.c_int()
        _check(_lib.esbgk_batch_get_tile(self._h, ctypes.byref(blk), ctypes.byref(pol)))
        return blk.value, pol.value

    def step(self, n=1, mode=PERSISTENT):
        _check(_lib.esbgk_batch_step(self._h, int(n), int(mode)))

    def step_timed(self, n, mode=PERSISTENT) -> float:
        ms = ctypes.c_double()
        _check(_lib.esbgk_batch_step_timed(self._h, int(n), int(mode), ctypes.byref(ms)))
        return ms.value

    def sync(self):
        _check(_lib.esbgk_batch_sync(self._h))

    def status(self) -> int:
        s = ctypes.c_int()
        _check(_lib.esbgk_batch_status(self._h, ctypes.byref(s)))
        return s.value

    def info(self):
        c, b = ctypes.c_int64(), ctypes.c_double()
        _check(_lib.esbgk_batch_info(self._h, ctypes.byref(c), ctypes.byref(b)))
        return c.value, b.value

    def read_moments(self, k, with_P=False):
        n, sh = self._ncell(k), self._shape(k)
        rho, u, T = np.zeros(n), np.zeros(self.D * n), np.zeros(n)
        npc = self.D * (self.D + 1) // 2
        P = np.zeros(npc * n) if with_P else None
        _check(_lib.esbgk_batch_read_moments(self._h, k, _p(rho), _p(u), _p(T), _p(P)))
        out = dict(rho=rho.reshape(sh), u=u.reshape((self.D,) + sh), T=T.reshape(sh))
        if with_P:
            out["P"] = P.reshape((npc,) + sh)
        return out

    def totals(self, k):
        out = np.zeros(2 + self.D)
        _check(_lib.esbgk_batch_totals(self._h, k, _p(out)))
        return out

    def read_populations(self, k):
        n, sh = self._ncell(k), self._shape(k)
        f = np.zeros(self.Q * n)
        g = np.zeros(self.Q * n) if self.domains[k]["Nf"] > 0 else None
        _check(_lib.esbgk_batch_read_populations(self._h, k, _p(f), _p(g)))
        return f.reshape((self.Q,) + sh), (g.reshape((self.Q,) + sh) if g is not None else None)
