"""CPU-side checks of the C ABI: the built library exports every function
include/esbgk.h declares, host-side validation rejects bad arguments
before touching a device, and the library's own lattice constants and
parameter mapping agree with the oracle's independent derivation."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esbgk.h")
LIB = os.path.join(ROOT, "paper_1611_02409_amd", "libesbgk.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(esbgk_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) > 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.fixture(scope="module")
def esb():
    import paper_1611_02409_amd as m
    return m


@pytest.mark.parametrize("D,Q", [(2, 37), (2, 33), (3, 39)])
def test_lattice_constants_agree_with_oracle(esb, D, Q):
    li = esb.lattice_info(D, Q)
    L = oracle.Lattice(D, Q)
    oc = [tuple(x) for x in L.c]
    perm = [oc.index(tuple(c)) for c in li["c"]]
    assert sorted(perm) == list(range(Q))
    assert abs(li["r"] - L.r) < 1e-15
    np.testing.assert_allclose(li["w"], L.w[perm], rtol=1e-14)
    # storage order: rest first, then +c/-c pairs
    assert not li["c"][0].any()
    for p in range((Q - 1) // 2):
        assert np.array_equal(li["c"][2 * p + 1], -li["c"][2 * p + 2])


@pytest.mark.parametrize("Nf,Pr,tau", [(3, 0.71, 0.6), (0, 2.0, 0.55), (1, 0.5, 1.2), (2, 0.71, 0.7)])
def test_parameter_mapping_agrees_with_oracle(esb, Nf, Pr, tau):
    a = esb.params(2, Nf, Pr, tau, 0.2)
    b = oracle.param_map(2, Nf, Pr, tau, 0.2)
    for k in ("omega", "omega_s", "nu", "gamma"):
        assert abs(a[k] - b[k]) < 1e-15


@pytest.mark.parametrize("args", [
    dict(D=2, Nf=3, Pr=0.71, tau=0.5),
    dict(D=2, Nf=3, Pr=0.0, tau=0.8),
    dict(D=2, Nf=-1, Pr=0.71, tau=0.8),
    dict(D=4, Nf=3, Pr=0.71, tau=0.8),
    dict(D=2, Nf=3, Pr=float("nan"), tau=0.8),
    dict(D=2, Nf=3, Pr=0.71, tau=0.8, kappa=1.0),
    dict(D=2, Nf=3, Pr=0.1, tau=1.0, kappa=0.0),       # nu = -4.5: Lambda could lose positive-definiteness
])
def test_invalid_parameters_rejected(esb, args):
    kappa = args.pop("kappa", 0.2)
    with pytest.raises(esb.EsbgkError) as e:
        esb.params(args["D"], args["Nf"], args["Pr"], args["tau"], kappa)
    assert e.value.code == -1


def test_create_rejects_bad_shapes_without_a_device(esb):
    lib = esb._lib
    h = ctypes.c_void_p()
    for D, Q, dims, storage, code in [(2, 35, (8, 8), 0, -2), (2, 37, (2, 8), 0, -1), (2, 37, (8, 8), 7, -1),
                                      (2, 37, (8, 8), 0x13, -1), (2, 37, (8, 8), 0x20, -1),
                                      (2, 37, (70000, 70000), 0, -2), (3, 39, (8, 8, 2), 0, -1)]:
        d = (ctypes.c_int64 * 3)(*(list(dims) + [1] * (3 - len(dims))))
        rc = lib.esbgk_create(D, Q, 3, 0.71, 0.8, d, storage, ctypes.byref(h))
        assert rc == code, (D, Q, dims, rc, lib.esbgk_last_error())
        assert lib.esbgk_last_error()


def test_storage_bytes(esb):
    n = esb.storage_bytes(2, 37, 3, (4096, 4096), "f32")
    assert n == 2 * 37 * 4096 * 4096 * 4
    assert esb.storage_bytes(2, 37, 0, (4096, 4096), "f16") == 37 * 4096 * 4096 * 2
    assert esb.storage_bytes(3, 39, 2, (256, 256, 256), "bf16") == 2 * 39 * 256 ** 3 * 2
    # two-copy pull keeps two whole copies (each set 256-byte aligned)
    assert esb.storage_bytes(2, 37, 3, (4096, 4096), "f32", "pull") == 2 * n
    assert esb.storage_bytes(2, 37, 1, (33, 35), "f32", "pull") == 2 * 2 * ((37 * 33 * 35 * 4 + 255) // 256 * 256)
    # FP16/BF16 with both populations: one set of (f_i, g_i) elements
    assert esb.storage_bytes(2, 37, 1, (33, 35), "f16", "pull") == 2 * ((37 * 33 * 35 * 4 + 255) // 256 * 256)
    assert esb.storage_bytes(2, 37, 0, (33, 35), "bf16", "pull") == 2 * ((37 * 33 * 35 * 2 + 255) // 256 * 256)
    with pytest.raises(ValueError):
        esb.storage_bytes(2, 37, 3, (64, 64), "f32", "push")
    # plane padding: unused bytes after every plane
    pad = 3 * 4096
    assert esb.storage_bytes(2, 37, 3, (4096, 4096), "f32", plane_pad=pad) == 2 * 37 * (4096 * 4096 * 4 + pad)
    assert esb.storage_bytes(2, 37, 1, (33, 35), "f16", "pull", plane_pad=pad) == \
        2 * ((37 * (33 * 35 * 4 + pad) + 255) // 256 * 256)
    for bad in (100, 256 * 4096, -4096):
        with pytest.raises(ValueError):
            esb.storage_bytes(2, 37, 3, (64, 64), "f32", plane_pad=bad)


def test_storage_codes_outside_the_defined_bits_are_rejected(esb):
    lib = esb._lib
    out = ctypes.c_size_t()
    dims = (ctypes.c_int64 * 3)(64, 64, 1)
    for code in (3, 4, 0x20, 0x10000, -1):
        assert lib.esbgk_storage_bytes(2, 37, 3, dims, code, ctypes.byref(out)) == -1, code
        assert "storage" in lib.esbgk_last_error().decode()
    assert lib.esbgk_storage_bytes(2, 37, 3, dims, esb.PULL | (255 << 8), ctypes.byref(out)) == 0
    assert out.value == 2 * 2 * 37 * (64 * 64 * 4 + 255 * 4096)


def test_batch_create_validates_before_touching_a_device(esb):
    """Unknown storage codes and invalid domains (in either streaming
    scheme) are refused before any device call."""
    lib = esb._lib
    desc = (esb.DomainDesc * 2)()
    for k in range(2):
        desc[k].N_f, desc[k].Pr, desc[k].tau, desc[k].kappa = 3, 0.71, 0.6, 0.2
        desc[k].dims[0], desc[k].dims[1], desc[k].dims[2] = 64, 64, 1
    desc[1].tau = 0.5
    h = ctypes.c_void_p()
    assert lib.esbgk_batch_create(2, 37, 2, desc, 3 | esb.PULL, ctypes.byref(h)) == -1
    assert "storage" in lib.esbgk_last_error().decode()
    for code in (esb.F32, esb.F32 | esb.PULL, esb.BF16_DEV | esb.PULL):
        assert lib.esbgk_batch_create(2, 37, 2, desc, code, ctypes.byref(h)) == -1
        assert lib.esbgk_last_error().decode().startswith("domain 1:")
        assert not h.value


def test_null_handles_are_rejected(esb):
    lib = esb._lib
    assert lib.esbgk_step(None, 1) == -1
    assert lib.esbgk_totals(None, None) == -1
    assert lib.esbgk_set_walls(None, None, None) == -1
    lib.esbgk_destroy(None)
    lib.esbgk_batch_destroy(None)


def test_stream_ceiling_rejects_bad_sizes_without_a_device(esb):
    lib = esb._lib
    out = ctypes.c_double()
    for cells, reps in ((100, 1), (1 << 30, 1), (1 << 20, 0)):
        assert lib.esbgk_stream_ceiling(cells, reps, ctypes.byref(out)) == -1
    assert lib.esbgk_stream_ceiling(1 << 20, 1, None) == -1
    for planes, sets in ((74, 1), (37, 2), (40, 2), (0, 1)):
        assert lib.esbgk_stream_ceiling_planes(1 << 20, planes, sets, 1, ctypes.byref(out)) == -1
        assert "planes" in lib.esbgk_last_error().decode()
    # a set over 4 GiB
    assert lib.esbgk_stream_ceiling_planes(30000000, 78, 2, 1, ctypes.byref(out)) == -1
