"""GPU checks of plane padding (ESBGK_PLANE_PAD): a padded layout gives
bitwise the populations, moments and totals of the unpadded one on every
lattice, storage mode and streaming scheme, with walls and open ends, in
batches, and across checkpoints (written unpadded, loaded into any
padding)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import workloads  # noqa: E402

pytestmark = pytest.mark.gpu

esb = pytest.importorskip("paper_1611_02409_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

CASES = [
    (2, 37, 3, (128, 40), "f32", "pull"),
    (2, 37, 3, (70, 33), "bf16", "aa"),
    (2, 37, 0, (64, 20), "f16", "pull"),
    (3, 39, 2, (16, 12, 10), "f32", "aa"),
    (3, 39, 0, (12, 9, 8), "bf16", "pull"),
    (2, 33, 1, (40, 24), "f32", "aa"),
]


def lattice(D, Q, Nf, dims, storage, streaming, pad, seed=11):
    lat = esb.Lattice(D, Q, Nf, 0.71, 0.7, dims, storage=storage, streaming=streaming, plane_pad=pad)
    lat.init_fields(*workloads.random_state(dims, seed=seed))
    return lat


def assert_same(a, b):
    fa, ga = a.read_populations()
    fb, gb = b.read_populations()
    assert np.array_equal(fa, fb)
    if ga is not None:
        assert np.array_equal(ga, gb)
    ma, mb = a.read_moments(with_P=True), b.read_moments(with_P=True)
    for k in ma:
        assert np.array_equal(ma[k], mb[k]), k


@pytest.mark.parametrize("D,Q,Nf,dims,storage,streaming", CASES)
def test_padded_layout_is_bitwise_the_unpadded_one(D, Q, Nf, dims, storage, streaming):
    ref = lattice(D, Q, Nf, dims, storage, streaming, 0)
    for pad in (4096, 16384):
        lat = lattice(D, Q, Nf, dims, storage, streaming, pad)
        assert lat.storage_tensor.numel() > ref.storage_tensor.numel()
        for n in (1, 4):
            lat.step(n)
        ref_n = lattice(D, Q, Nf, dims, storage, streaming, 0)
        ref_n.step(5)
        assert_same(lat, ref_n)
        assert np.array_equal(lat.totals(), ref_n.totals())


def test_walls_and_open_ends_with_padding():
    dims = (64, 30)
    for setup in ("walls", "open"):
        runs = []
        for pad in (0, 8192):
            lat = esb.Lattice(2, 37, 3, 0.71, 0.8, dims, streaming="pull", plane_pad=pad)
            lat.init_fields(*workloads.random_state(dims, seed=3))
            if setup == "walls":
                lat.set_walls((0.0, 0.0, 1.0), (0.05, 0.0, 1.02))
            else:
                lat.set_open_x(True)
            lat.step(7)
            runs.append(lat)
        assert_same(*runs)


def test_checkpoint_moves_between_paddings(tmp_path):
    dims, path = (96, 40), str(tmp_path / "ck.bin")
    src = lattice(2, 37, 3, dims, "f32", "pull", 12288)
    src.step(3)
    src.save(path)
    src.step(4)
    for pad in (0, 4096):
        dst = esb.Lattice(2, 37, 3, 0.71, 0.7, dims, streaming="pull", plane_pad=pad)
        dst.load(path)
        assert dst.steps == 3
        dst.step(4)
        assert_same(src, dst)


@pytest.mark.parametrize("streaming", ["aa", "pull"])
def test_padded_batch(streaming):
    doms = [dict(dims=(64, 48), Nf=3, Pr=0.71, tau=0.6), dict(dims=(33, 35), Nf=0, Pr=1.5, tau=0.9),
            dict(dims=(40, 36), Nf=1, Pr=0.8, tau=0.7)]
    res = []
    for pad in (0, 8192):
        b = esb.Batch(2, 37, doms, streaming=streaming, plane_pad=pad)
        for k, d in enumerate(doms):
            b.init_fields(k, *workloads.random_state(d["dims"], seed=50 + k))
        b.step(5)
        assert b.status() == 0
        res.append([b.read_populations(k) for k in range(len(doms))])
    for (fa, ga), (fb, gb) in zip(*res):
        assert np.array_equal(fa, fb)
        if ga is not None:
            assert np.array_equal(ga, gb)


def test_benchmark_size_paddings_match_unpadded():
    """The 4096^2 FP32 two-copy workload at the plane paddings the benchmark
    chooses from: moments after three steps bitwise equal the unpadded
    run's, and sampled cells' populations too."""
    n = 4096
    fields = workloads.waves_noise_2d(n)
    ref = esb.Lattice(2, 37, 3, 0.71, 0.6, (n, n), streaming="pull")
    ref.init_fields(*fields)
    ref.step(3)
    mref = ref.read_moments()
    cells = np.random.default_rng(7).integers(0, n * n, 4096)
    cref = ref.read_cells(cells)
    del ref
    torch.cuda.empty_cache()
    for pad in (16384, 24576, 49152):
        lat = esb.Lattice(2, 37, 3, 0.71, 0.6, (n, n), streaming="pull", plane_pad=pad)
        lat.init_fields(*fields)
        lat.step(3)
        m = lat.read_moments()
        for k in mref:
            assert np.array_equal(m[k], mref[k]), (pad, k)
        c = lat.read_cells(cells)
        for a, b in zip(c, cref):
            assert np.array_equal(a, b), pad
        del lat
        torch.cuda.empty_cache()


@pytest.mark.parametrize("streaming", ["aa", "pull"])
def test_autotune_chooses_padding_for_library_owned_storage(tmp_path, streaming):
    """With library-owned storage the autotuner also times plane paddings on
    allocations of their own and keeps the fastest; the state survives
    bitwise, later steps equal an untuned caller-owned run, and a second
    handle takes the padding from the cache."""
    dims, cache = (256, 96), str(tmp_path / "tune.txt")
    fields = workloads.random_state(dims, seed=21)
    ref = esb.Lattice(2, 37, 3, 0.71, 0.7, dims, streaming=streaming)
    ref.init_fields(*fields)
    own = esb.Lattice(2, 37, 3, 0.71, 0.7, dims, streaming=streaming, owned=True)
    assert own.storage_tensor is None and own.plane_pad_bytes == 0
    own.init_fields(*fields)
    ref.step(3)
    own.step(3)
    own.autotune(cache_path=cache)
    pad = own.plane_pad_bytes
    assert pad in (0, 16384, 24576, 49152)
    assert own.steps == 3
    assert_same(ref, own)
    ref.step(4)
    own.step(4)
    assert_same(ref, own)
    with open(cache) as fh:
        assert any(line.endswith(f"plane_pad {pad}") for line in fh.read().splitlines())
    second = esb.Lattice(2, 37, 3, 0.71, 0.7, dims, streaming=streaming, owned=True)
    second.init_fields(*fields)
    second.autotune(cache_path=cache)
    assert second.plane_pad_bytes == pad
    second.step(7)
    assert_same(ref, second)
    # caller-owned storage keeps its layout
    ref.autotune()
    assert ref.plane_pad_bytes == 0
