"""Diffusely reflecting walls (thermal Couette flow, Sec. VI.A) on the GPU
against the oracle's walls.

* Parity: random states between a resting and a moving, warmer wall, in
  D2Q37, D2Q33 and D3Q39, FP32 and FP16/BF16-deviation storage: gas rows
  after a few hundred steps.
* Couette: the impulsive start between walls at rest and at u0 (D2Q37,
  N_f = 3, tau = 1) against the oracle at 2000 and 40000 steps (steady), the
  steady profile linear with symmetric slip, and mass conserved.
* The call's error paths.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
import workloads  # noqa: E402
from gpu_helpers import pert_l2, rel_l2  # noqa: E402

pytestmark = pytest.mark.gpu

esb = pytest.importorskip("paper_1611_02409_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def wall_reach(D, Q):
    c = np.array(oracle.Lattice(D, Q).c)
    return int(np.max(c[:, 1]))


def run_pair(D, Q, Nf, dims, bottom, top, steps, storage="f32", tau=0.8, Pr=0.71, seed=5):
    fields = workloads.random_state(dims, seed, amp_rho=0.02, amp_u=0.02, amp_T=0.02)
    lat = esb.Lattice(D, Q, Nf, Pr, tau, dims, storage=storage, streaming="pull")
    lat.init_fields(*fields)
    lat.set_walls(bottom, top)
    prev = oracle.set_threads(0)
    oracle.set_threads(min(8, os.cpu_count() or 1))
    try:
        sim = oracle.Sim(D, Q, Nf, Pr, tau, dims)
        sim.init(*fields)
        sim.set_walls(bottom, top)
        lat.step(steps)
        sim.step(steps)
        return lat.read_moments(), sim.moments()
    finally:
        oracle.set_threads(prev)


def gas(a, R, ny, D):
    """gas rows of a (..., [z,] y, x) field"""
    return a[..., R:ny - R, :] if D == 2 else a[..., :, R:ny - R, :]


# (D, Q, N_f, dims, bottom, top, steps)
WALL_CASES = [
    (2, 37, 3, (8, 40), (0.0, 0.0, 1.0), (0.08, 0.0, 1.03), 300),
    (2, 37, 3, (64, 20), (0.03, 0.0, 1.01), (0.06, 0.0, 0.99), 200),    # whole-wave rows
    (2, 37, 0, (6, 30), (0.0, 0.0, 1.0), (0.05, 0.0, 1.0), 300),
    (2, 33, 3, (8, 40), (0.02, 0.0, 0.98), (-0.05, 0.0, 1.02), 300),
    (3, 39, 2, (4, 16, 4), (0.0, 0.0, 0.0, 1.0), (0.05, 0.0, 0.03, 1.02), 150),
]

# relative L2 bounds on the gas rows, (rho and T perturbations, u), by
# (N_f, storage).  FP32: the 1e-5 target (measured <= 3.4e-6; the N_f = 0
# case has the smallest perturbations left after 300 steps, hence the
# largest relative error).  FP16/BF16: about three times the measured value.
WALL_BOUNDS = {
    (3, "f32"): (1e-5, 1e-5), (0, "f32"): (1e-5, 1e-5), (2, "f32"): (1e-5, 1e-5),
    (3, "f16"): (3e-3, 1e-3), (0, "f16"): (4e-2, 5e-4),
    (3, "bf16"): (7e-2, 3e-2), (0, "bf16"): (0.4, 3e-2),
}


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("case", WALL_CASES, ids=lambda c: f"D{c[0]}Q{c[1]}_Nf{c[2]}_{'x'.join(map(str, c[3]))}")
def test_walls_match_oracle(case, storage):
    D, Q, Nf, dims, bottom, top, steps = case
    if storage != "f32" and dims not in ((8, 40), (6, 30)):
        pytest.skip("reduced storage covered on the two small D2Q37 cases")
    mg, mo = run_pair(D, Q, Nf, dims, bottom, top, steps, storage=storage)
    R, ny = wall_reach(D, Q), dims[1]
    e_rho = pert_l2(gas(mg["rho"], R, ny, D), gas(mo["rho"], R, ny, D))
    e_T = pert_l2(gas(mg["T"], R, ny, D), gas(mo["T"], R, ny, D))
    e_u = rel_l2(gas(mg["u"], R, ny, D), gas(mo["u"], R, ny, D))
    print(f"walls D{D}Q{Q} N_f={Nf} {dims} {storage} x {steps}: rho {e_rho:.2e} u {e_u:.2e} T {e_T:.2e}")
    b = WALL_BOUNDS[(Nf, storage)]
    assert e_rho < b[0] and e_T < b[0] and e_u < b[1], (e_rho, e_u, e_T)


def test_couette_start_and_steady_state_match_oracle():
    u0, tau, Nf, Pr = 0.1, 1.0, 3, 0.71
    R, L, nx = 3, 64, 4
    ny = L + 2 * R
    dims = (nx, ny)
    rest = (np.ones((ny, nx)), np.zeros((2, ny, nx)), np.ones((ny, nx)))
    lat = esb.Lattice(2, 37, Nf, Pr, tau, dims, streaming="pull")
    lat.init_fields(*rest)
    lat.set_walls((0.0, 0.0, 1.0), (u0, 0.0, 1.0))
    prev = oracle.set_threads(0)
    oracle.set_threads(min(8, os.cpu_count() or 1))
    try:
        sim = oracle.Sim(2, 37, Nf, Pr, tau, dims)
        sim.init(*rest)
        sim.set_walls((0.0, 0.0, 1.0), (u0, 0.0, 1.0))
        mass0 = float(np.sum(lat.read_moments()["rho"][R:ny - R]))
        for t in (2000, 40000):
            lat.step(t - lat.steps)
            sim.step(t - sim.steps)
            mg, mo = lat.read_moments(), sim.moments()
            ug, uo = mg["u"][0].mean(1)[R:ny - R], mo["u"][0].mean(1)[R:ny - R]
            Tg, To = mg["T"].mean(1)[R:ny - R], mo["T"].mean(1)[R:ny - R]
            mass = float(np.sum(mg["rho"][R:ny - R]))
            e_u = rel_l2(ug, uo)
            e_T = float(np.max(np.abs(Tg - To)) / max(np.max(np.abs(To - 1)), 1e-12))
            print(f"Couette step {t}: u {e_u:.2e} T(heating) {e_T:.2e} mass drift {abs(mass - mass0) / mass0:.2e}")
            # transient: the 1e-5 target (measured 2.3e-7).  Steady state: a
            # time-independent state repeats the same FP32 rounding every
            # step, which then acts as a fixed forcing: a sag of the profile
            # of the same relative size for any u0 (measured 1.9e-5 to 2.3e-5
            # at 40000 steps, 2.9e-5 at 20000; with 32 gas rows 1e-5, of which
            # an FP64 run that rounds the stored deviations to FP32 after each
            # step shows a quarter, the rest is the FP32 collision arithmetic)
            assert e_u < (1e-5 if t <= 2000 else 6e-5), (t, e_u)
            assert abs(mass - mass0) / mass0 < 1e-7          # measured 9e-9 at 40000 steps
        assert e_T < 1e-3                                   # of the heating (4e-4 of T); measured 1e-4
    finally:
        oracle.set_threads(prev)
    # linear beyond the walls' kinetic layer (a few rows, 2e-4 of u0 at the
    # second row), with the same slip at both walls
    rows = np.arange(L) + 0.5
    core = slice(2 * R, L - 2 * R)
    b, a = np.polyfit(rows[core], ug[core] / u0, 1)
    assert np.max(np.abs(ug[core] / u0 - (a + b * rows[core]))) < 5e-5
    assert abs(a - (1 - (a + b * L))) < 1e-4


def test_wall_errors():
    dims = (8, 40)
    aa = esb.Lattice(2, 37, 3, 0.71, 0.8, dims)
    with pytest.raises(RuntimeError, match="ESBGK_PULL"):
        aa.set_walls((0.0, 0.0, 1.0), (0.1, 0.0, 1.0))
    short = esb.Lattice(2, 37, 3, 0.71, 0.8, (8, 6), streaming="pull")
    with pytest.raises(RuntimeError, match="ny >= 7"):
        short.set_walls((0.0, 0.0, 1.0), (0.1, 0.0, 1.0))
    lat = esb.Lattice(2, 37, 3, 0.71, 0.8, dims, streaming="pull")
    lat.init_fields(*workloads.random_state(dims, 3))
    with pytest.raises(RuntimeError, match="temperature"):
        lat.set_walls((0.0, 0.0, 0.0), (0.1, 0.0, 1.0))
    lat.set_walls((0.0, 0.0, 1.0), (0.1, 0.0, 1.0))
    with pytest.raises(RuntimeError, match="ghost cells"):
        lat.totals()
    lat.step(3)
    lat.set_walls(None, None)
    t = lat.totals()
    assert np.all(np.isfinite(t))


def test_walls_checkpoint_resume_is_bitwise(tmp_path):
    dims = (64, 24)
    fields = workloads.random_state(dims, 9, amp_rho=0.02, amp_u=0.02, amp_T=0.02)
    walls = ((0.0, 0.0, 1.0), (0.1, 0.0, 1.02))
    a = esb.Lattice(2, 37, 3, 0.71, 0.8, dims, streaming="pull")
    a.init_fields(*fields)
    a.set_walls(*walls)
    a.step(41)
    path = str(tmp_path / "walls.ckpt")
    a.save(path)
    a.step(30)
    b = esb.Lattice(2, 37, 3, 0.71, 0.8, dims, streaming="pull")
    b.load(path)
    b.set_walls(*walls)
    b.step(30)
    fa, ga = a.read_populations()
    fb, gb = b.read_populations()
    R = 3
    assert np.array_equal(fa[:, R:-R], fb[:, R:-R]) and np.array_equal(ga[:, R:-R], gb[:, R:-R])
