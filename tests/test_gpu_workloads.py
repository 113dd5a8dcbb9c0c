"""Workload-level GPU parity against the FP64 oracle.

* 3D: D3Q39 thermal Taylor-Green vortex at 32^3 (u0 = 0.02, T wave 1e-2,
  N_f = 2, Pr = 0.71, tau = 0.7): kinetic energy history and final fields.
* D2Q37 waves + noise (N_f = 3, Pr = 0.71, tau = 0.6) at 4096^2 (1000 steps)
  and 1024^2 (1000 and 5000 steps) against the stored oracle references
  (block means on a 512^2 / 256^2 grid), for FP32, FP16- and BF16-deviation
  storage: relative L2 of rho, u, T, and the drift of total mass and energy,
  against the bounds in BOUNDS.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import oracle  # noqa: E402
import workloads  # noqa: E402
from gpu_helpers import rel_l2  # noqa: E402

pytestmark = pytest.mark.gpu

esb = pytest.importorskip("paper_1611_02409_amd")
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kinetic_energy(m):
    return 0.5 * float(np.sum(m["rho"] * (m["u"] ** 2).sum(0)))


def test_taylor_green_32_kinetic_energy_history():
    n, steps, every = 32, 200, 40
    fields = workloads.taylor_green_3d(n)
    lat = esb.Lattice(3, 39, 2, 0.71, 0.7, (n, n, n))
    lat.init_fields(*fields)
    prev = oracle.set_threads(0)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        sim = oracle.Sim(3, 39, 2, 0.71, 0.7, (n, n, n))
        sim.init(*fields)
        k0 = kinetic_energy(sim.moments())
        for t in range(every, steps + 1, every):
            lat.step(every)
            sim.step(every)
            mg, mo = lat.read_moments(), sim.moments()
            kg, ko = kinetic_energy(mg), kinetic_energy(mo)
            print(f"TGV 32^3 step {t}: KE/KE0 gpu {kg / k0:.6e} oracle {ko / k0:.6e}")
            assert abs(kg - ko) / ko < 1e-5
        assert ko / k0 > 1e-3          # still well resolved
        for key in ("rho", "u", "T"):
            assert rel_l2(mg[key], mo[key]) < 1e-5
    finally:
        oracle.set_threads(prev)


def _reference(n=4096, Pr=0.71):
    path = os.path.join(GOLDEN, f"ref_waves{n}_pr{Pr:g}.npz")
    if not os.path.exists(path):
        pytest.skip(f"reference {os.path.basename(path)} not generated (tests/golden/make_references.py)")
    return np.load(path)


# relative L2 of (rho, u, T) and relative drift of total mass and energy,
# by (storage, steps).  FP32: the collision target and the temperatures are
# evaluated in FP64 and the error is the FP32 storage and relaxation rounding
# (measured <= 1.3e-7 in u, <= 2e-10 in rho and T, drifts <= 1e-10); the
# bounds keep the 1e-5 target with room.  FP16/BF16: twice the largest value
# measured over the 4096^2 and 1024^2 runs at that step count.
BOUNDS = {
    ("f32", 1000): (1e-9, 1e-6, 1e-9, 1e-10, 1e-9),
    ("f32", 5000): (1e-9, 1e-6, 1e-9, 1e-10, 1e-9),
    ("f16", 1000): (1e-6, 3e-4, 1e-6, 4e-8, 6e-9),
    ("f16", 5000): (6e-6, 2e-3, 5e-6, 3e-7, 5e-8),
    ("bf16", 1000): (3.5e-5, 2.5e-2, 2.5e-5, 7e-7, 5e-8),
    ("bf16", 5000): (5e-5, 8e-2, 7e-5, 2e-6, 2e-7),
}


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("n,steps", [(4096, 1000), (4096, 5000), (1024, 1000), (1024, 5000)])
def test_waves_against_fp64_reference(storage, n, steps):
    ref = _reference(n)
    if f"rho_{steps}" not in ref.files:
        pytest.skip(f"reference has no snapshot at step {steps}")
    fields = workloads.waves_noise_2d(n)
    lat = esb.Lattice(2, 37, 3, 0.71, float(ref["tau"]), (n, n), storage=storage)
    lat.init_fields(*fields)
    t0 = lat.totals()
    lat.step(steps)
    t1 = lat.totals()
    m = lat.read_moments()
    bm = lambda a: workloads.block_mean(a, int(ref["out_n"]))
    rho_r = 1.0 + ref[f"rho_{steps}"].astype(np.float64)
    T_r = 1.0 + ref[f"T_{steps}"].astype(np.float64)
    u_r = np.stack([ref[f"ux_{steps}"], ref[f"uy_{steps}"]]).astype(np.float64)
    e_rho = rel_l2(1.0 + bm(m["rho"] - 1.0), rho_r)
    e_T = rel_l2(1.0 + bm(m["T"] - 1.0), T_r)
    e_u = rel_l2(np.stack([bm(m["u"][0]), bm(m["u"][1])]), u_r)
    to = ref[f"totals_{steps}"]
    d_mass = abs(t1[0] - t0[0]) / t0[0]
    d_en = abs(t1[-1] - t0[-1]) / t0[-1]
    print(f"{storage} {n}^2 x {steps}: rho {e_rho:.2e} u {e_u:.2e} T {e_T:.2e} | mass drift {d_mass:.2e} "
          f"energy drift {d_en:.2e} | gpu-oracle totals {(t1 - to) / to[0]}")
    b = BOUNDS[(storage, steps)]
    assert e_rho < b[0] and e_u < b[1] and e_T < b[2], (storage, steps, e_rho, e_u, e_T, b)
    assert d_mass < b[3] and d_en < b[4], (storage, steps, d_mass, d_en, b[3:])


def test_d2q33_shock_tube_matches_oracle():
    """The paper's shock tube (D2Q33, 1000 x 16, density 4:1, gamma 1.4,
    tau 2/3, 174 steps) on the GPU against the oracle: a strongly nonlinear
    state (deviations up to 3 w_i)."""
    nx, ny, steps = 1000, 16, 174
    x = np.tile(np.arange(nx, dtype=float), (ny, 1))
    fields = (np.where(x < 500, 4.0, 1.0), np.zeros((2, ny, nx)), np.ones((ny, nx)))
    lat = esb.Lattice(2, 33, 3, 0.71, 2 / 3, (nx, ny))
    lat.init_fields(*fields)
    lat.step(steps)
    prev = oracle.set_threads(0)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        sim = oracle.Sim(2, 33, 3, 0.71, 2 / 3, (nx, ny))
        sim.init(*fields)
        sim.step(steps)
    finally:
        oracle.set_threads(prev)
    mg, mo = lat.read_moments(), sim.moments()
    er, eu, eT = rel_l2(mg["rho"], mo["rho"]), rel_l2(mg["u"], mo["u"]), rel_l2(mg["T"], mo["T"])
    print(f"shock tube D2Q33: rho {er:.2e} u {eu:.2e} T {eT:.2e}")
    assert er < 1e-5 and eu < 1e-5 and eT < 1e-5


@pytest.mark.parametrize("Nf,kappa", [(3, 0.25), (3, 0.9)])
def test_sound_attenuation_on_gpu(Nf, kappa):
    """The library's FP32 pressure wave decays at the linearised
    Navier-Stokes rate with the lattice shear, bulk (kappa) and thermal
    coefficients, and travels at sqrt(gamma)/r (the closed forms pinned on the
    oracle in test_oracle_sound)."""
    from test_oracle_sound import fit_attenuation, predicted_attenuation
    n, ny, tau, Pr, D = 256, 4, 0.8, 1.0, 2
    r = esb.lattice_info(2, 37)["r"]
    cs = np.sqrt((Nf + D + 2) / (Nf + D)) / r
    lat = esb.Lattice(2, 37, Nf, Pr, tau, (n, ny), kappa=kappa)
    x = np.tile(np.arange(n, dtype=float), (ny, 1))
    lat.init_fields(1 + 1e-4 * np.cos(2 * np.pi * x / n), np.zeros((2, ny, n)), np.ones((ny, n)))
    c = np.cos(2 * np.pi * x / n)
    amp = []
    for _ in range(int(6 * n / cs) + 1):
        m = lat.read_moments()
        amp.append(2 * np.mean((m["rho"] * m["T"] - 1) * c))
        lat.step(1)
    G, w = fit_attenuation(amp, 2 * np.pi / n, cs)
    Gp = predicted_attenuation(Nf, kappa, tau, Pr, n)
    print(f"sound N_f={Nf} kappa={kappa}: Gamma {G:.5e} predicted {Gp:.5e} (ratio {G / Gp:.4f}), "
          f"frequency ratio {w / (cs * 2 * np.pi / n):.5f}")
    assert abs(G / Gp - 1) < 0.015 and abs(w / (cs * 2 * np.pi / n) - 1) < 0.003


def test_reduced_storage_4096_5000_steps():
    """The reduced-precision workload at its full size and length (4096^2,
    5000 steps, block means on 512^2).  No FP64 reference exists at this
    size (the oracle would need ~10 host-hours); the FP32-storage run serves
    as the reference instead -- it stays within 1.3e-7 (u) and 2e-10 (rho, T)
    of the FP64 oracle at 1024^2 x 5000 and 4096^2 x 1000 (BOUNDS above),
    far below the FP16/BF16 errors measured here.  Drifts are of the FP64
    GPU totals of each run."""
    n, steps, out_n = 4096, 5000, 512
    fields = workloads.waves_noise_2d(n)
    res = {}
    for storage in ("f32", "f16", "bf16"):
        lat = esb.Lattice(2, 37, 3, 0.71, 0.6, (n, n), storage=storage, streaming="pull")
        lat.init_fields(*fields)
        t0 = lat.totals()
        lat.step(steps)
        t1 = lat.totals()
        m = lat.read_moments()
        bm = lambda a: workloads.block_mean(a, out_n)
        res[storage] = (bm(m["rho"] - 1.0), np.stack([bm(m["u"][0]), bm(m["u"][1])]), bm(m["T"] - 1.0),
                        abs(t1[0] - t0[0]) / t0[0], abs(t1[-1] - t0[-1]) / t0[-1])
        del lat
        torch.cuda.empty_cache()
    r_rho, r_u, r_T = res["f32"][:3]
    # (rho, u, T, mass drift, energy drift): twice the measured values
    # (FP16 3.3e-6, 2.9e-3, 3.5e-6, 2.7e-8, 1.3e-8; BF16 8.1e-5, 9.8e-2,
    # 5.5e-5, 3.4e-7, 2.7e-7)
    bounds = {"f16": (7e-6, 6e-3, 7e-6, 6e-8, 3e-8), "bf16": (1.6e-4, 2e-1, 1.1e-4, 7e-7, 6e-7)}
    for storage in ("f16", "bf16"):
        d_rho, d_u, d_T, dm, de = res[storage]
        e_rho = rel_l2(1.0 + d_rho, 1.0 + r_rho)
        e_T = rel_l2(1.0 + d_T, 1.0 + r_T)
        e_u = rel_l2(d_u, r_u)
        print(f"{storage} 4096^2 x 5000 vs FP32: rho {e_rho:.2e} u {e_u:.2e} T {e_T:.2e} | "
              f"mass drift {dm:.2e} energy drift {de:.2e} (FP32: {res['f32'][3]:.2e} {res['f32'][4]:.2e})")
        b = bounds[storage]
        assert e_rho < b[0] and e_u < b[1] and e_T < b[2], (storage, e_rho, e_u, e_T)
        assert dm < b[3] and de < b[4], (storage, dm, de)
