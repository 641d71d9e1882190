"""Langevin (OVRVO) dynamics and its noise on the device, against the oracle.

* The device's normal deviates equal the oracle's Philox4x32-10 +
  Box-Muller deviates to within the last bits of the transcendental
  functions (the integers underneath are the same or the deviates would
  differ by O(1)).
* OVRVO steps of molten NaCl through maze_md_step match the oracle's OVRVO
  steps (its noise computed on the host and passed in) to the MD parity
  bar, and gamma = 0 leaves velocity Verlet bit for bit unchanged.
* The batched MD step draws the same noise as the step alone.
* A canonical run started cold reaches the target kinetic temperature.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import langevin  # noqa: E402
from paper_2505_20418_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_20418_amd import maze
    maze.lib()


@pytest.mark.parametrize("seed,step,half,n", [(0, 0, 0, 1), (7, 3, 1, 300), (2 ** 40 + 5, 2 ** 33 + 1, 0, 1000)])
def test_noise_matches_oracle(gpu, seed, step, half, n):
    from paper_2505_20418_amd import observables
    print(f"case: noise seed {seed} step {step} half {half} n {n}", flush=True)
    z = observables.langevin_noise(seed, step, half, n).cpu().numpy()
    ref = langevin.normals(seed, step, half, n)
    assert np.abs(z - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def _oracle_state(s, tol):
    o = oracle.Session(s.charges, s.pos, s.box, s.grid_spacing, tol=tol,
                       coulomb_k=inputs.COULOMB_K_EV_A)
    pos, vel = s.pos.copy(), s.vel.copy()
    F_es = o.step(pos)["forces"]
    F_sr, _ = oracle.bmh(pos, s.species, s.box, inputs.BMH_TABLE, inputs.BMH_CUTOFF)
    return o, pos, vel, F_es, F_sr


def test_ovrvo_matches_oracle(gpu):
    from paper_2505_20418_amd.md import MDRun
    s = inputs.molten_nacl(2, seed=1)
    T, gamma, seed = 1550.0, 0.05, 123
    run = MDRun(s, tol=1e-12, gamma=gamma, temperature=T, seed=seed)
    o, pos, vel, F_es, F_sr = _oracle_state(s, 1e-12)
    work = np.zeros(1)
    kT = inputs.KB_EV_PER_K * T
    print("case: OVRVO nacl64 32^3, 8 steps", flush=True)
    # the MD step's noise counter is the session's step count at entry; the
    # priming step advanced it to 1
    for k in range(8):
        run.step()
        out = langevin.ovrvo_step(o, pos, vel, s.masses, s.species, inputs.BMH_TABLE,
                                  inputs.BMH_CUTOFF, 1.0, inputs.ACCEL_FACTOR, F_es, F_sr, work,
                                  gamma, kT, seed, k + 1)
    assert np.abs(run.pos.cpu().numpy() - pos).max() <= 1e-9
    assert np.abs(run.vel.cpu().numpy() - vel).max() <= 1e-10
    obs = run.observables()
    assert abs(obs["ke"] - out["ke"]) <= 1e-9 * out["ke"]
    assert np.abs(obs["momentum"] - out["momentum"]).max() <= 1e-9
    assert abs(obs["work"] - work[0]) <= 1e-8 * max(1.0, abs(work[0]))
    run.close()


def test_gamma_zero_is_unchanged_velocity_verlet(gpu):
    from paper_2505_20418_amd.md import MDRun
    s = inputs.molten_nacl(2, seed=4)
    a = MDRun(s, tol=1e-10)
    b = MDRun(s, tol=1e-10, gamma=0.0, temperature=1550.0, seed=99)
    for _ in range(5):
        a.step()
        b.step()
    assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)
    assert torch.equal(a.scalars, b.scalars)
    a.close()
    b.close()


def test_batched_langevin_equals_alone(gpu):
    from paper_2505_20418_amd import md
    specs = [(2, 11), (3, 12)]
    alone = [md.MDRun(inputs.molten_nacl(n, seed=sd), tol=1e-10, gamma=0.02, temperature=1400.0,
                      seed=sd) for n, sd in specs]
    batch = [md.MDRun(inputs.molten_nacl(n, seed=sd), tol=1e-10, gamma=0.02, temperature=1400.0,
                      seed=sd) for n, sd in specs]
    for _ in range(4):
        for r in alone:
            r.step()
        md.step_many(batch)
    for a, b in zip(alone, batch):
        assert torch.equal(a.pos, b.pos) and torch.equal(a.vel, b.vel)
        a.close()
        b.close()


def test_nvt_reaches_target_temperature(gpu):
    from paper_2505_20418_amd.md import MDRun
    s = inputs.molten_nacl(3, seed=6)          # 216 ions
    s.vel *= np.sqrt(300.0 / 1200.0)
    T = 1550.0
    run = MDRun(s, tol=1e-8, precision=1, gamma=0.05, temperature=T, seed=5, dt=1.0)
    ke = []
    for k in range(600):
        run.step()
        if k >= 200:
            ke.append(run.observables()["ke"])
    t_kin = 2.0 * np.mean(ke) / (3 * s.n_ions * inputs.KB_EV_PER_K)
    print(f"kinetic temperature {t_kin:.1f} K (target {T} K)", flush=True)
    # one sample spreads by sqrt(2 / 3N) = 5.6%; about 20 independent samples
    assert abs(t_kin / T - 1.0) < 0.06
    run.close()
