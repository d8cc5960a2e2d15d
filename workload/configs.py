"""Workload descriptions for the drifting-plasma runs.

Units: c = eps0 = m_e = e = 1; lengths in c / omega_p, times in 1 / omega_p
(omega_p of the density n = 1 on the simulation grid).  Electrons: q = -1,
m = 1, weight w = n dV / ppc.  The plasma drifts along -z with Lorentz
factor gamma; the co-moving frame velocity v_gal equals the drift velocity
(the Galilean choice) or zero (standard PSATD).

Named workloads:

* ``c1_cic_fp64``   16x16x64, 8 electrons/cell, gamma 10 cold, CIC, FP64,
                    50 steps (correctness run; also run with v_gal = 0).
* ``c2_cubic_mixed`` 128x128x256, 8 electrons/cell, gamma 30 with a
                    Gaussian thermal spread u_th = 1e-3 per component,
                    cubic shape, mixed precision, 500 steps.
* ``c3_boosted_laser`` 256x256x512, 4 electrons/cell, gamma_boost 20 plus a
                    Gaussian laser pulse (a0 2, waist 16 cells, wavelength 20
                    cells, 1/e half-length 30 cells) moving +z, cubic, mixed,
                    1000 steps.
* ``c5_batched``    64 independent runs, grids drawn from {32,64}^2 x
                    {64,128,256}, gamma ~ U[5, 50], density scale ~
                    U[0.5, 2], 4 electrons/cell, u_th = 1e-3, cubic, mixed,
                    200 steps.
* reduced ("lite") variants of c2 and c3 used by tests.
"""

from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class RunConfig:
    name: str
    shape: tuple            # (nx, ny, nz) nodes, z contiguous
    spacing: tuple = (1.0, 1.0, 1.0)
    dt: float = 1.0         # = dz / c for every named workload
    ppc: int = 8
    gamma: float = 10.0     # drift Lorentz factor, drift along -z
    u_th: float = 0.0       # Gaussian spread of each u component
    density: float = 1.0
    order: int = 1          # 1 = CIC, 3 = cubic
    precision: str = "fp64"  # "fp64" or "mixed"
    steps: int = 50
    galilean: bool = True   # v_gal = drift velocity if True else 0
    laser: dict = field(default=None)
    seed: int = 1000
    stencil: tuple = (0, 0, 0)  # field-solve stencil order per axis (0: spectral)

    @property
    def n_cells(self):
        return self.shape[0] * self.shape[1] * self.shape[2]

    @property
    def n_particles(self):
        return self.n_cells * self.ppc

    @property
    def n_modes(self):
        return self.shape[0] * self.shape[1] * (self.shape[2] // 2 + 1)

    @property
    def q(self):
        return -1.0

    @property
    def m(self):
        return 1.0

    @property
    def w(self):
        dv = self.spacing[0] * self.spacing[1] * self.spacing[2]
        return self.density * dv / self.ppc

    def drift_u(self):
        """u_z of the cold drift, rounded to float32 (stored that way)."""
        return float(np.float32(-np.sqrt(self.gamma * self.gamma - 1.0)))

    def v_gal(self):
        """(0, 0, v_z) with v_z = u_z / sqrt(1 + u_z^2) of the stored drift."""
        if not self.galilean:
            return (0.0, 0.0, 0.0)
        uz = self.drift_u()
        return (0.0, 0.0, uz / np.sqrt(1.0 + uz * uz))

    def with_(self, **kw):
        return replace(self, **kw)


LASER_C3 = {"a0": 2.0, "waist": 16.0, "wavelength": 20.0, "length": 30.0}

CONFIGS = {
    "c1_cic_fp64": RunConfig("c1_cic_fp64", (16, 16, 64), ppc=8, gamma=10.0,
                             order=1, precision="fp64", steps=50, seed=1000),
    "c2_cubic_mixed": RunConfig("c2_cubic_mixed", (128, 128, 256), ppc=8, gamma=30.0,
                                u_th=1e-3, order=3, precision="mixed", steps=500, seed=1001),
    "c3_boosted_laser": RunConfig("c3_boosted_laser", (256, 256, 512), ppc=4, gamma=20.0,
                                  order=3, precision="mixed", steps=1000,
                                  laser=LASER_C3, seed=1002),
    # reduced variants for tests (same physics, smaller grids)
    "c2_lite": RunConfig("c2_lite", (16, 16, 32), ppc=8, gamma=30.0, u_th=1e-3,
                         order=3, precision="mixed", steps=20, seed=1101),
    "c3_lite": RunConfig("c3_lite", (32, 32, 64), ppc=4, gamma=20.0, order=3,
                         precision="mixed", steps=20,
                         laser={"a0": 2.0, "waist": 6.0, "wavelength": 10.0, "length": 8.0},
                         seed=1102),
}


def get_config(name):
    return CONFIGS[name]


def batched_runs(n_runs=64, seed=1004, precision="mixed", order=3, ppc=4, steps=200):
    """The batched workload: independent runs of uneven sizes and boosts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    runs = []
    for r in range(n_runs):
        nx = int(rng.choice([32, 64]))
        ny = int(rng.choice([32, 64]))
        nz = int(rng.choice([64, 128, 256]))
        gamma = float(rng.uniform(5.0, 50.0))
        scale = float(rng.uniform(0.5, 2.0))
        runs.append(RunConfig(f"c5_run{r:02d}", (nx, ny, nz), ppc=ppc, gamma=gamma,
                              u_th=1e-3, density=scale, order=order, precision=precision,
                              steps=steps, seed=5000 + r))
    return runs
