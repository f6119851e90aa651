"""Named synthetic workloads.

The paper measures on a heterogeneous extruded mesh that is not available;
these seeded boxes stand in for it with the same element types (hexahedral
Q_p, Gauss rule with p+1 points per direction), material law and DoF counts of
the same order as its 3D benchmark meshes.

Displacement amplitudes: each workload names a nominal amplitude of its
random sine modes.  Taken literally, several of them invert cells (det F <= 0
at some quadrature points), which makes the tangent meaningless.  The rule is
to halve the nominal amplitude until the smallest det F over all quadrature
points is at least 0.1; ``amplitude`` holds the result of that rule (it is
checked by the test-suite, which recomputes det F with the oracle).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import generators as g


@dataclass(frozen=True)
class Workload:
    name: str
    cfg_id: int
    nx: int
    ny: int
    nz: int
    degree: int
    lengths: tuple = (1.0, 1.0, 1.0)
    jitter: float = 0.0          # fraction of the element size, interior vertices only
    mu: float = 1.0
    lam: float = 10.0
    amplitude: float = 0.05      # displacement amplitude of the sine modes (after the J guard)
    nominal_amplitude: float = 0.05  # amplitude named by the workload before the J guard
    n_w: int = 1                 # number of random test vectors
    description: str = ""

    @property
    def counts(self) -> dict:
        return g.box_counts(self.nx, self.ny, self.nz, self.degree)

    @property
    def n_dofs(self) -> int:
        return self.counts["n_dofs"]

    @property
    def n_elems(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_qpoints(self) -> int:
        return self.n_elems * (self.degree + 1) ** 3

    def vertices(self) -> np.ndarray:
        rng = g.rng_for(self.cfg_id, 0) if self.jitter > 0 else None
        return g.box_vertices(self.nx, self.ny, self.nz, self.lengths, self.jitter, rng)

    def displacement(self) -> np.ndarray:
        return g.sine_displacement(self.nx, self.ny, self.nz, self.degree, self.amplitude,
                                   g.rng_for(self.cfg_id, 1))

    def test_vector(self, k: int) -> np.ndarray:
        return g.random_vectors(self.n_dofs, 1, g.rng_for(self.cfg_id, 2 + k))[0]

    def test_vectors(self) -> np.ndarray:
        return np.stack([self.test_vector(k) for k in range(self.n_w)])


CONFIGS = {
    # 4^3 unit cube, Q2, 2187 DoF: every oracle pin and element-wise GPU parity.
    "cube4_q2": Workload("cube4_q2", 0, 4, 4, 4, 2, jitter=0.0, amplitude=0.05,
                         nominal_amplitude=0.05, n_w=8,
                         description="4x4x4 unit cube, Q2, 3^3 Gauss, 2187 DoF"),
    # same cube with jittered interior vertices (non-affine elements)
    "cube4_q2_jit": Workload("cube4_q2_jit", 10, 4, 4, 4, 2, jitter=0.1, amplitude=0.025,
                             nominal_amplitude=0.05, n_w=8,
                             description="4x4x4 jittered unit cube, Q2, 2187 DoF"),
    # 48^3 box, Q2, 2,738,019 DoF: the headline apply workload.
    "box48_q2": Workload("box48_q2", 1, 48, 48, 48, 2, jitter=0.1, amplitude=0.05,
                         nominal_amplitude=0.1, n_w=1,
                         description="48^3 jittered unit box, Q2, 3^3 Gauss, 2,738,019 DoF"),
    # higher degrees at the same (Q4) or smaller (Q6) DoF count.
    "box24_q4": Workload("box24_q4", 2, 24, 24, 24, 4, jitter=0.1, amplitude=0.025,
                         nominal_amplitude=0.1, n_w=1,
                         description="24^3 jittered unit box, Q4, 5^3 Gauss, 2,738,019 DoF"),
    "box12_q6": Workload("box12_q6", 20, 12, 12, 12, 6, jitter=0.1, amplitude=0.025,
                         nominal_amplitude=0.1, n_w=1,
                         description="12^3 jittered unit box, Q6, 7^3 Gauss, 1,167,051 DoF"),
    # twisted beam of the Newton-CG solve (geometry only at this point).
    "beam64_q2": Workload("beam64_q2", 3, 64, 16, 16, 2, lengths=(4.0, 1.0, 1.0), jitter=0.0,
                          lam=100.0, amplitude=0.0,
                          nominal_amplitude=0.0, n_w=1,
                          description="64x16x16 beam [0,4]x[0,1]^2, Q2, 421,443 DoF"),
}


def get_config(name: str) -> Workload:
    try:
        return CONFIGS[name]
    except KeyError as exc:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(CONFIGS)}") from exc
