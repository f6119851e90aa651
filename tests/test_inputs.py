"""Synthetic input generators: reproducibility, layout, and the det F guard
that fixes each workload's displacement amplitude."""

import numpy as np
import pytest

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh


def test_reproducible_and_layout():
    cfg = synthetic.get_config("box48_q2")
    v1, v2 = cfg.vertices(), cfg.vertices()
    assert np.array_equal(v1, v2) and v1.shape == (49 ** 3, 3)
    assert np.array_equal(cfg.test_vector(0), cfg.test_vector(0))
    assert not np.array_equal(cfg.test_vector(0), cfg.test_vector(1))
    # x fastest: vertex 1 is (h, 0, 0)
    assert np.allclose(v1[1], [1 / 48, 0, 0]) and np.allclose(v1[49], [0, 1 / 48, 0])
    assert cfg.n_dofs == 2_738_019 and cfg.n_qpoints == 2_985_984


def test_jitter_keeps_box_and_is_bounded():
    cfg = synthetic.get_config("cube4_q2_jit")
    v = cfg.vertices()
    ref = synthetic.box_vertices(4, 4, 4)
    d = np.abs(v - ref)
    assert d.max() <= 0.1 * 0.25 + 1e-15 and d.max() > 0.01
    on_bnd = (np.isclose(ref, 0) | np.isclose(ref, 1)).any(axis=1)
    assert np.array_equal(v[on_bnd], ref[on_bnd])


def test_displacement_dof_layout():
    u = synthetic.sine_displacement(2, 2, 2, 2, 1.0, np.random.default_rng(0), n_modes=1)
    assert u.shape == (3 * 125,)
    # a single product mode: component ratios are the same at every node
    U = u.reshape(-1, 3)
    big = np.abs(U[:, 0]) > 1e-3
    r = U[big, 1] / U[big, 0]
    assert np.allclose(r, r[0])


def _min_det_per_amplitude(cfg, amps):
    """min over all quadrature points of det(I + (a / amplitude) H) for each a."""
    mesh = BoxMesh(cfg.nx, cfg.ny, cfg.nz, cfg.degree, cfg.vertices())
    P = Problem(mesh, cfg.mu, cfg.lam, chunk=512)
    u = cfg.displacement()
    out = np.full(len(amps), np.inf)
    for el in P._chunks():
        H = P.deformation_gradient(u, el) - np.eye(3)
        for i, a in enumerate(amps):
            out[i] = min(out[i], np.linalg.det(np.eye(3) + (a / cfg.amplitude) * H).min())
    return out


@pytest.mark.parametrize("name", ["cube4_q2", "cube4_q2_jit", "box48_q2", "box24_q4", "box12_q6"])
def test_amplitude_guard(name):
    """amplitude = nominal amplitude halved until min det F >= 0.1."""
    cfg = synthetic.get_config(name)
    amps = [cfg.nominal_amplitude * 0.5 ** k for k in range(4)]
    dets = _min_det_per_amplitude(cfg, amps)
    first_ok = next(i for i, d in enumerate(dets) if d >= 0.1)
    assert amps[first_ok] == cfg.amplitude
