"""The benchmark's work model and roofline arithmetic (host only).

The per-point flop counts of the Q2 strategies are checked against an
independent tally of the operations (Sec. 2.4 sum factorization with the
even-odd 1D kernels, Sec. 2.5.1 / Alg. 2 point-wise products), and the
algorithmic bytes against the storage each strategy streams (Sec. 3.2.2:
nothing, the Jacobians, 17 or 36 numbers per point)."""

import json
import os

import pytest

import bench


def tally_sweep_q2():
    """One forward (or backward) sum factorization of a 3-vector field at Q2
    (n = 3 points per direction), per quadrature point: per component, three
    interpolation sweeps and three collocation-derivative sweeps, each a 1D
    product of a 3 x 3 matrix in even-odd form (2 x 2 even block, 1 x 1 odd
    block: 5 FMAs) plus the 2 additions and 2 subtractions that split and
    join the halves, per 1D line of 3 points."""
    per_line = 2 * (2 * 2 + 1 * 1) + 4 * 1    # FMAs x 2 flops + splits/joins
    per_point_per_sweep = per_line / 3.0
    return 3 * 6 * per_point_per_sweep        # 3 components x 6 sweeps


def test_sweep_flops_match_a_direct_tally():
    assert bench.sweep_flops_per_q(3) == pytest.approx(tally_sweep_q2())
    assert tally_sweep_q2() == pytest.approx(84.0)


@pytest.mark.parametrize("strategy,flops,cached", [("otf", 776, 0), ("otf_ad", 776, 0), ("otf_geom", 626, 80),
                                                   ("t2", 356, 136), ("t4", 399, 288)])
def test_per_point_counts_q2(strategy, flops, cached):
    sweep = tally_sweep_q2()
    transform = 54.0          # a 3 x 3 by 3 x 3 product: 27 FMAs
    geom, kin, jxw = 150.0, 50.0, 9.0
    pointwise = {"otf": 153.0, "otf_ad": 153.0, "otf_geom": 153.0, "t2": 80.0, "t4": 123.0}[strategy]
    if strategy in ("otf", "otf_ad"):   # u and w forward, w backward; both fields and Q transformed
        expect = 3 * sweep + 3 * transform + jxw + geom + kin + pointwise
    elif strategy == "otf_geom":        # geometry loaded instead of computed
        expect = 3 * sweep + 3 * transform + jxw + kin + pointwise
    else:                               # w forward and backward; h = dw M and Q = g M^T
        expect = 2 * sweep + 2 * transform + pointwise
    m = bench.work_model(strategy, 2, 2738019, 2985984, 49 ** 3)
    assert expect == pytest.approx(flops)
    assert m["flops_per_q"] == pytest.approx(flops)
    assert m["bytes_per_q"] == pytest.approx(cached)   # 0, 10 doubles, 17 doubles, 36 doubles


def test_headline_bytes_and_roofline_arithmetic():
    n_dofs, n_q = 2738019, 2985984
    m = bench.work_model("t2", 2, n_dofs, n_q, 49 ** 3)
    # the T2 cache (17 doubles per point) streamed once, w read and v written once
    assert m["bytes"] == pytest.approx(17 * 8 * n_q + 2 * 8 * n_dofs)
    assert m["bytes"] / 1e6 == pytest.approx(449.9, abs=0.1)
    assert m["bound"] == "hbm"
    rl = bench.roofline(m, 0.09, 12345)
    assert rl["achieved"] == pytest.approx(m["bytes"] / 0.09e-3 / 1e9, rel=1e-3)
    assert rl["frac"] == pytest.approx(rl["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert rl["traffic"] == 12345
    otf = bench.work_model("otf", 2, n_dofs, n_q, 49 ** 3)
    assert otf["bound"] == "alu"
    assert bench.roofline(otf, 0.1, None)["unit"] == "TFLOP/s"


def test_measured_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    """Traffic is reported only under the hash of the kernel sources it was measured on."""
    h = bench.kernel_source_hash()
    root = tmp_path
    (root / "profiles").mkdir()
    data = {"box48_q2/t2": {"bytes_per_launch": 123, "source_hash": h},
            "box48_q2/t4": {"bytes_per_launch": 456, "source_hash": "0" * 16}}
    (root / "profiles" / "traffic.json").write_text(json.dumps(data))
    for rel in bench.KERNEL_SOURCES:   # the same sources, so the same hash
        dst = root / rel
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(bench.ROOT, rel), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(root))
    assert bench.kernel_source_hash() == h
    assert bench.measured_traffic("box48_q2", "t2") == 123
    assert bench.measured_traffic("box48_q2", "t4") is None
    assert bench.measured_traffic("box48_q2", "otf") is None


@pytest.mark.parametrize("strategy,degree,precision,kernel", [
    ("t2", 2, "fp64", "wave_kernel"), ("t4", 2, "fp32", "wave_kernel"), ("otf", 2, "fp64", "cell_kernel"),
    ("otf", 2, "fp32", "cell_kernel"), ("otf_ad", 2, "fp64", "cell_kernel"), ("otf_geom", 2, "fp64", "cell_kernel"),
    ("otf_geom", 2, "fp32", "wave_kernel"), ("t2", 4, "fp64", "cell_kernel"), ("t4", 6, "fp32", "cell_kernel")])
def test_kernel_label_follows_the_routing(strategy, degree, precision, kernel):
    """The roofline's kernel label names the kernel the library routes the
    apply to (the cached strategies and the FP32 geometry-cached one on Q2
    boxes run in the wavefront kernel, the rest in the brick kernel)."""
    assert bench.apply_kernel_name(strategy, degree, precision) == f"{kernel} apply {strategy} {precision}"


def test_oracle_check_is_the_relative_error_of_every_strategy():
    import numpy as np
    ref = np.array([3.0, 4.0])
    out = bench.oracle_check({"t2": ref + np.array([0.0, 5e-3]), "otf": ref.copy()},
                             {"assembled_csr": ref, "naive_loop": 2 * ref})
    assert out["assembled_csr"]["t2"] == pytest.approx(1e-3) and out["assembled_csr"]["otf"] == 0.0
    assert out["naive_loop"]["otf"] == pytest.approx(0.5)
