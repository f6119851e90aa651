"""The oracle's C parts (CSR pattern, assembly and product) built with gcc's
address and undefined-behaviour sanitizers into a small standalone driver and
run on two small boxes and an empty-row matrix: any out-of-bounds access,
leak or undefined operation aborts the driver.  Its results must still equal
the numpy assembly and scipy's product.

Host only; the driver is compiled into the test's temporary directory."""

import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import synthetic
from oracle.fem import Problem
from oracle.mesh import BoxMesh

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

# reads the inputs the test writes, calls the three C entry points, writes the results
DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t csr_pattern_box(int nx, int ny, int nz, int p, int64_t* indptr);
int csr_assemble_box(int nx, int ny, int nz, int p, int nq3, const double* verts, const double* u, double mu,
                     double lam, const double* qw, const double* tri_grads, const double* basis_grads,
                     const int64_t* indptr, int32_t* indices, double* data);
int csr_spmv(int64_t n, const int64_t* indptr, const int32_t* indices, const double* data, const double* x,
             double* y);

static void* slurp(const char* dir, const char* name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "cannot open %s\n", path); exit(2); }
    void* buf = malloc(bytes ? bytes : 1);
    if (fread(buf, 1, bytes, f) != bytes) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return buf;
}

static void spill(const char* dir, const char* name, const void* buf, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE* f = fopen(path, "wb");
    if (!f || fwrite(buf, 1, bytes, f) != bytes) { fprintf(stderr, "cannot write %s\n", path); exit(2); }
    fclose(f);
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    const char* dir = argv[1];
    int64_t* hdr = slurp(dir, "header.bin", 8 * sizeof(int64_t));
    const int nx = (int)hdr[0], ny = (int)hdr[1], nz = (int)hdr[2], p = (int)hdr[3], nq3 = (int)hdr[4];
    const int64_t nverts = hdr[5], ndofs = hdr[6];
    const int n3 = (p + 1) * (p + 1) * (p + 1);
    double* mat = slurp(dir, "material.bin", 2 * sizeof(double));
    double* verts = slurp(dir, "verts.bin", (size_t)nverts * 3 * sizeof(double));
    double* u = slurp(dir, "u.bin", (size_t)ndofs * sizeof(double));
    double* x = slurp(dir, "x.bin", (size_t)ndofs * sizeof(double));
    double* qw = slurp(dir, "qw.bin", (size_t)nq3 * sizeof(double));
    double* tg = slurp(dir, "tri_grads.bin", (size_t)nq3 * 24 * sizeof(double));
    double* bg = slurp(dir, "basis_grads.bin", (size_t)nq3 * n3 * 3 * sizeof(double));
    int64_t* indptr = malloc((size_t)(ndofs + 1) * sizeof(int64_t));
    const int64_t nnz = csr_pattern_box(nx, ny, nz, p, indptr);
    int32_t* indices = malloc((size_t)nnz * sizeof(int32_t));
    double* data = malloc((size_t)nnz * sizeof(double));
    double* y = malloc((size_t)ndofs * sizeof(double));
    if (csr_assemble_box(nx, ny, nz, p, nq3, verts, u, mat[0], mat[1], qw, tg, bg, indptr, indices, data) < 1)
        return 3;
    if (csr_spmv(ndofs, indptr, indices, data, x, y) < 1) return 4;
    spill(dir, "indptr.bin", indptr, (size_t)(ndofs + 1) * sizeof(int64_t));
    spill(dir, "indices.bin", indices, (size_t)nnz * sizeof(int32_t));
    spill(dir, "data.bin", data, (size_t)nnz * sizeof(double));
    spill(dir, "y.bin", y, (size_t)ndofs * sizeof(double));
    /* a matrix with empty rows through the product alone */
    int64_t* eh = slurp(dir, "e_header.bin", 2 * sizeof(int64_t));
    int64_t* eptr = slurp(dir, "e_indptr.bin", (size_t)(eh[0] + 1) * sizeof(int64_t));
    int32_t* eidx = slurp(dir, "e_indices.bin", (size_t)eh[1] * sizeof(int32_t));
    double* edat = slurp(dir, "e_data.bin", (size_t)eh[1] * sizeof(double));
    double* ex = slurp(dir, "e_x.bin", (size_t)eh[0] * sizeof(double));
    double* ey = malloc((size_t)eh[0] * sizeof(double));
    if (csr_spmv(eh[0], eptr, eidx, edat, ex, ey) < 1) return 5;
    spill(dir, "e_y.bin", ey, (size_t)eh[0] * sizeof(double));
    free(hdr); free(mat); free(verts); free(u); free(x); free(qw); free(tg); free(bg);
    free(indptr); free(indices); free(data); free(y);
    free(eh); free(eptr); free(eidx); free(edat); free(ex); free(ey);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    d = tmp_path_factory.mktemp("sanitized")
    src = d / "driver.c"
    src.write_text(DRIVER)
    exe = d / "driver"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-o", str(exe), str(src),
           os.path.join(ORACLE, "csr_assemble.c"), os.path.join(ORACLE, "csr_spmv.c"), "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


@pytest.mark.parametrize("nx,ny,nz,p,jit", [(3, 2, 2, 2, 0.15), (2, 1, 2, 3, 0.1)])
def test_oracle_c_parts_under_sanitizers(driver, tmp_path, nx, ny, nz, p, jit):
    rng = np.random.default_rng(7 * nx + p)
    verts = synthetic.box_vertices(nx, ny, nz, (1.0, 0.8, 0.9), jit, rng)
    mesh = BoxMesh(nx, ny, nz, p, verts)
    u = synthetic.sine_displacement(nx, ny, nz, p, 0.03, np.random.default_rng(p + 1))
    x = np.random.default_rng(p + 2).standard_normal(mesh.n_dofs)
    mu, lam = 1.0, 10.0
    qw = np.ascontiguousarray(mesh.basis.weights, dtype=np.float64)
    np.array([nx, ny, nz, p, qw.size, verts.shape[0], mesh.n_dofs, 0], dtype=np.int64).tofile(tmp_path / "header.bin")
    np.array([mu, lam]).tofile(tmp_path / "material.bin")
    np.ascontiguousarray(verts, dtype=np.float64).tofile(tmp_path / "verts.bin")
    np.ascontiguousarray(u, dtype=np.float64).tofile(tmp_path / "u.bin")
    x.tofile(tmp_path / "x.bin")
    qw.tofile(tmp_path / "qw.bin")
    np.ascontiguousarray(mesh._tri_grads, dtype=np.float64).tofile(tmp_path / "tri_grads.bin")
    np.ascontiguousarray(mesh.basis.grads, dtype=np.float64).tofile(tmp_path / "basis_grads.bin")
    E = sp.random(40, 40, density=0.05, format="csr", random_state=np.random.default_rng(9))   # empty rows
    assert np.any(np.diff(E.indptr) == 0)
    ex = np.random.default_rng(10).standard_normal(40)
    np.array([40, E.nnz], dtype=np.int64).tofile(tmp_path / "e_header.bin")
    E.indptr.astype(np.int64).tofile(tmp_path / "e_indptr.bin")
    E.indices.astype(np.int32).tofile(tmp_path / "e_indices.bin")
    E.data.astype(np.float64).tofile(tmp_path / "e_data.bin")
    ex.tofile(tmp_path / "e_x.bin")

    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(driver), str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]

    K = Problem(mesh, mu, lam).assemble_tangent(u).tocsr()
    K.sort_indices()
    indptr = np.fromfile(tmp_path / "indptr.bin", dtype=np.int64)
    indices = np.fromfile(tmp_path / "indices.bin", dtype=np.int32)
    data = np.fromfile(tmp_path / "data.bin", dtype=np.float64)
    assert np.array_equal(indptr, K.indptr) and np.array_equal(indices, K.indices)
    assert np.max(np.abs(data - K.data)) <= 1e-13 * np.max(np.abs(K.data))
    y = np.fromfile(tmp_path / "y.bin", dtype=np.float64)
    assert np.linalg.norm(y - K @ x) <= 1e-13 * np.linalg.norm(K @ x)
    assert np.allclose(np.fromfile(tmp_path / "e_y.bin", dtype=np.float64), E @ ex, rtol=1e-14, atol=1e-14)
