// Cell kernels on general hexahedral meshes: the templates of mfe_cell.hpp
// instantiated for groups of consecutive cells gathered and scattered through
// the cell-node table (every node written with FP64 atomics).

#include "mfe_cell.hpp"

namespace mfe {

hipError_t launch_cell_kernel_hex(int mode, const Tables1D& t, const KParams& p, hipStream_t stream, bool fp32,
                                  const LaunchTiming& tm) {
    if (p.ne <= 0) return hipSuccess;
    switch (t.n) {
        case 2: return launch_n<2, true>(mode, fp32, t, p, stream, 0, tm);
        case 3: return launch_n<3, true>(mode, fp32, t, p, stream, 0, tm);
        case 4: return launch_n<4, true>(mode, fp32, t, p, stream, 0, tm);
        case 5: return launch_n<5, true>(mode, fp32, t, p, stream, 0, tm);
        case 6: return launch_n<6, true>(mode, fp32, t, p, stream, 0, tm);
        case 7: return launch_n<7, true>(mode, fp32, t, p, stream, 0, tm);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_diagonal_hex(const Tables1D& t, const KParams& p, double* diag, hipStream_t stream) {
    if (p.ne <= 0) return hipSuccess;
    switch (t.n) {
        case 2: return launch_diag_n<2, true>(t, p, diag, stream);
        case 3: return launch_diag_n<3, true>(t, p, diag, stream);
        case 4: return launch_diag_n<4, true>(t, p, diag, stream);
        case 5: return launch_diag_n<5, true>(t, p, diag, stream);
        case 6: return launch_diag_n<6, true>(t, p, diag, stream);
        case 7: return launch_diag_n<7, true>(t, p, diag, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mfe
