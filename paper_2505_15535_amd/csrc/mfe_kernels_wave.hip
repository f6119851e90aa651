// Instantiations and launch of the Q2 box tangent applies organised around
// the wavefront (mfe_wave.hpp).

#include "mfe_wave.hpp"

namespace mfe {

bool wave_apply(int n, int mode, bool hex, int sweep, bool fp32, bool coloured) {
    if (n != 3 || hex || sweep != 0) return false;
    switch (mode) {
        // the on-the-fly strategies are bound by their arithmetic and run
        // faster with the brick kernel, whose 256 lanes all hold a point,
        // than with 54 of 64 lanes per wavefront (48^3 Q2, FP64: OTF 120
        // against 140 us, OTF-AD 129 against 140 us; FP32 OTF: equal); the
        // FP32 geometry-cached one is faster here (98 against 113 us)
        case MODE_APPLY_OTF:
        case MODE_APPLY_OTF_AD: return coloured;
        case MODE_APPLY_OTF_GEOM: return fp32 || coloured;
        case MODE_APPLY_T2:
        case MODE_APPLY_T4:
        case MODE_APPLY_OTF_AD_SPLIT: return true;
        default: return false;
    }
}

int64_t colour_bricks(int nbx, int nby, int nbz, int colour) {
    if (colour < 1 || colour > 8) return 0;
    const int c = colour - 1;
    return (int64_t)((nbx - (c & 1) + 1) / 2) * ((nby - ((c >> 1) & 1) + 1) / 2) * ((nbz - (c >> 2) + 1) / 2);
}

template <int MODE, typename R>
static hipError_t launch_wave_m(const Tables<3>& T, const KParams& p, hipStream_t stream, const LaunchTiming& tm) {
    const int64_t nb = p.colour > 0 ? colour_bricks(p.nbx, p.nby, p.nbz, p.colour) : (int64_t)p.nbx * p.nby * p.nbz;
    if (nb <= 0) return hipSuccess;
    Tables<3, R> TR;
    if constexpr (std::is_same_v<R, float>) TR = to_float<3>(T);
    else TR = T;
    if (tm.start)
        hipExtLaunchKernelGGL((wave_kernel<MODE, R>), dim3((unsigned)nb), dim3(WaveGeo::NT), 0, stream, tm.start, tm.stop, 0,
                              p, T, TR);
    else
        hipLaunchKernelGGL((wave_kernel<MODE, R>), dim3((unsigned)nb), dim3(WaveGeo::NT), 0, stream, p, T, TR);
    return hipGetLastError();
}

template <typename R>
static hipError_t launch_wave_r(int mode, const Tables<3>& T, const KParams& p, hipStream_t s,
                                const LaunchTiming& tm) {
    switch (mode) {
        case MODE_APPLY_OTF: return launch_wave_m<MODE_APPLY_OTF, R>(T, p, s, tm);
        case MODE_APPLY_OTF_GEOM: return launch_wave_m<MODE_APPLY_OTF_GEOM, R>(T, p, s, tm);
        case MODE_APPLY_T2: return launch_wave_m<MODE_APPLY_T2, R>(T, p, s, tm);
        case MODE_APPLY_T4: return launch_wave_m<MODE_APPLY_T4, R>(T, p, s, tm);
        case MODE_APPLY_OTF_AD: return launch_wave_m<MODE_APPLY_OTF_AD, R>(T, p, s, tm);
        case MODE_APPLY_OTF_AD_SPLIT: return launch_wave_m<MODE_APPLY_OTF_AD_SPLIT, R>(T, p, s, tm);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_wave(int mode, bool fp32, const Tables1D& t, const KParams& p, hipStream_t stream,
                       const LaunchTiming& tm) {
    if (p.ne <= 0) return hipSuccess;
    const Tables<3> T = make_tables<3>(t);
    return fp32 ? launch_wave_r<float>(mode, T, p, stream, tm) : launch_wave_r<double>(mode, T, p, stream, tm);
}

}  // namespace mfe
