// Instantiations of the F32 eigenbasis-transform GEMMs.
#include "gemm_impl.h"

namespace tpt {

// x pass (B = basis, b_nk = 1): A is the FP64 right-hand side or an FP32
// buffer; C is an FP32 buffer, or the FP64 solution (stored or accumulated).
// y pass (A = basis, b_nk = 0): FP32 in and out.
hipError_t launch_gemm_f32(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks, int variant,
                           hipStream_t s) {
    if (g.b_nk) {
        if (g.tA == DT_F64 && g.tC == DT_F32 && g.epi == EPI_STORE)
            return launch_gemm_typed<GP_F32, double, float, float, EPI_STORE, true>(g, d_work, nwork, blocks, variant, s);
        if (g.tA == DT_F32 && g.tC == DT_F32 && g.epi == EPI_STORE)
            return launch_gemm_typed<GP_F32, float, float, float, EPI_STORE, true>(g, d_work, nwork, blocks, variant, s);
        if (g.tA == DT_F32 && g.tC == DT_F64 && g.epi == EPI_STORE)
            return launch_gemm_typed<GP_F32, float, float, double, EPI_STORE, true>(g, d_work, nwork, blocks, variant, s);
        if (g.tA == DT_F32 && g.tC == DT_F64 && g.epi == EPI_ACCUM_F64)
            return launch_gemm_typed<GP_F32, float, float, double, EPI_ACCUM_F64, true>(g, d_work, nwork, blocks, variant, s);
        return hipErrorInvalidValue;
    }
    if (g.tB == DT_F32 && g.tC == DT_F32 && g.epi == EPI_STORE)
        return launch_gemm_typed<GP_F32, float, float, float, EPI_STORE, false>(g, d_work, nwork, blocks, variant, s);
    return hipErrorInvalidValue;
}

hipError_t launch_gemm_worklist_f32(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long tiles,
                                    hipStream_t s) {
    if (g.b_nk) {
        if (g.tA == DT_F64 && g.tC == DT_F32 && g.epi == EPI_STORE)
            return launch_worklist_typed<GP_F32, double, float, float, EPI_STORE, true>(d_work, nwork, tiles, s);
        if (g.tA == DT_F32 && g.tC == DT_F32 && g.epi == EPI_STORE)
            return launch_worklist_typed<GP_F32, float, float, float, EPI_STORE, true>(d_work, nwork, tiles, s);
        if (g.tA == DT_F32 && g.tC == DT_F64 && g.epi == EPI_STORE)
            return launch_worklist_typed<GP_F32, float, float, double, EPI_STORE, true>(d_work, nwork, tiles, s);
        if (g.tA == DT_F32 && g.tC == DT_F64 && g.epi == EPI_ACCUM_F64)
            return launch_worklist_typed<GP_F32, float, float, double, EPI_ACCUM_F64, true>(d_work, nwork, tiles, s);
        return hipErrorInvalidValue;
    }
    if (g.tB == DT_F32 && g.tC == DT_F32 && g.epi == EPI_STORE)
        return launch_worklist_typed<GP_F32, float, float, float, EPI_STORE, false>(d_work, nwork, tiles, s);
    return hipErrorInvalidValue;
}

}  // namespace tpt
