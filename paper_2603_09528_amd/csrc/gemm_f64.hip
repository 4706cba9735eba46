// Instantiations of the FP64 eigenbasis-transform GEMMs.
#include "gemm_impl.h"

namespace tpt {

hipError_t launch_gemm_f64(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks, int variant,
                           hipStream_t s) {
    if (g.tA != DT_F64 || g.tB != DT_F64 || g.tC != DT_F64 || g.epi != EPI_STORE) return hipErrorInvalidValue;
    if (g.b_nk) return launch_gemm_typed<GP_F64, double, double, double, EPI_STORE, true>(g, d_work, nwork, blocks, variant, s);
    return launch_gemm_typed<GP_F64, double, double, double, EPI_STORE, false>(g, d_work, nwork, blocks, variant, s);
}

hipError_t launch_gemm_worklist_f64(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long tiles,
                                    hipStream_t s) {
    if (g.tA != DT_F64 || g.tB != DT_F64 || g.tC != DT_F64 || g.epi != EPI_STORE) return hipErrorInvalidValue;
    if (g.b_nk) return launch_worklist_typed<GP_F64, double, double, double, EPI_STORE, true>(d_work, nwork, tiles, s);
    return launch_worklist_typed<GP_F64, double, double, double, EPI_STORE, false>(d_work, nwork, tiles, s);
}

}  // namespace tpt
