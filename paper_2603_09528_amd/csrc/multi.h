// Multi-problem execution: one launch per stage (and tile variant) covering
// the tiles, lines and stencil blocks of many independent problems.  Used by
// batches (tpt_batch_*) and the serving loop (tpt_server_*).
#pragma once
#include <vector>

#include "internal.h"

namespace tpt {

// A fully resolved work list for one set of problems and one set of device
// pointers (rhs, out, workspace): descriptor arrays in one host blob, copied
// to the device once, plus the launch sequence that consumes them.
class MultiExec {
   public:
    // Validates the plans (same precision, nrhs == 1, fixed refinement for
    // mixed plans) and computes the workspace layout.
    int init(const std::vector<tpt_plan_s*>& plans);
    size_t workspace_bytes() const { return ws_total_; }
    // Build the descriptor blob for these pointers; d_desc must hold
    // desc_bytes() bytes of device memory (uploaded by upload()).
    int build(const double* const* rhs, double* const* out, void* ws);
    size_t desc_bytes() const { return blob_.size(); }
    int upload(void* d_desc, hipStream_t s);  // async copy of the blob (pinned staging)
    // Enqueue every launch on s (graph-capturable: kernels only).
    int enqueue(hipStream_t s) const;
    int count() const { return (int)plans_.size(); }
    int iterations() const { return iters_; }
    // per-problem device sums (TPT_STATS doubles, StatSlot order), STATS_BYTES
    // apart and back to back from norms(0)
    const double* norms(int i) const { return (const double*)((const char*)ws_ + norm_off_[i]); }
    static constexpr size_t STATS_BYTES = 256;
    tpt_plan_s* plan(int i) const { return plans_[i]; }
    ~MultiExec();

   private:
    struct Launch {
        int kind;     // 0 gemm, 1 sequential Thomas, 2 residual, 3 reduce, 4 x-line FFT, 5 partitioned Thomas,
                      // 6 right-hand-side check, 7 folding of fused-check partials,
                      // 8 work-list GEMM (persistent, all problems of the stage),
                      // 9 one GEMM problem on its own (single-problem kernel)
        // sequential Thomas: variant holds the largest nz; partitioned: the
        // configuration, prec the storage type
        int prec, variant, b_nk;
        size_t off;   // byte offset of the first descriptor in the blob
        int nwork;
        long long total;
    };
    // nb (if given): per problem of the stage, the blocks / tiles its GEMM
    // launch runs (the norm partials an accumulating stage writes)
    int add_gemm_stage(int stage, int prec, const std::vector<GemmDesc>& g, const std::vector<char>& use,
                       std::vector<long long>* nb = nullptr);
    int add_fft_stage(const std::vector<FftDesc>& f, const std::vector<char>& use);
    std::vector<tpt_plan_s*> plans_;
    int prec_ = GP_F64;
    bool mixed_ = false;
    int iters_ = 0;
    size_t ws_total_ = 0;
    std::vector<size_t> ws_off_, norm_off_;
    void* ws_ = nullptr;
    std::vector<char> blob_;
    std::vector<Launch> seq_;
    char* d_desc_ = nullptr;
    void* pinned_ = nullptr;
    size_t pinned_bytes_ = 0;
};

}  // namespace tpt
