// Multi-problem execution (batches of uneven independent problems) and the
// GEMM tile autotuner.
#include "multi.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <tuple>

namespace tpt {

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

MultiExec::~MultiExec() {
    if (pinned_) (void)hipHostFree(pinned_);
}

int MultiExec::init(const std::vector<tpt_plan_s*>& plans) {
    if (plans.empty()) return fail(TPT_ERR_INVALID, "empty batch");
    plans_ = plans;
    const int prec = plans[0]->desc.precision;
    for (auto* p : plans) {
        if (!p) return fail(TPT_ERR_INVALID, "NULL plan in batch");
        if (p->host_only) return fail(TPT_ERR_INVALID, "host-only plan in batch");
        if (p->desc.nrhs != 1) return fail(TPT_ERR_UNSUPPORTED, "batched plans must have nrhs = 1");
        if (p->desc.precision != prec) return fail(TPT_ERR_UNSUPPORTED, "batched plans must share a precision");
        if (prec != TPT_FP64 && p->desc.fixed_refine < 0)
            return fail(TPT_ERR_UNSUPPORTED, "batched mixed plans need fixed_refine >= 0");
        if (prec != TPT_FP64 && p->desc.fixed_refine != plans[0]->desc.fixed_refine)
            return fail(TPT_ERR_UNSUPPORTED, "batched mixed plans must share fixed_refine");
    }
    prec_ = plan_gemm_prec(plans[0]);
    mixed_ = prec != TPT_FP64;
    iters_ = mixed_ ? plans[0]->desc.fixed_refine : 0;
    ws_off_.clear();
    norm_off_.clear();
    size_t off = 0;
    for (auto* p : plans) {
        ws_off_.push_back(off);
        off += al256(plan_workspace_bytes(p));
    }
    // the per-problem sums back to back at the end, so one copy reads them all
    for (size_t i = 0; i < plans.size(); ++i) {
        norm_off_.push_back(off);
        off += STATS_BYTES;
    }
    ws_total_ = off;
    return TPT_OK;
}

template <typename T>
static size_t append(std::vector<char>& blob, const std::vector<T>& v) {
    size_t off = (blob.size() + 15) & ~(size_t)15;
    blob.resize(off + sizeof(T) * v.size());
    std::memcpy(blob.data() + off, v.data(), sizeof(T) * v.size());
    return off;
}

int MultiExec::add_gemm_stage(int stage, int prec, const std::vector<GemmDesc>& gs, const std::vector<char>& use,
                              std::vector<long long>* nb) {
    // A problem whose single solve runs the persistent tile runs it here too,
    // one launch per problem, while there are at most four
    // of them (large grids: each launch fills the GPU); the other FP64 / FP32
    // problems share one work-list launch of the persistent work-list tile;
    // anything else (BF16x3, extents past the work-list kernel's 32-bit
    // offsets) one launch per tile variant of the plain tile kernel.
    std::vector<int> var(gs.size());
    int npersist = 0, nuse = 0;
    bool all_big = true;
    for (size_t i = 0; i < gs.size(); ++i) {
        var[i] = use[i] ? stage_variant(plans_[i], stage, gs[i], prec) : -1;
        if (!use[i]) continue;
        ++nuse;
        if (tv_persistent(var[i])) ++npersist;
        if (gemm_blocks(gs[i], TV_128x128) < 1024) all_big = false;
    }
    const bool solo_persist = npersist <= 4;
    // at most four problems that each fill the GPU (>= 1024 tiles of 128 x
    // 128): every one its own launch of the tile its single solve runs
    if (nuse > 0 && nuse <= 4 && all_big) {
        for (size_t i = 0; i < gs.size(); ++i) {
            if (!use[i]) continue;
            int bm, bn;
            tile_variant_shape(var[i], &bm, &bn);
            GemmDesc g = gs[i];
            g.tiles_m = (g.M + bm - 1) / bm;
            g.tiles_n = (g.N + bn - 1) / bn;
            g.block_begin = 0;
            if (nb) (*nb)[i] = gemm_blocks(gs[i], var[i]);
            Launch L{};
            L.kind = 9;
            L.prec = prec;
            L.variant = var[i];
            L.b_nk = g.b_nk;
            L.off = append(blob_, std::vector<GemmDesc>{g});
            L.nwork = 1;
            L.total = gemm_blocks(gs[i], var[i]);
            seq_.push_back(L);
        }
        return TPT_OK;
    }
    std::vector<char> wl(gs.size(), 0);
    {
        std::vector<GemmDesc> grp;
        long long total = 0;
        for (size_t i = 0; i < gs.size(); ++i) {
            if (!use[i] || prec == GP_BF16X3 || (solo_persist && tv_persistent(var[i])) || !worklist_ok(gs[i], prec))
                continue;
            wl[i] = 1;
            GemmDesc g = gs[i];
            worklist_shape(g);
            g.block_begin = total;
            const long long t = (long long)g.tiles_m * g.tiles_n;
            total += t;
            if (nb) (*nb)[i] = t;
            grp.push_back(g);
        }
        if (!grp.empty()) {
            Launch L{};
            L.kind = 8;
            L.prec = prec;
            L.b_nk = grp[0].b_nk;
            L.off = append(blob_, grp);
            L.nwork = (int)grp.size();
            L.total = total;
            seq_.push_back(L);
        }
    }
    for (int v = 0; v < TV_COUNT; ++v) {
        std::vector<GemmDesc> grp;
        long long total = 0;
        int bm, bn;
        tile_variant_shape(v, &bm, &bn);
        for (size_t i = 0; i < gs.size(); ++i) {
            if (var[i] != v || wl[i]) continue;
            GemmDesc g = gs[i];
            g.tiles_m = (g.M + bm - 1) / bm;
            g.tiles_n = (g.N + bn - 1) / bn;
            g.block_begin = total;
            total += (long long)g.tiles_m * g.tiles_n * g.batch;
            if (nb) (*nb)[i] = gemm_blocks(gs[i], v);
            grp.push_back(g);
        }
        if (grp.empty()) continue;
        Launch L{};
        L.kind = 0;
        L.prec = prec;
        L.variant = v;
        L.b_nk = grp[0].b_nk;
        L.off = append(blob_, grp);
        L.nwork = (int)grp.size();
        L.total = total;
        seq_.push_back(L);
    }
    return TPT_OK;
}

int MultiExec::add_fft_stage(const std::vector<FftDesc>& fs, const std::vector<char>& use) {
    // one persistent launch per line length (block shape and LDS depend on it)
    std::vector<int> lens;
    for (size_t i = 0; i < fs.size(); ++i)
        if (use[i] && std::find(lens.begin(), lens.end(), fs[i].n) == lens.end()) lens.push_back(fs[i].n);
    for (int n : lens) {
        std::vector<FftDesc> grp;
        long long total = 0;
        for (size_t i = 0; i < fs.size(); ++i) {
            if (!use[i] || fs[i].n != n) continue;
            FftDesc f = fs[i];
            f.block_begin = total;
            total += fft_blocks(f);
            grp.push_back(f);
        }
        Launch L{};
        L.kind = 4;
        L.off = append(blob_, grp);
        L.nwork = (int)grp.size();
        L.total = total;
        seq_.push_back(L);
    }
    return TPT_OK;
}

int MultiExec::build(const double* const* rhs, double* const* out, void* ws) {
    blob_.clear();
    seq_.clear();
    ws_ = ws;
    const int n = (int)plans_.size();
    std::vector<Ws> w(n);
    for (int i = 0; i < n; ++i) {
        if (!rhs[i] || !out[i]) return fail(TPT_ERR_INVALID, "NULL rhs/out in batch");
        w[i] = carve(plans_[i], (char*)ws + ws_off_[i]);
    }
    // right-hand-side checks (filled below): descriptors, and which ride in
    // the first x forward pass
    std::vector<CheckDesc> chk(n);
    std::vector<char> fused(n, 0);
    std::vector<CheckDesc> fused_list;
    // per stage: which problems apply it (a direction the plan leaves
    // explicit has no transform), and of those which take the fast
    // transform, which the GEMM
    auto applies = [&](int i, int stage) {
        return (stage == ST_XF || stage == ST_XI) ? plans_[i]->tx : plans_[i]->ty;
    };
    auto fast_mask = [&](int stage, bool fast) {
        std::vector<char> m(n);
        for (int i = 0; i < n; ++i) m[i] = applies(i, stage) && stage_is_fast(plans_[i], stage) == fast ? 1 : 0;
        return m;
    };
    // one transform stage of every problem that applies it: GEMM launches
    // grouped by tile variant, fast-transform launches grouped by line length
    auto stage = [&](int st, const std::vector<const void*>& in, int tin, const std::vector<void*>& outp, int tout,
                     int epi, std::vector<long long>* nb, bool with_check = false) {
        std::vector<GemmDesc> g(n);
        std::vector<FftDesc> f(n);
        for (int i = 0; i < n; ++i) {
            if (!applies(i, st)) continue;
            double* part = epi == EPI_ACCUM_F64 ? w[i].partials : nullptr;
            if (stage_is_fast(plans_[i], st)) {
                f[i] = stage_fft(plans_[i], st, in[i], tin, outp[i], tout, epi, part, 1);
                if (with_check && fused[i]) attach_check(plans_[i], chk[i], f[i]);
                if (nb) (*nb)[i] = fft_blocks(f[i]);
            } else {
                g[i] = stage_gemm(plans_[i], st, prec_, in[i], tin, outp[i], tout, epi, part, 1);
            }
        }
        add_gemm_stage(st, prec_, g, fast_mask(st, false), nb);
        add_fft_stage(f, fast_mask(st, true));
    };
    std::vector<void*> w1(n), w2(n), outv(n);
    std::vector<const void*> w1c(n), w2c(n), rhsv(n), resv(n);
    for (int i = 0; i < n; ++i) {
        w1[i] = w[i].w1;
        w2[i] = w[i].w2;
        w1c[i] = w[i].w1;
        w2c[i] = w[i].w2;
        outv[i] = out[i];
        rhsv[i] = rhs[i];
        resv[i] = w[i].r;
    }
    // one application of M^{-1}; returns the x-inverse block count of every
    // problem (the number of norm partials it wrote)
    // Data flow of one problem: rhs (or residual) -> [x fwd -> w1] -> [y fwd
    // -> w2] -> Thomas -> [y inv] -> [x inv] -> out, the bracketed stages only
    // for transformed directions (plans with an explicit direction are FP64,
    // where every buffer has one type).
    auto minv = [&](bool from_rhs, int epi) {
        const int tmid = mixed_ ? DT_F32 : DT_F64;
        std::vector<long long> nb(n);
        std::vector<const void*> src(from_rhs ? rhsv : resv);
        stage(ST_XF, src, from_rhs ? DT_F64 : DT_F32, w1, tmid, EPI_STORE, nullptr, from_rhs);
        if (from_rhs && !fused_list.empty()) {
            Launch L{};
            L.kind = 7;
            L.off = append(blob_, fused_list);
            L.nwork = (int)fused_list.size();
            seq_.push_back(L);
        }
        for (int i = 0; i < n; ++i)
            if (plans_[i]->tx) src[i] = w1c[i];
        stage(ST_YF, src, tmid, w2, tmid, EPI_STORE, nullptr);
        // one launch per Thomas kernel: each problem runs the variant its
        // single-problem solve runs, so batch and single results agree bit
        // for bit; a z-only problem solves straight from rhs into out
        std::vector<ThomasDesc> all(n);
        std::vector<int> var(n);
        for (int i = 0; i < n; ++i) {
            const bool zonly = !plans_[i]->ty;
            all[i] = plan_thomas(plans_[i], zonly ? src[i] : w[i].w2, tmid, zonly ? outv[i] : w[i].w2, tmid,
                                 w[i].scratch, 1);
            var[i] = thomas_variant(all[i]);
        }
        std::vector<int> kinds(var);
        std::sort(kinds.begin(), kinds.end());
        kinds.erase(std::unique(kinds.begin(), kinds.end()), kinds.end());
        for (int v : kinds) {
            std::vector<ThomasDesc> t;
            long long blocks = 0;
            int nz_max = 1;
            for (int i = 0; i < n; ++i) {
                if (var[i] != v) continue;
                ThomasDesc d = all[i];
                d.block_begin = blocks;
                blocks += v == THOMAS_SEQ ? thomas_blocks(d) : thomas_part_blocks(d, v - THOMAS_PART);
                nz_max = std::max(nz_max, d.nz);
                t.push_back(d);
            }
            Launch L{};
            L.kind = v == THOMAS_SEQ ? 1 : 5;
            L.off = append(blob_, t);
            L.nwork = (int)t.size();
            L.total = blocks;
            L.variant = v == THOMAS_SEQ ? nz_max : v - THOMAS_PART;
            L.prec = tmid;
            seq_.push_back(L);
        }
        std::vector<void*> yout(w1);
        for (int i = 0; i < n; ++i)
            if (!plans_[i]->tx) yout[i] = outv[i];
        stage(ST_YI, w2c, tmid, yout, tmid, EPI_STORE, nullptr);
        stage(ST_XI, w1c, tmid, outv, DT_F64, epi, &nb);
        return nb;
    };
    // right-hand-side checks of the plans that ask for them: in the loads of
    // the first x forward pass where a single solve fuses it (the same
    // partials, so batch and single results stay bitwise equal), else a
    // separate pass first
    {
        std::vector<CheckDesc> cd;
        long long blocks = 0;
        for (int i = 0; i < n; ++i) {
            if (!plans_[i]->run_check) continue;
            CheckDesc c = check_desc(plans_[i], rhs[i], w[i].partials);
            c.out = (double*)((char*)ws + norm_off_[i]) + SS_WF;
            chk[i] = c;
            if (check_fused(plans_[i])) {
                fused[i] = 1;
                c.nblk = check_fused_blocks(plans_[i]);
                fused_list.push_back(c);
                continue;
            }
            c.block_begin = blocks;
            blocks += check_blocks(c);
            cd.push_back(c);
        }
        if (!cd.empty()) {
            Launch L{};
            L.kind = 6;
            L.off = append(blob_, cd);
            L.nwork = (int)cd.size();
            L.total = blocks;
            seq_.push_back(L);
        }
    }
    std::vector<long long> xi = minv(true, EPI_STORE);
    for (int it = 0; it < iters_; ++it) {
        std::vector<StencilDesc> st(n);
        std::vector<ReduceDesc> rd(n);
        long long blocks = 0;
        for (int i = 0; i < n; ++i) {
            st[i] = plan_stencil(plans_[i], out[i], rhs[i], w[i].r, w[i].partials,
                                 (const double*)((char*)ws + norm_off_[i]));
            st[i].block_begin = blocks;
            const int nb = residual_blocks(st[i]);
            blocks += nb;
            rd[i].partials = w[i].partials;
            rd[i].n = nb;
            rd[i].out = (double*)((char*)ws + norm_off_[i]);
        }
        Launch L{};
        L.kind = 2;
        L.off = append(blob_, st);
        L.nwork = n;
        L.total = blocks;
        seq_.push_back(L);
        Launch R{};
        R.kind = 3;
        R.off = append(blob_, rd);
        R.nwork = n;
        seq_.push_back(R);
        xi = minv(false, EPI_ACCUM_F64);
        for (int i = 0; i < n; ++i) {
            rd[i].partials = w[i].partials;
            rd[i].n = (int)xi[i];
            rd[i].out = (double*)((char*)ws + norm_off_[i]) + 2;
        }
        Launch R2{};
        R2.kind = 3;
        R2.off = append(blob_, rd);
        R2.nwork = n;
        seq_.push_back(R2);
    }
    return TPT_OK;
}

int MultiExec::upload(void* d_desc, hipStream_t s) {
    d_desc_ = (char*)d_desc;
    if (blob_.empty()) return TPT_OK;
    if (pinned_bytes_ < blob_.size()) {
        if (pinned_) TPT_HIP(hipHostFree(pinned_));
        pinned_ = nullptr;
        pinned_bytes_ = 0;
        TPT_HIP(hipHostMalloc(&pinned_, blob_.size(), hipHostMallocDefault));
        pinned_bytes_ = blob_.size();
    }
    std::memcpy(pinned_, blob_.data(), blob_.size());
    TPT_HIP(hipMemcpyAsync(d_desc, pinned_, blob_.size(), hipMemcpyHostToDevice, s));
    TPT_HIP(hipStreamSynchronize(s));
    return TPT_OK;
}

int MultiExec::enqueue(hipStream_t s) const {
    for (const Launch& L : seq_) {
        hipError_t e = hipSuccess;
        switch (L.kind) {
            case 9: {
                // one large problem on its own (its single-solve tile)
                TimedScope ts("multi_gemm", s);
                e = launch_gemm(*(const GemmDesc*)(blob_.data() + L.off), L.prec, L.variant, s);
                break;
            }
            case 8: {
                TimedScope ts("multi_gemm", s);
                const GemmDesc& rep = *(const GemmDesc*)(blob_.data() + L.off);
                e = launch_gemm_worklist(rep, (const GemmDesc*)(d_desc_ + L.off), L.nwork, L.total, L.prec, s);
                break;
            }
            case 0: {
                const GemmDesc* hd = (const GemmDesc*)(blob_.data() + L.off);
                if (tv_persistent(L.variant) && L.nwork <= 4) {
                    // a few problems on a persistent tile: one launch each.  A
                    // work list runs the plain 128 x 128 tile instead (the
                    // persistent one prefetches the next tile of the same
                    // problem), about 10 % slower on large K; every output sees
                    // the same MFMA sequence either way, so results are the same
                    for (int k = 0; k < L.nwork && e == hipSuccess; ++k) {
                        TimedScope ts("multi_gemm", s);
                        e = launch_gemm(hd[k], L.prec, L.variant, s);
                    }
                } else {
                    TimedScope ts("multi_gemm", s);
                    e = launch_gemm_multi(hd[0], (const GemmDesc*)(d_desc_ + L.off), L.nwork, L.total, L.prec,
                                          L.variant, s);
                }
                break;
            }
            case 1: {
                TimedScope ts("multi_thomas", s);
                e = launch_thomas_multi((const ThomasDesc*)(d_desc_ + L.off), L.nwork, L.total, L.variant, s);
                break;
            }
            case 5: {
                TimedScope ts("multi_thomas", s);
                e = launch_thomas_part_multi((const ThomasDesc*)(d_desc_ + L.off), L.nwork, L.total, L.variant,
                                             L.prec, s);
                break;
            }
            case 2: {
                TimedScope ts("multi_residual", s);
                e = launch_residual_multi((const StencilDesc*)(d_desc_ + L.off), L.nwork, L.total, s);
                break;
            }
            case 3: {
                TimedScope ts("multi_reduce", s);
                e = launch_reduce_pairs_multi((const ReduceDesc*)(d_desc_ + L.off), L.nwork, s);
                break;
            }
            case 6: {
                TimedScope ts("multi_check", s);
                e = launch_check_multi((const CheckDesc*)(d_desc_ + L.off), L.nwork, L.total, s);
                break;
            }
            case 7: {
                TimedScope ts("multi_check_reduce", s);
                e = launch_check_reduce_multi((const CheckDesc*)(d_desc_ + L.off), L.nwork, s);
                break;
            }
            case 4: {
                TimedScope ts("multi_fft", s);
                const FftDesc& rep = *(const FftDesc*)(blob_.data() + L.off);
                e = launch_fft(rep, (const FftDesc*)(d_desc_ + L.off), L.nwork, L.total, s);
                break;
            }
        }
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("multi launch: ") + hipGetErrorString(e));
    }
    return TPT_OK;
}

}  // namespace tpt

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
struct tpt_batch_s {
    tpt::MultiExec exec;
    int device = 0;
    void* d_desc = nullptr;
    size_t d_desc_bytes = 0;
    // cached work list / graph for one pointer set and stream
    std::vector<const void*> key;
    bool built = false;
    hipGraphExec_t gexec = nullptr;
    hipStream_t capture = nullptr;  // private stream used only to record the graph
    ~tpt_batch_s() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (capture) (void)hipStreamDestroy(capture);
        if (d_desc) (void)hipFree(d_desc);
    }
};

using namespace tpt;

extern "C" {

int tpt_batch_create(int count, const tpt_plan* plans, tpt_batch* out) {
    if (count < 1 || !plans || !out) return fail(TPT_ERR_INVALID, "bad batch arguments");
    *out = nullptr;
    std::unique_ptr<tpt_batch_s> b(new tpt_batch_s());
    std::vector<tpt_plan_s*> v(plans, plans + count);
    int rc = b->exec.init(v);
    if (rc) return rc;
    TPT_HIP(hipGetDevice(&b->device));
    *out = b.release();
    return TPT_OK;
}

int tpt_batch_destroy(tpt_batch b) {
    delete b;
    return TPT_OK;
}

int tpt_batch_workspace_bytes(tpt_batch b, size_t* bytes) {
    if (!b || !bytes) return fail(TPT_ERR_INVALID, "NULL argument");
    *bytes = b->exec.workspace_bytes();
    return TPT_OK;
}

int tpt_batch_info(tpt_batch b, int index, tpt_info* info) {
    if (!b || !info) return fail(TPT_ERR_INVALID, "NULL argument");
    if (index < 0 || index >= b->exec.count()) return fail(TPT_ERR_INVALID, "problem index out of range");
    if (!b->built) return fail(TPT_ERR_INVALID, "the batch has not been solved");
    tpt_plan_s* p = b->exec.plan(index);
    double h[TPT_STATS];
    TPT_HIP(hipMemcpy(h, b->exec.norms(index), sizeof(h), hipMemcpyDeviceToHost));
    tpt_info inf{};
    inf.iters = b->exec.iterations();
    inf.null_line = p->null_line;
    inf.rel_correction = 0.0;
    inf.rel_residual = -1.0;
    inf.compat_defect = -1.0;
    inf.nonfinite = -1;
    stats_to_info(p, h, inf.iters > 0, &inf);
    *info = inf;
    return TPT_OK;
}

int tpt_batch_solve(tpt_batch b, const double* const* rhs, double* const* out, void* ws, size_t ws_bytes,
                    void* stream, int use_graph) {
    if (!b || !rhs || !out || !ws) return fail(TPT_ERR_INVALID, "NULL argument");
    if (ws_bytes < b->exec.workspace_bytes()) return fail(TPT_ERR_WORKSPACE, "batch workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int n = b->exec.count();
    std::vector<const void*> key;
    key.reserve(2 * n + 2);
    for (int i = 0; i < n; ++i) {
        key.push_back(rhs[i]);
        key.push_back(out[i]);
    }
    key.push_back(ws);
    key.push_back((const void*)s);
    if (!b->built || key != b->key) {
        if (b->gexec) {
            TPT_HIP(hipGraphExecDestroy(b->gexec));
            b->gexec = nullptr;
        }
        int rc = b->exec.build(rhs, out, ws);
        if (rc) return rc;
        if (b->d_desc_bytes < b->exec.desc_bytes()) {
            if (b->d_desc) TPT_HIP(hipFree(b->d_desc));
            b->d_desc = nullptr;
            b->d_desc_bytes = 0;
            if (hipMalloc(&b->d_desc, b->exec.desc_bytes()) != hipSuccess) {
                (void)hipGetLastError();
                return fail(TPT_ERR_OOM, "batch descriptors");
            }
            b->d_desc_bytes = b->exec.desc_bytes();
        }
        rc = b->exec.upload(b->d_desc, s);
        if (rc) return rc;
        b->key = key;
        b->built = true;
    }
    if (!use_graph) return b->exec.enqueue(s);
    if (!b->gexec) {
        // record on a private stream (the caller's may be the legacy null
        // stream, which cannot be captured), replay on the caller's stream
        if (!b->capture) TPT_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        TPT_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        int rc = b->exec.enqueue(b->capture);
        hipError_t e = hipStreamEndCapture(b->capture, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            return fail(TPT_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
    }
    TimedScope ts("batch_graph", s);
    TPT_HIP(hipGraphLaunch(b->gexec, s));
    return TPT_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: time every tile variant on the plan's own GEMM shapes and keep
// the fastest per (precision, pass, shape); likewise the Thomas kernel per
// (precision, line count, line length).
// ---------------------------------------------------------------------------
int tpt_autotune(int count, const tpt_plan* plans, void* stream) {
    if (count < 1 || !plans) return fail(TPT_ERR_INVALID, "bad autotune arguments");
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    TPT_HIP(hipEventCreate(&e0));
    TPT_HIP(hipEventCreate(&e1));
    std::vector<std::tuple<int, int, int, int, int>> done;
    int rc = TPT_OK;
    for (int pi = 0; pi < count && rc == TPT_OK; ++pi) {
        tpt_plan_s* p = plans[pi];
        if (!p || p->host_only) {
            rc = fail(TPT_ERR_INVALID, "bad plan for autotune");
            break;
        }
        const int prec = plan_gemm_prec(p);
        const size_t elem = prec == GP_F64 ? 8 : 4;
        const size_t bytes = (size_t)p->dof * elem + 256;
        void *in = nullptr, *outb = nullptr;
        if (hipMalloc(&in, bytes) != hipSuccess || hipMalloc(&outb, bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (in) (void)hipFree(in);
            rc = fail(TPT_ERR_OOM, "autotune buffers");
            break;
        }
        // non-zero operands (MFMA timing depends on the data): every 32-bit
        // word 0x3FF80000, i.e. 1.9375 in FP32 and about 1.5 in FP64
        (void)hipMemsetD32Async((hipDeviceptr_t)in, 0x3FF80000u, bytes / 4, s);
        for (int stage : {ST_XF, ST_YF}) {
            if (stage_is_fast(p, stage)) continue;  // no GEMM in this pass
            if (stage == ST_XF ? !p->tx : !p->ty) continue;  // explicit direction
            const int dt = prec == GP_F64 ? DT_F64 : DT_F32;
            GemmDesc g = stage_gemm(p, stage, prec, in, dt, outb, dt, EPI_STORE, nullptr, 1);
            const int kind = stage == ST_XF ? 0 : 1;
            auto key = std::make_tuple(prec, kind, kind == 0 ? 0 : g.M, g.N, g.K);
            if (std::find(done.begin(), done.end(), key) != done.end()) continue;
            done.push_back(key);
            int best = -1;
            float best_ms = 1e30f;
            for (int v = 0; v < TV_COUNT; ++v) {
                if (launch_gemm(g, prec, v, s) != hipSuccess) continue;  // warm-up
                float ms_min = 1e30f;
                for (int r = 0; r < 5; ++r) {
                    (void)hipEventRecord(e0, s);
                    (void)launch_gemm(g, prec, v, s);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ms_min = std::min(ms_min, ms);
                }
                if (ms_min < best_ms) {
                    best_ms = ms_min;
                    best = v;
                }
            }
            if (best >= 0) autotune_record(prec, kind, g.M, g.N, g.K, best);
        }
        // Thomas kernel: the sequential one and every partitioned
        // configuration that fits, on the plan's own lines (one system)
        if (!p->op[2].periodic && !p->seq_thomas) {
            const int dt = prec == GP_F64 ? DT_F64 : DT_F32;
            const long long lines = (long long)p->N[0] * p->N[1];
            auto key = std::make_tuple(prec, TUNE_THOMAS, (int)lines, p->N[2], 0);
            void* scratch = nullptr;
            const size_t sbytes = 8 * (size_t)thomas_scratch_doubles(p->N[0], p->N[1], p->N[2], 1, 0) + 256;
            if (std::find(done.begin(), done.end(), key) == done.end() && hipMalloc(&scratch, sbytes) == hipSuccess) {
                done.push_back(key);
                ThomasDesc t = plan_thomas(p, in, dt, outb, dt, (double*)scratch, 1);
                int best = -1;
                float best_ms = 1e30f;
                for (int v = THOMAS_SEQ; v < THOMAS_PART + THOMAS_NPART; ++v) {
                    t.variant = v;
                    if (thomas_variant(t) != v || launch_thomas(t, s) != hipSuccess) continue;  // warm-up
                    float ms_min = 1e30f;
                    for (int r = 0; r < 5; ++r) {
                        (void)hipEventRecord(e0, s);
                        (void)launch_thomas(t, s);
                        (void)hipEventRecord(e1, s);
                        (void)hipEventSynchronize(e1);
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, e0, e1);
                        ms_min = std::min(ms_min, ms);
                    }
                    if (ms_min < best_ms) {
                        best_ms = ms_min;
                        best = v;
                    }
                }
                if (best >= 0) autotune_record(prec, TUNE_THOMAS, (int)lines, p->N[2], 0, best);
                (void)hipStreamSynchronize(s);
                (void)hipFree(scratch);
            } else {
                (void)hipGetLastError();
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(in);
        (void)hipFree(outb);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
