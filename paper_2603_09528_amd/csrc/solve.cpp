// Solve sequencing (§2.2.2 solution steps 2.1–2.5 on one GPU, no transposes),
// mixed-precision refinement, GEMM tile selection and kernel timing.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <fstream>
#include <sstream>

#include "internal.h"

namespace tpt {

// ---- kernel timing ------------------------------------------------------------
namespace {
struct TimingRec {
    std::string name;
    hipEvent_t e0, e1;
};
std::mutex g_timing_mu;
bool g_timing = false;
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool timing_enabled() { return g_timing; }

LaunchEvents& launch_events() {
    static thread_local LaunchEvents le;
    return le;
}

// A timed scope wraps one kernel launch: it hands a pair of events to that
// launch (recorded at the kernel's start and end) and keeps the pair.
TimedScope::TimedScope(const char* n, hipStream_t st) : name(n), s(st) {
    if (!g_timing) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    e0 = get_event();
    e1 = get_event();
    if (!e0 || !e1) {
        if (e0) g_pool.push_back(e0);
        if (e1) g_pool.push_back(e1);
        return;
    }
    LaunchEvents& le = launch_events();
    le.start = e0;
    le.stop = e1;
    le.used = false;
    on = true;
}

TimedScope::~TimedScope() {
    if (!on) return;
    LaunchEvents& le = launch_events();
    const bool used = le.used;
    le.start = le.stop = nullptr;
    le.used = false;
    std::lock_guard<std::mutex> lock(g_timing_mu);
    if (used) {
        g_recs.push_back({name, e0, e1});
    } else {
        g_pool.push_back(e0);
        g_pool.push_back(e1);
    }
}

// ---- GEMM tile selection ---------------------------------------------------------
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;

std::string tune_key(int prec, int kind, int M, int N, int K) {
    // the x pass has M = N_y N_z rows (large): its tile choice depends on N, K only
    if (kind == 0) M = 0;
    std::ostringstream os;
    os << prec << ' ' << kind << ' ' << M << ' ' << N << ' ' << K;
    return os.str();
}
}  // namespace

void autotune_record(int prec, int kind, int M, int N, int K, int variant) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[tune_key(prec, kind, M, N, K)] = variant;
}

int tuned_thomas(int prec, long long lines, int nz) {
    if (lines > 0x7fffffffLL) return THOMAS_AUTO;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(tune_key(prec, TUNE_THOMAS, (int)lines, nz, 0));
    return it != g_tune.end() ? it->second : THOMAS_AUTO;
}

int choose_variant(int prec, int kind, int M, int N, int K) {
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune.find(tune_key(prec, kind, M, N, K));
        if (it != g_tune.end()) return it->second;
    }
    // heuristic: the persistent 128 x 128 tile (FP64 / FP32) where its edge
    // tiles waste at most a tenth of the work; else least padded area, then
    // the larger tile
    if (prec != GP_BF16X3 && K >= 16 &&
        std::ceil(M / 128.0) * std::ceil(N / 128.0) * 128.0 * 128.0 <= 1.1 * (double)M * N)
        return TV_128x128_P;
    int best = TV_128x128;
    double best_cost = 1e300;
    for (int v = 0; v <= TV_32x64; ++v) {
        int bm, bn;
        tile_variant_shape(v, &bm, &bn);
        const double pm = std::ceil((double)M / bm) * bm, pn = std::ceil((double)N / bn) * bn;
        const double waste = pm * pn / ((double)M * N);
        const double small = 1.0 + 0.08 * (128.0 * 128.0 / (bm * bn));  // smaller tiles reuse less
        const double cost = waste * small;
        if (cost < best_cost - 1e-12) {
            best_cost = cost;
            best = v;
        }
    }
    return best;
}

// ---- stage descriptors ---------------------------------------------------------------
GemmDesc stage_gemm(const tpt_plan_s* p, int stage, int prec, const void* in, int tin, void* out, int tout, int epi,
                    double* partials, int nrhs) {
    GemmDesc g{};
    const int nx = p->N[0], ny = p->N[1], nz = p->N[2];
    const DirBasis* b = (stage == ST_XF || stage == ST_XI) ? p->bx.get() : p->by.get();
    const bool fwd = stage == ST_XF || stage == ST_YF;
    const void* basis = nullptr;
    const uint16_t *bh = nullptr, *bl = nullptr;
    int tbasis = DT_F64;
    if (prec == GP_F64) {
        basis = fwd ? b->d_qinv : b->d_q;
    } else if (prec == GP_F32) {
        basis = fwd ? b->s_qinv : b->s_q;
        tbasis = DT_F32;
    } else {
        bh = fwd ? b->h_qinv : b->h_q;
        bl = fwd ? b->l_qinv : b->l_q;
        tbasis = DT_F32;
    }
    g.basis_hi = bh;
    g.basis_lo = bl;
    g.ldp = bh ? b->ldp : 0;
    g.epi = epi;
    g.partials = partials;
    g.tC = tout;
    if (stage == ST_XF || stage == ST_XI) {
        // C[m][p] = sum_i F[m][i] Qinv[p][i]  /  Phi[m][i] = sum_p S[m][p] Q[i][p]
        g.A = in;
        g.tA = tin;
        g.B = basis;
        g.tB = tbasis;
        g.basis_is_A = 0;
        g.b_nk = 1;
        g.M = ny * nz * nrhs;
        g.N = nx;
        g.K = nx;
        g.lda = nx;
        g.ldb = nx;
        g.ldc = nx;
        g.batch = 1;
    } else {
        // per z slab: C[q][p] = sum_j Qinv_y[q][j] S[j][p]  /  C[j][p] = sum_q Q_y[j][q] S[q][p]
        g.A = basis;
        g.tA = tbasis;
        g.B = in;
        g.tB = tin;
        g.basis_is_A = 1;
        g.b_nk = 0;
        g.M = ny;
        g.N = nx;
        g.K = ny;
        g.lda = ny;
        g.ldb = nx;
        g.ldc = nx;
        g.sA = 0;
        g.sB = (long long)nx * ny;
        g.sC = (long long)nx * ny;
        g.batch = nz * nrhs;
    }
    g.C = out;
    return g;
}

bool stage_is_fast(const tpt_plan_s* p, int stage) {
    return p->fast[(stage == ST_XF || stage == ST_XI) ? 0 : 1] >= 0;
}

FftDesc stage_fft(const tpt_plan_s* p, int stage, const void* in, int tin, void* out, int tout, int epi,
                  double* partials, int nrhs) {
    const bool xdir = stage == ST_XF || stage == ST_XI;
    const DirBasis* b = xdir ? p->bx.get() : p->by.get();
    const int nx = p->N[0], ny = p->N[1], nz = p->N[2];
    FftDesc f{};
    f.kind = p->fast[xdir ? 0 : 1];
    f.inverse = (stage == ST_XI || stage == ST_YI) ? 1 : 0;
    if (xdir) {
        f.n = nx;
        f.ylines = 0;
        f.lines = (long long)ny * nz * nrhs;
    } else {
        // the columns of every z slab: line (slab, i) starts at slab nx ny + i
        f.n = ny;
        f.ylines = 1;
        f.lines = (long long)nx * nz * nrhs;
        f.inner = nx;
        f.s_elem = nx;
        f.s_outer = (long long)nx * ny;
    }
    f.in = in;
    f.out = out;
    f.tin = tin;
    f.tout = tout;
    f.epi = epi;
    // forward Q^{-1} = sqrt(h) Q~^T, inverse Q = Q~ / sqrt(h) (uniform D = h I)
    f.scale = f.inverse ? 1.0 / std::sqrt(b->h) : std::sqrt(b->h);
    f.twiddle = b->d_twiddle;
    f.qtw = b->d_qtw;
    f.partials = partials;
    return f;
}

ThomasDesc plan_thomas(const tpt_plan_s* p, const void* f, int tf, void* x, int tx, double* scratch, int nrhs) {
    ThomasDesc t{};
    t.nx = p->N[0];
    t.ny = p->N[1];
    t.nz = p->N[2];
    t.nsys = nrhs;
    // an explicit direction adds no eigenvalue to the line shift
    t.lamx = p->tx ? p->bx->d_lam : p->buf.zeros;
    t.lamy = p->ty ? p->by->d_lam : p->buf.zeros;
    t.az = p->buf.az;
    t.bz = p->buf.bz;
    t.cz = p->buf.cz;
    t.sigma = p->sigma;
    t.tau = p->tau;
    t.pin_line = p->null_line;
    t.periodic = p->op[2].periodic ? 1 : 0;
    t.f = f;
    t.tf = tf;
    t.x = x;
    t.tx = tx;
    t.scratch = scratch;
    // the sequential kernel if asked for, else what the autotuner recorded
    // for these lines, else the automatic choice
    t.variant = p->seq_thomas ? THOMAS_SEQ : tuned_thomas(plan_gemm_prec(p), (long long)t.nx * t.ny * nrhs, t.nz);
    if (thomas_variant(t) < 0) t.variant = THOMAS_AUTO;
    return t;
}

StencilDesc plan_stencil(const tpt_plan_s* p, const double* x, const double* f, float* r, double* partials,
                         const double* stats) {
    StencilDesc st{};
    st.nx = p->N[0];
    st.ny = p->N[1];
    st.nz = p->N[2];
    // an explicit direction (implicit options yz, z) is not part of the
    // operator: zero coefficients
    const double* zx = p->buf.zeros;
    st.ax = p->tx ? p->buf.ax : zx; st.bx = p->tx ? p->buf.bx : zx; st.cx = p->tx ? p->buf.cx : zx;
    st.ay = p->ty ? p->buf.ay : zx; st.by = p->ty ? p->buf.by : zx; st.cy = p->ty ? p->buf.cy : zx;
    st.az = p->buf.az; st.bz = p->buf.bz; st.cz = p->buf.cz;
    st.perx = p->op[0].periodic ? 1 : 0;
    st.pery = p->op[1].periodic ? 1 : 0;
    st.perz = p->op[2].periodic ? 1 : 0;
    st.helmholtz = p->desc.kind == TPT_HELMHOLTZ ? 1 : 0;
    st.alpha = p->desc.alpha;
    st.x = x;
    st.f = f;
    st.r = r;
    st.partials = partials;
    // singular problems: the residual drops the incompatible part of f (the
    // constant on the last z plane that the pin of §3 absorbs, whose image in
    // modal space is the dropped last equation of the null line), so the
    // low-precision corrections see a compatible residual
    if (p->null_line >= 0 && stats) {
        st.wsum = stats + SS_WF;
        st.wscale = p->last_area_inv;
    }
    st.pair = residual_pairs_ok(st) ? 1 : 0;
    return st;
}

int stage_variant(const tpt_plan_s* p, int stage, const GemmDesc& g, int prec) {
    int v = p->gemm_variant[stage];
    if (v < 0) {
        const int kind = (stage == ST_XF || stage == ST_XI) ? 0 : 1;
        v = choose_variant(prec, kind, g.M, g.N, g.K);
    }
    // the persistent tile is FP64 / FP32 only
    if (tv_persistent(v) && prec == GP_BF16X3) v = TV_128x128;
    return v;
}

const char* stage_name(int stage, int prec) {
    static const char* n[3][4] = {
        {"gemm_x_fwd_f64", "gemm_y_fwd_f64", "gemm_y_inv_f64", "gemm_x_inv_f64"},
        {"gemm_x_fwd_f32", "gemm_y_fwd_f32", "gemm_y_inv_f32", "gemm_x_inv_f32"},
        {"gemm_x_fwd_bf16x3", "gemm_y_fwd_bf16x3", "gemm_y_inv_bf16x3", "gemm_x_inv_bf16x3"}};
    return n[prec][stage];
}

static int run_gemm(const tpt_plan_s* p, int stage, int prec, const void* in, int tin, void* out, int tout, int epi,
                    double* partials, int nrhs, hipStream_t s, long long* nblocks = nullptr) {
    GemmDesc g = stage_gemm(p, stage, prec, in, tin, out, tout, epi, partials, nrhs);
    const int v = stage_variant(p, stage, g, prec);
    if (nblocks) *nblocks = gemm_blocks(g, v);
    TimedScope ts(stage_name(stage, prec), s);
    hipError_t e = launch_gemm(g, prec, v, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("GEMM launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

static const char* fast_name(int stage, int tin, int tout) {
    static const char* n[4][2] = {{"fft_x_fwd_f64", "fft_x_fwd_f32io"},
                                  {"fft_y_fwd_f64", "fft_y_fwd_f32io"},
                                  {"fft_y_inv_f64", "fft_y_inv_f32io"},
                                  {"fft_x_inv_f64", "fft_x_inv_f32io"}};
    return n[stage][(tin == DT_F64 && tout == DT_F64) ? 0 : 1];
}

// One transform stage: the fast transform where the plan uses one for that
// direction, else the GEMM.  chk (x forward by fast transform only): the
// right-hand-side check fused into its loads.
static int run_stage(const tpt_plan_s* p, int stage, int prec, const void* in, int tin, void* out, int tout,
                     int epi, double* partials, int nrhs, hipStream_t s, long long* nblocks = nullptr,
                     const CheckDesc* chk = nullptr) {
    if (!stage_is_fast(p, stage)) return run_gemm(p, stage, prec, in, tin, out, tout, epi, partials, nrhs, s, nblocks);
    FftDesc f = stage_fft(p, stage, in, tin, out, tout, epi, partials, nrhs);
    if (chk) attach_check(p, *chk, f);
    const long long nb = fft_blocks(f);
    if (nblocks) *nblocks = nb;
    TimedScope ts(fast_name(stage, tin, tout), s);
    hipError_t e = launch_fft(f, nullptr, 0, nb, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("fast transform launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

static int run_thomas(const tpt_plan_s* p, const void* f, int tf, void* x, int tx, double* scratch, int nrhs,
                      hipStream_t s) {
    ThomasDesc t = plan_thomas(p, f, tf, x, tx, scratch, nrhs);
    TimedScope ts(tf == DT_F64 ? "thomas_f64" : "thomas_f32io", s);
    hipError_t e = launch_thomas(t, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("Thomas launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

// The right-hand-side check of a solve (weighted sums and non-finite count of
// every rhs, into the plan's stats; partials in the workspace's partial
// slots, which are free until the first refinement residual).
CheckDesc check_desc(const tpt_plan_s* p, const double* rhs, double* partials) {
    CheckDesc c{};
    c.nx = p->N[0];
    c.ny = p->N[1];
    c.nz = p->N[2];
    c.nsys = p->desc.nrhs;
    c.f = rhs;
    c.vx = p->buf.vx;
    c.vy = p->buf.vy;
    c.vz = p->buf.vz;
    c.vyz = p->buf.vyz;
    c.partials = partials;
    c.out = p->buf.norms + SS_WF;
    c.out_stride = TPT_STATS;
    return c;
}

// Whether the check rides in the loads of the x forward pass: x by fast
// transform on FP64 input, and no block of x lines spans two right-hand sides.
bool check_fused(const tpt_plan_s* p) {
    if (!p->run_check || !p->tx || !stage_is_fast(p, ST_XF) || p->fuse_xy) return false;
    const long long rows = (long long)p->N[1] * p->N[2];
    return rows * p->desc.nrhs < 0xffffffffLL && rows % fft_lines_per_block(p->N[0]) == 0;
}

long long check_fused_blocks(const tpt_plan_s* p) {
    return (long long)p->N[1] * p->N[2] / fft_lines_per_block(p->N[0]);
}

void attach_check(const tpt_plan_s* p, const CheckDesc& c, FftDesc& f) {
    f.cvx = c.vx;
    f.cvyz = c.vyz;
    f.cpart = c.partials;
    f.crows = (unsigned)((long long)p->N[1] * p->N[2]);
}

// Fold the partials the fused check wrote in the x forward pass.
static int finish_fused_check(const tpt_plan_s* p, const CheckDesc& c, hipStream_t s) {
    const long long nb = check_fused_blocks(p);
    TimedScope ts("check_reduce", s);
    hipError_t e = launch_check_reduce(c, nb, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("check launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

static int run_check(const tpt_plan_s* p, const double* rhs, double* partials, hipStream_t s) {
    if (!p->run_check || check_fused(p)) return TPT_OK;
    const CheckDesc c = check_desc(p, rhs, partials);
    TimedScope ts("check", s);
    hipError_t e = launch_check(c, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("check launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

// sqrt(a / b) of two sums of squares: 0 when both vanish, NaN when either is
// not finite
static double ratio(double a, double b) {
    if (!std::isfinite(a) || !std::isfinite(b)) return NAN;
    if (b > 0) return std::sqrt(a / b);
    return a > 0 ? INFINITY : 0.0;
}

// Info fields from the reduced per-rhs sums h (TPT_STATS doubles per rhs):
// the refinement norms when `norms`, the check fields when the plan checks.
void stats_to_info(const tpt_plan_s* p, const double* h, bool norms, tpt_info* info) {
    const int R = p->desc.nrhs;
    if (norms) {
        double rc = 0.0, rr = 0.0;
        for (int r = 0; r < R; ++r) {
            const double* q = h + (size_t)TPT_STATS * r;
            const double c = ratio(q[SS_E2], q[SS_X2]);
            const double e = ratio(q[SS_R2], q[SS_F2]);
            rc = (c == c && rc == rc) ? std::max(rc, c) : NAN;
            rr = (e == e && rr == rr) ? std::max(rr, e) : NAN;
        }
        info->rel_correction = rc;
        info->rel_residual = rr;
    }
    if (p->check) {
        double defect = 0.0, bad = 0.0;
        for (int r = 0; r < R; ++r) {
            const double* q = h + (size_t)TPT_STATS * r;
            bad += q[SS_BAD];
            if (p->null_line >= 0 && q[SS_WABS] > 0) defect = std::max(defect, std::fabs(q[SS_WF]) / q[SS_WABS]);
        }
        info->compat_defect = defect;
        info->nonfinite = bad > 2147483647.0 ? 2147483647 : (int)bad;
    }
}

static void info_from_stats(tpt_plan_s* p, const double* h, bool norms) { stats_to_info(p, h, norms, &p->info); }

static inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

Ws carve(const tpt_plan_s* p, void* ws) {
    Ws w{};
    w.base = (char*)ws;
    w.n = (size_t)p->dof * p->desc.nrhs;
    const size_t n = w.n;
    size_t o = 0;
    const size_t tsc = 8 * (size_t)thomas_scratch_doubles(p->N[0], p->N[1], p->N[2], p->desc.nrhs, p->op[2].periodic ? 1 : 0);
    if (p->desc.precision == TPT_FP64) {
        w.w1 = w.base + o; o += al256(8 * n);
        w.w2 = w.base + o; o += al256(8 * n);
        w.scratch = (double*)(w.base + o); o += al256(tsc);
        w.r = nullptr;
    } else {
        w.scratch = (double*)(w.base + o); o += al256(tsc);
        w.w1 = w.base + o; o += al256(4 * n);
        w.w2 = w.base + o; o += al256(4 * n);
        w.r = (float*)(w.base + o); o += al256(4 * n);
    }
    w.partials = (double*)(w.base + o);
    return w;
}

long long plan_residual_blocks(const tpt_plan_s* p) {
    StencilDesc st = plan_stencil(p, nullptr, nullptr, nullptr, nullptr, nullptr);
    st.pair = 0;  // the larger count: the paired form may not apply to the caller's buffers
    return residual_blocks(st);
}

// Fused x transform + y GEMM (FP64): forward rhs -> w2 (2.1 + 2.2), inverse
// w2 -> out (2.5 + 2.4: the x inverse is applied first, in the loads).
// Returns 1 when the operands do not fit the fused kernel (the caller runs
// the separate passes).
static int run_fused(const tpt_plan_s* p, bool inverse, const double* in, double* out, int nrhs, hipStream_t s) {
    const GemmDesc g = stage_gemm(p, inverse ? ST_YI : ST_YF, GP_F64, in, DT_F64, out, DT_F64, EPI_STORE, nullptr, nrhs);
    const FftDesc xf = stage_fft(p, inverse ? ST_XI : ST_XF, nullptr, DT_F64, nullptr, DT_F64, EPI_STORE, nullptr, nrhs);
    if (!xgemm_supported(g, xf)) return 1;
    TimedScope ts(inverse ? "xgemm_inv_f64" : "xgemm_fwd_f64", s);
    hipError_t e = launch_xgemm(g, xf, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("fused transform launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

// FP64 path: 2.1 x forward, 2.2 y forward, 2.3 Thomas, 2.4 y inverse, 2.5 x inverse.
static int solve_fp64(tpt_plan_s* p, const double* rhs, double* out, const Ws& w, hipStream_t s) {
    const int R = p->desc.nrhs;
    int rc;
    if ((rc = run_check(p, rhs, w.partials, s))) return rc;
    p->info_on_device = p->check;
    p->info.iters = 0;
    p->info.rel_correction = 0.0;
    p->info.rel_residual = -1.0;
    if (!p->tx) {
        // x explicit: y forward, Thomas, y inverse (yz); Thomas alone (z)
        if (!p->ty) return run_thomas(p, rhs, DT_F64, out, DT_F64, w.scratch, R, s);
        if ((rc = run_stage(p, ST_YF, GP_F64, rhs, DT_F64, w.w2, DT_F64, EPI_STORE, nullptr, R, s))) return rc;
        if ((rc = run_thomas(p, w.w2, DT_F64, w.w2, DT_F64, w.scratch, R, s))) return rc;
        return run_stage(p, ST_YI, GP_F64, w.w2, DT_F64, out, DT_F64, EPI_STORE, nullptr, R, s);
    }
    if (p->fuse_xy && (rc = run_fused(p, false, rhs, (double*)w.w2, R, s)) <= 0) {
        if (rc) return rc;
        if ((rc = run_thomas(p, w.w2, DT_F64, w.w2, DT_F64, w.scratch, R, s))) return rc;
        if ((rc = run_fused(p, true, (const double*)w.w2, out, R, s)) < 0) return rc;
        if (rc == 0) {
            p->info.iters = 0;
            p->info.rel_correction = 0.0;
            p->info.rel_residual = -1.0;
            return TPT_OK;
        }
        // output not aligned for the fused kernel: separate passes for the inverse
        if ((rc = run_stage(p, ST_YI, GP_F64, w.w2, DT_F64, w.w1, DT_F64, EPI_STORE, nullptr, R, s))) return rc;
        if ((rc = run_stage(p, ST_XI, GP_F64, w.w1, DT_F64, out, DT_F64, EPI_STORE, nullptr, R, s))) return rc;
        p->info.iters = 0;
        p->info.rel_correction = 0.0;
        p->info.rel_residual = -1.0;
        return TPT_OK;
    }
    const bool fchk = check_fused(p);
    const CheckDesc chk = check_desc(p, rhs, w.partials);
    if ((rc = run_stage(p, ST_XF, GP_F64, rhs, DT_F64, w.w1, DT_F64, EPI_STORE, nullptr, R, s, nullptr,
                        fchk ? &chk : nullptr)))
        return rc;
    if (fchk && (rc = finish_fused_check(p, chk, s))) return rc;
    if ((rc = run_stage(p, ST_YF, GP_F64, w.w1, DT_F64, w.w2, DT_F64, EPI_STORE, nullptr, R, s))) return rc;
    if ((rc = run_thomas(p, w.w2, DT_F64, w.w2, DT_F64, w.scratch, R, s))) return rc;
    if ((rc = run_stage(p, ST_YI, GP_F64, w.w2, DT_F64, w.w1, DT_F64, EPI_STORE, nullptr, R, s))) return rc;
    if ((rc = run_stage(p, ST_XI, GP_F64, w.w1, DT_F64, out, DT_F64, EPI_STORE, nullptr, R, s))) return rc;
    p->info.iters = 0;
    p->info.rel_correction = 0.0;
    p->info.rel_residual = -1.0;
    return TPT_OK;
}

// Low-precision application of M^{-1} to `in` (FP64 rhs or FP32 residual):
// result stored into out (epi STORE) or added to out (epi ACCUM).  An
// accumulating application runs its last pass once per right-hand side, so
// that the norm partials of the correction and the updated iterate of each
// rhs are reduced into that rhs's stats.
static int apply_minv(tpt_plan_s* p, int prec, const void* in, int tin, double* out, int epi, const Ws& w,
                      hipStream_t s) {
    const int R = p->desc.nrhs;
    int rc;
    // the first application reads the rhs: its check may ride in the x pass
    const bool fchk = tin == DT_F64 && check_fused(p);
    const CheckDesc chk = check_desc(p, (const double*)in, w.partials);
    if ((rc = run_stage(p, ST_XF, prec, in, tin, w.w1, DT_F32, EPI_STORE, nullptr, R, s, nullptr,
                        fchk ? &chk : nullptr)))
        return rc;
    if (fchk && (rc = finish_fused_check(p, chk, s))) return rc;
    if ((rc = run_stage(p, ST_YF, prec, w.w1, DT_F32, w.w2, DT_F32, EPI_STORE, nullptr, R, s))) return rc;
    if ((rc = run_thomas(p, w.w2, DT_F32, w.w2, DT_F32, w.scratch, R, s))) return rc;
    if ((rc = run_stage(p, ST_YI, prec, w.w2, DT_F32, w.w1, DT_F32, EPI_STORE, nullptr, R, s))) return rc;
    if (epi != EPI_ACCUM_F64)
        return run_stage(p, ST_XI, prec, w.w1, DT_F32, out, DT_F64, epi, nullptr, R, s);
    for (int r = 0; r < R; ++r) {
        const size_t off = (size_t)r * p->dof;
        long long nb = 0;
        if ((rc = run_stage(p, ST_XI, prec, (const float*)w.w1 + off, DT_F32, out + off, DT_F64, epi, w.partials, 1,
                            s, &nb)))
            return rc;
        TimedScope ts("reduce", s);
        hipError_t e = launch_reduce_pairs(w.partials, (int)nb, p->buf.norms + (size_t)TPT_STATS * r + SS_E2, s);
        if (e != hipSuccess) return fail(TPT_ERR_HIP, hipGetErrorString(e));
    }
    return TPT_OK;
}

// Mixed path: x0 = M^{-1} f; then repeat r = f - A x (FP64), x += M^{-1} r.
// Adaptive stop (per rhs, all must pass): c_k = ||e_k|| / ||x_k|| is the
// size of correction k, i.e. about the error left by iterate k-1, so
// c_k <= rtol meets the target; from the second correction on, the observed
// contraction rho = c_k / c_{k-1} < 1 bounds the error after x_k by the
// geometric tail c_k rho / (1 - rho).  The first correction alone gives no
// rate, so it stops only on c_1 <= rtol.
static int solve_mixed(tpt_plan_s* p, const double* rhs, double* out, const Ws& w, hipStream_t s) {
    const int prec = plan_gemm_prec(p);
    const int R = p->desc.nrhs;
    int rc;
    if ((rc = run_check(p, rhs, w.partials, s))) return rc;
    if ((rc = apply_minv(p, prec, rhs, DT_F64, out, EPI_STORE, w, s))) return rc;
    const bool adaptive = p->desc.fixed_refine < 0;
    const int max_it = adaptive ? p->desc.max_refine : p->desc.fixed_refine;
    double* dn = p->buf.norms;
    std::vector<double> prev(R, -1.0);
    int it = 0;
    double est = 1.0;
    for (it = 0; it < max_it;) {
        // residual of every rhs and its norms
        for (int r = 0; r < R; ++r) {
            StencilDesc st = plan_stencil(p, out + (size_t)r * p->dof, rhs + (size_t)r * p->dof,
                                          w.r + (size_t)r * p->dof, w.partials, dn + (size_t)TPT_STATS * r);
            {
                TimedScope ts("residual_f64", s);
                hipError_t e = launch_residual(st, s);
                if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("residual launch: ") + hipGetErrorString(e));
            }
            TimedScope ts("reduce", s);
            hipError_t e = launch_reduce_pairs(w.partials, residual_blocks(st), dn + (size_t)TPT_STATS * r + SS_R2, s);
            if (e != hipSuccess) return fail(TPT_ERR_HIP, hipGetErrorString(e));
        }
        if ((rc = apply_minv(p, prec, w.r, DT_F32, out, EPI_ACCUM_F64, w, s))) return rc;
        ++it;
        if (adaptive) {
            const size_t nst = (size_t)TPT_STATS * R;
            TPT_HIP(hipMemcpyAsync(p->h_norms, dn, nst * sizeof(double), hipMemcpyDeviceToHost, s));
            TPT_HIP(hipStreamSynchronize(s));
            const double* h = p->h_norms;
            info_from_stats(p, h, true);
            est = 0.0;
            for (int r = 0; r < R; ++r) {
                const double* q = h + (size_t)TPT_STATS * r;
                const double c = ratio(q[SS_E2], q[SS_X2]);
                if (!std::isfinite(c) || (p->check && p->info.nonfinite > 0)) {
                    p->info.iters = it;
                    return fail(TPT_ERR_NOT_CONVERGED,
                                p->check && p->info.nonfinite > 0
                                    ? "right-hand side holds " + std::to_string(p->info.nonfinite) + " non-finite values"
                                    : std::string("non-finite correction"));
                }
                double est_r = c;
                if (c > p->desc.rtol && prev[r] > 0.0) {
                    const double rho = c / prev[r];
                    if (rho < 1.0) est_r = c * rho / (1.0 - rho);
                }
                prev[r] = c;
                est = std::max(est, est_r);
            }
            if (est <= p->desc.rtol) break;
        }
    }
    p->info.iters = it;
    if (!adaptive) {
        // norms and check results are read back lazily by tpt_solve_info
        p->info.rel_correction = it > 0 ? -2.0 : 0.0;
        p->info.rel_residual = -1.0;
        p->info_on_device = it > 0 || p->check;
    } else {
        if (it == 0) {
            p->info.rel_correction = 0.0;
            p->info.rel_residual = -1.0;
            p->info_on_device = p->check;
        } else {
            p->info_on_device = false;
        }
        if (it > 0 && est > p->desc.rtol && it >= max_it)
            return fail(TPT_ERR_NOT_CONVERGED, "refinement stopped with estimated error " + std::to_string(est));
    }
    return TPT_OK;
}

int solve_one(tpt_plan_s* p, const double* rhs, double* out, void* ws, size_t ws_bytes, hipStream_t s) {
    if (p->host_only) return fail(TPT_ERR_INVALID, "host-only plan cannot solve");
    if (!rhs || !out) return fail(TPT_ERR_INVALID, "NULL rhs or out");
    const size_t bytes = (size_t)p->dof * p->desc.nrhs * sizeof(double);
    const char* a0 = (const char*)rhs;
    const char* b0 = (const char*)out;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return fail(TPT_ERR_ALIAS, "rhs and out overlap");
    const size_t need = plan_workspace_bytes(p);
    if (!ws) {
        if (p->own_ws_bytes < need) {
            if (p->own_ws) TPT_HIP(hipFree(p->own_ws));
            p->own_ws = nullptr;
            p->own_ws_bytes = 0;
            if (hipMalloc(&p->own_ws, need) != hipSuccess) {
                (void)hipGetLastError();
                return fail(TPT_ERR_OOM, "cannot allocate the plan workspace");
            }
            p->own_ws_bytes = need;
        }
        ws = p->own_ws;
        ws_bytes = p->own_ws_bytes;
    }
    if (ws_bytes < need) return fail(TPT_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need));
    Ws w = carve(p, ws);
    if (p->desc.precision == TPT_FP64) return solve_fp64(p, rhs, out, w, s);
    return solve_mixed(p, rhs, out, w, s);
}

}  // namespace tpt

using namespace tpt;

extern "C" {

int tpt_solve(tpt_plan plan, const double* rhs, double* out, void* workspace, size_t workspace_bytes, void* stream) {
    if (!plan) return fail(TPT_ERR_INVALID, "NULL plan");
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) TPT_HIP(hipSetDevice(plan->device));
    return solve_one(plan, rhs, out, workspace, workspace_bytes, (hipStream_t)stream);
}

int tpt_residual(tpt_plan plan, const double* x, const double* f, float* r, void* stream) {
    if (!plan) return fail(TPT_ERR_INVALID, "NULL plan");
    if (plan->host_only) return fail(TPT_ERR_INVALID, "host-only plan has no device operator");
    if (!x || !f || !r) return fail(TPT_ERR_INVALID, "NULL array");
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) TPT_HIP(hipSetDevice(plan->device));
    for (int q = 0; q < plan->desc.nrhs; ++q) {
        const size_t o = (size_t)q * plan->dof;
        StencilDesc st = plan_stencil(plan, x + o, f + o, r + o, nullptr, nullptr);
        hipError_t e = launch_residual(st, (hipStream_t)stream);
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("residual launch: ") + hipGetErrorString(e));
    }
    return TPT_OK;
}

int tpt_solve_info(tpt_plan plan, tpt_info* info) {
    if (!plan || !info) return fail(TPT_ERR_INVALID, "NULL argument");
    if (plan->info_on_device) {
        // fixed-refinement norms and the check sums of the last solve are on the device
        std::vector<double> h((size_t)TPT_STATS * plan->desc.nrhs);
        TPT_HIP(hipMemcpy(h.data(), plan->buf.norms, h.size() * sizeof(double), hipMemcpyDeviceToHost));
        info_from_stats(plan, h.data(), plan->info.rel_correction == -2.0);
        plan->info_on_device = false;
    }
    *info = plan->info;
    return TPT_OK;
}

int tpt_thomas(int nx, int ny, int nz, int nsys, const double* lamx, const double* lamy, const double* az,
               const double* bz, const double* cz, int periodic_z, double sigma, double tau, int pin_line,
               const double* f, double* x, double* scratch, int variant, void* stream) {
    if (nx < 1 || ny < 1 || nz < 1 || nsys < 1) return fail(TPT_ERR_INVALID, "bad sizes");
    if (variant < -1 || variant > THOMAS_NPART) return fail(TPT_ERR_INVALID, "bad Thomas variant");
    if (periodic_z && nz < 2) return fail(TPT_ERR_INVALID, "cyclic lines need nz >= 2");
    if (!lamx || !lamy || !az || !bz || !cz || !f || !x || !scratch) return fail(TPT_ERR_INVALID, "NULL pointer");
    if (pin_line >= nx * ny) return fail(TPT_ERR_INVALID, "pin_line out of range");
    ThomasDesc t{};
    t.nx = nx; t.ny = ny; t.nz = nz; t.nsys = nsys;
    t.lamx = lamx; t.lamy = lamy; t.az = az; t.bz = bz; t.cz = cz;
    t.sigma = sigma; t.tau = tau; t.pin_line = pin_line; t.periodic = periodic_z ? 1 : 0;
    t.f = f; t.tf = DT_F64; t.x = x; t.tx = DT_F64; t.scratch = scratch;
    t.variant = variant < 0 ? THOMAS_AUTO : variant == 0 ? THOMAS_SEQ : THOMAS_PART + variant - 1;
    if (thomas_variant(t) < 0)
        return fail(TPT_ERR_INVALID, "Thomas variant does not fit (cyclic lines, or P*L < nz)");
    TimedScope ts("thomas_f64", (hipStream_t)stream);
    hipError_t e = launch_thomas(t, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, hipGetErrorString(e));
    return TPT_OK;
}

int tpt_gemm(int prec, int b_nk, int variant, int M, int N, int K, int batch, const void* A, long long strideA,
             const void* B, long long strideB, void* C, long long strideC, void* stream) {
    if (M < 1 || N < 1 || K < 1 || batch < 1 || !A || !B || !C) return fail(TPT_ERR_INVALID, "bad GEMM arguments");
    if (prec < TPT_FP64 || prec > TPT_MIXED_BF16X3) return fail(TPT_ERR_INVALID, "bad precision");
    if (variant < -1 || variant >= TV_COUNT) return fail(TPT_ERR_INVALID, "bad tile variant");
    hipStream_t s = (hipStream_t)stream;
    GemmDesc g{};
    g.A = A; g.B = B; g.C = C;
    g.M = M; g.N = N; g.K = K;
    g.lda = K; g.ldb = b_nk ? K : N; g.ldc = N;
    g.sA = strideA; g.sB = strideB; g.sC = strideC; g.batch = batch;
    g.b_nk = b_nk ? 1 : 0;
    const int t = prec == TPT_FP64 ? DT_F64 : DT_F32;
    g.tA = g.tB = g.tC = t;
    g.epi = EPI_STORE;
    const int gp = prec == TPT_FP64 ? GP_F64 : (prec == TPT_MIXED_FP32 ? GP_F32 : GP_BF16X3);
    void* planes = nullptr;
    if (gp == GP_BF16X3) {
        // split the basis-side operand into bf16 planes
        const void* src = b_nk ? B : A;
        const long long stride = b_nk ? strideB : strideA;
        const long long one = b_nk ? (long long)N * K : (long long)M * K;
        const long long na = stride ? stride * (batch - 1) + one : one;
        if (hipMalloc(&planes, 2 * sizeof(uint16_t) * na) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TPT_ERR_OOM, "GEMM planes");
        }
        uint16_t* hi = (uint16_t*)planes;
        uint16_t* lo = hi + na;
        hipError_t e = launch_split_bf16((const float*)src, hi, lo, na, s);
        if (e != hipSuccess) {
            (void)hipFree(planes);
            return fail(TPT_ERR_HIP, hipGetErrorString(e));
        }
        g.basis_hi = hi;
        g.basis_lo = lo;
        g.basis_is_A = b_nk ? 0 : 1;
    }
    int v = variant >= 0 ? variant : choose_variant(gp, b_nk ? 0 : 1, M, N, K);
    if (variant < 0 && tv_persistent(v) && gp == GP_BF16X3) v = TV_128x128;
    hipError_t e;
    {
        TimedScope ts("gemm_test", s);
        e = launch_gemm(g, gp, v, s);
    }
    if (planes) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(planes);
    }
    if (e != hipSuccess) return fail(TPT_ERR_HIP, hipGetErrorString(e));
    return TPT_OK;
}

int tpt_timing_enable(int enable) {
    std::lock_guard<std::mutex> lock(g_timing_mu);
    g_timing = enable != 0;
    return TPT_OK;
}

int tpt_timing_collect(int* count, char* names, size_t names_len, double* total_ms, long long* launches) {
    if (!count) return fail(TPT_ERR_INVALID, "NULL count");
    std::lock_guard<std::mutex> lock(g_timing_mu);
    std::vector<std::string> kinds;
    std::vector<double> ms;
    std::vector<long long> cnt;
    for (auto& r : g_recs) {
        if (hipEventSynchronize(r.e1) != hipSuccess) return fail(TPT_ERR_HIP, "event sync failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) t = 0.f;
        size_t k = 0;
        for (; k < kinds.size(); ++k)
            if (kinds[k] == r.name) break;
        if (k == kinds.size()) {
            kinds.push_back(r.name);
            ms.push_back(0.0);
            cnt.push_back(0);
        }
        ms[k] += t;
        cnt[k] += 1;
        g_pool.push_back(r.e0);
        g_pool.push_back(r.e1);
    }
    g_recs.clear();
    const int cap = *count;
    size_t pos = 0;
    for (int k = 0; k < (int)kinds.size() && k < cap; ++k) {
        if (total_ms) total_ms[k] = ms[k];
        if (launches) launches[k] = cnt[k];
        if (names && pos + kinds[k].size() + 1 <= names_len) {
            std::memcpy(names + pos, kinds[k].c_str(), kinds[k].size() + 1);
            pos += kinds[k].size() + 1;
        }
    }
    *count = (int)kinds.size();
    return TPT_OK;
}

int tpt_autotune_save(const char* path) {
    if (!path) return fail(TPT_ERR_INVALID, "NULL path");
    std::lock_guard<std::mutex> lock(g_tune_mu);
    std::ofstream f(path);
    if (!f) return fail(TPT_ERR_INVALID, "cannot open " + std::string(path));
    f << "# prec kind M N K variant\n";
    for (auto& kv : g_tune) f << kv.first << ' ' << kv.second << '\n';
    return TPT_OK;
}

int tpt_autotune_load(const char* path) {
    if (!path) return fail(TPT_ERR_INVALID, "NULL path");
    std::ifstream f(path);
    if (!f) return fail(TPT_ERR_INVALID, "cannot open " + std::string(path));
    std::string line;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    while (std::getline(f, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        int prec, kind, M, N, K, v;
        if (!(is >> prec >> kind >> M >> N >> K >> v)) continue;
        if (prec < GP_F64 || prec > GP_BF16X3 || kind < 0 || kind > TUNE_THOMAS) continue;
        if (kind == TUNE_THOMAS ? (v < THOMAS_SEQ || v >= THOMAS_PART + THOMAS_NPART) : (v < 0 || v >= TV_COUNT))
            continue;
        g_tune[tune_key(prec, kind, M, N, K)] = v;
    }
    return TPT_OK;
}

}  // extern "C"
