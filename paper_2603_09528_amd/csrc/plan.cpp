// Plans: initialization steps 1.1–1.3 of the three-dimensional procedure
// (§2.2.2) — 1-D operators, eigenbases of x and y, device copies — and the
// device-resident eigenbasis cache shared by plans with the same grid.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace tpt {

// ---- errors -----------------------------------------------------------------
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}
const char* last_error_cstr() { return g_last_error.c_str(); }

// ---- bf16 rounding on the host (round to nearest even) ----------------------
static uint16_t host_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static float host_bf16_to_f(uint16_t h) {
    uint32_t u = ((uint32_t)h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

DirBasis::~DirBasis() {
    if (block) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        (void)hipFree(block);
        (void)hipSetDevice(cur);
    }
}

// ---- eigenbasis cache ---------------------------------------------------------
static std::mutex g_cache_mu;
static std::map<std::string, std::weak_ptr<DirBasis>> g_cache;

static std::string cache_key(int device, int ncells, const double* faces, int bc_lo, int bc_hi, int loc,
                             bool host_only) {
    std::string k;
    k.reserve(32 + 8 * (ncells + 1));
    int hdr[6] = {device, ncells, bc_lo, bc_hi, loc, host_only ? 1 : 0};
    k.append((const char*)hdr, sizeof(hdr));
    k.append((const char*)faces, sizeof(double) * (ncells + 1));
    return k;
}

std::shared_ptr<DirBasis> basis_cache_get(int ncells, const double* faces, int bc_lo, int bc_hi, int loc,
                                          bool host_only, std::string& err) {
    int device = 0;
    if (!host_only) {
        if (hipGetDevice(&device) != hipSuccess) {
            err = "hipGetDevice failed";
            return nullptr;
        }
    }
    const std::string key = cache_key(device, ncells, faces, bc_lo, bc_hi, loc, host_only);
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
        if (auto sp = it->second.lock()) return sp;
    }
    Op1D op;
    err = build_op1d(ncells, faces, bc_lo, bc_hi, loc, op);
    if (!err.empty()) return nullptr;
    auto b = std::make_shared<DirBasis>();
    b->device = device;
    b->n = op.n;
    err = eig_op1d(op, b->eig);
    if (!err.empty()) return nullptr;
    if (!host_only) {
        const int n = op.n;
        const size_t nn = (size_t)n * n;
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t o_lam = 0;
        const size_t o_qinv = o_lam + al(8 * (size_t)n);
        const size_t o_q = o_qinv + al(8 * nn);
        const size_t o_sqinv = o_q + al(8 * nn);
        const size_t o_sq = o_sqinv + al(4 * nn);
        // bf16 planes: rows padded to a multiple of 8 elements (16 bytes), so
        // the split-BF16 tiles load them as vectors whatever n is
        const int ldp = (n + 7) / 8 * 8;
        const size_t np = (size_t)n * ldp;
        const size_t o_hqinv = o_sq + al(4 * nn);
        const size_t o_lqinv = o_hqinv + al(2 * np);
        const size_t o_hq = o_lqinv + al(2 * np);
        const size_t o_lq = o_hq + al(2 * np);
        int fk = -1;
        if (b->eig.analytic && fft_supported(n)) {
            if (op.periodic) fk = UT_FOURIER;
            else if (op.loc == LOC_C && op.bc_lo == BC_N && op.bc_hi == BC_N) fk = UT_DCT;
            else if (op.loc == LOC_C && op.bc_lo == BC_D && op.bc_hi == BC_D) fk = UT_DST;
        }
        const bool fft = fk >= 0;
        const size_t o_tw = o_lq + al(2 * np);
        const size_t o_qtw = o_tw + (fft ? al(16 * (size_t)(n / 2)) : 0);
        const size_t total = o_qtw + (fft ? al(16 * (size_t)(n / 2 + 1)) : 0);
        std::vector<char> host(total, 0);
        double* lam = (double*)(host.data() + o_lam);
        double* qinv = (double*)(host.data() + o_qinv);
        double* q = (double*)(host.data() + o_q);
        float* sqinv = (float*)(host.data() + o_sqinv);
        float* sq = (float*)(host.data() + o_sq);
        uint16_t* hqinv = (uint16_t*)(host.data() + o_hqinv);
        uint16_t* lqinv = (uint16_t*)(host.data() + o_lqinv);
        uint16_t* hq = (uint16_t*)(host.data() + o_hq);
        uint16_t* lq = (uint16_t*)(host.data() + o_lq);
        for (int p = 0; p < n; ++p) lam[p] = b->eig.lam[p];
        for (int i = 0; i < n; ++i) {
            const double si = std::sqrt(op.vol[i]);
            for (int p = 0; p < n; ++p) {
                const double qt = b->eig.Qt[(size_t)i * n + p];
                qinv[(size_t)p * n + i] = qt * si;  // Q^{-1} = Q~^T D^{1/2}
                q[(size_t)i * n + p] = qt / si;     // Q = D^{-1/2} Q~
            }
        }
        if (fft) {
            // twiddles of the length-n real transform and the quarter-wave
            // factors of the cosine / sine transforms, in long double
            double* tw = (double*)(host.data() + o_tw);
            double* qw = (double*)(host.data() + o_qtw);
            const long double pi = 3.14159265358979323846264338327950288L;
            for (int k = 0; k < n / 2; ++k) {
                const long double a = 2.0L * pi * (long double)k / (long double)n;
                tw[2 * k] = (double)std::cos(a);
                tw[2 * k + 1] = (double)-std::sin(a);
            }
            for (int k = 0; k <= n / 2; ++k) {
                const long double a = pi * (long double)k / (2.0L * n);
                qw[2 * k] = (double)std::cos(a);
                qw[2 * k + 1] = (double)-std::sin(a);
            }
        }
        b->fast_kind = fk;
        b->h = op.vol[0];
        for (size_t e = 0; e < nn; ++e) {
            sqinv[e] = (float)qinv[e];
            sq[e] = (float)q[e];
            const size_t ep = e / n * ldp + e % n;  // padded position (padding stays 0)
            uint16_t h = host_bf16((float)qinv[e]);
            hqinv[ep] = h;
            lqinv[ep] = host_bf16((float)(qinv[e] - (double)host_bf16_to_f(h)));
            h = host_bf16((float)q[e]);
            hq[ep] = h;
            lq[ep] = host_bf16((float)(q[e] - (double)host_bf16_to_f(h)));
        }
        b->ldp = ldp;
        void* blk = nullptr;
        if (hipMalloc(&blk, total) != hipSuccess) {
            err = "out of device memory for an eigenbasis";
            (void)hipGetLastError();
            return nullptr;
        }
        if (hipMemcpy(blk, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(blk);
            err = "hipMemcpy of an eigenbasis failed";
            return nullptr;
        }
        char* d = (char*)blk;
        b->block = blk;
        b->bytes = total;
        b->d_lam = (double*)(d + o_lam);
        b->d_qinv = (double*)(d + o_qinv);
        b->d_q = (double*)(d + o_q);
        b->s_qinv = (float*)(d + o_sqinv);
        b->s_q = (float*)(d + o_sq);
        b->h_qinv = (uint16_t*)(d + o_hqinv);
        b->l_qinv = (uint16_t*)(d + o_lqinv);
        b->h_q = (uint16_t*)(d + o_hq);
        b->l_q = (uint16_t*)(d + o_lq);
        if (fft) {
            b->d_twiddle = (double2*)(d + o_tw);
            b->d_qtw = (double2*)(d + o_qtw);
        }
    }
    g_cache[key] = b;
    return b;
}

size_t basis_cache_bytes() {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    size_t s = 0;
    for (auto& kv : g_cache)
        if (auto sp = kv.second.lock()) s += sp->bytes;
    return s;
}

int plan_gemm_prec(const tpt_plan_s* p) {
    switch (p->desc.precision) {
        case TPT_MIXED_FP32: return GP_F32;
        case TPT_MIXED_BF16X3: return GP_BF16X3;
        default: return GP_F64;
    }
}

// Bytes per unknown of the workspace: two transform buffers and the Thomas
// scratch (c', d' in FP64).  Mixed modes use FP32 transform buffers plus an
// FP32 residual; the tail holds partial sums.
static size_t partial_slots(const tpt_plan_s* p) {
    const long long dof = p->dof * p->desc.nrhs;
    // enough for the residual blocks of all rhs and for the x-inverse GEMM
    // blocks of the smallest tile (32 x 64)
    long long res = 0;
    for (int r = 0; r < p->desc.nrhs; ++r) res += (p->dof + 255) / 256;
    long long xi = ((long long)p->N[1] * p->N[2] * p->desc.nrhs + 31) / 32 * ((p->N[0] + 63) / 64);
    // the x-inverse fast transform: at most one block per x line
    const long long fx = (long long)p->N[1] * p->N[2] * p->desc.nrhs;
    // the right-hand-side check: 4 doubles (two slots) per block
    CheckDesc c{};
    c.nx = p->N[0];
    c.ny = p->N[1];
    c.nz = p->N[2];
    long long chk = 2 * check_blocks(c) * p->desc.nrhs;
    if (fft_supported(p->N[0])) chk = std::max(chk, 2 * check_fused_blocks(p) * p->desc.nrhs);
    (void)dof;
    return (size_t)std::max(std::max(std::max(res, xi), fx), chk) + 8;
}

size_t plan_workspace_bytes(const tpt_plan_s* p) {
    const size_t n = (size_t)p->dof * p->desc.nrhs;
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t tsc = 8 * (size_t)thomas_scratch_doubles(p->N[0], p->N[1], p->N[2], p->desc.nrhs, p->op[2].periodic ? 1 : 0);
    const size_t main = (p->desc.precision == TPT_FP64) ? 2 * al(8 * n) + al(tsc) : al(tsc) + 3 * al(4 * n);
    return main + 16 * partial_slots(p) + 256;
}

}  // namespace tpt

tpt_plan_s::~tpt_plan_s() {
    if (buf.block || own_ws || h_norms) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(device);
        if (buf.block) (void)hipFree(buf.block);
        if (own_ws) (void)hipFree(own_ws);
        if (h_norms) (void)hipHostFree(h_norms);
        (void)hipSetDevice(cur);
    }
}

using namespace tpt;

extern "C" {

void tpt_plan_desc_init(tpt_plan_desc* d) {
    if (!d) return;
    std::memset(d, 0, sizeof(*d));
    for (int i = 0; i < 3; ++i) {
        d->n[i] = 2;
        d->bc[i][0] = d->bc[i][1] = TPT_BC_NEUMANN;
        d->loc[i] = TPT_LOC_CENTER;
    }
    d->kind = TPT_POISSON;
    d->precision = TPT_FP64;
    d->rtol = 1e-12;
    d->max_refine = 8;
    d->fixed_refine = -1;
    d->nrhs = 1;
}

int tpt_plan_create(const tpt_plan_desc* desc, tpt_plan* out) {
    if (!desc || !out) return fail(TPT_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (desc->nrhs < 1) return fail(TPT_ERR_INVALID, "nrhs must be >= 1");
    if (desc->kind != TPT_POISSON && desc->kind != TPT_HELMHOLTZ) return fail(TPT_ERR_INVALID, "unknown kind");
    if (desc->kind == TPT_HELMHOLTZ && !(desc->alpha > 0.0))
        return fail(TPT_ERR_INVALID, "Helmholtz needs alpha > 0");
    if (desc->precision < TPT_FP64 || desc->precision > TPT_MIXED_BF16X3)
        return fail(TPT_ERR_INVALID, "unknown precision");
    if (desc->implicit < TPT_IMPLICIT_XYZ || desc->implicit > TPT_IMPLICIT_Z)
        return fail(TPT_ERR_INVALID, "unknown implicit directions");
    if (desc->implicit != TPT_IMPLICIT_XYZ && desc->kind != TPT_HELMHOLTZ)
        return fail(TPT_ERR_INVALID, "only a Helmholtz plan can leave directions explicit");
    if (desc->implicit != TPT_IMPLICIT_XYZ && desc->precision != TPT_FP64)
        return fail(TPT_ERR_UNSUPPORTED, "yz and z implicit plans are FP64 only");
    for (int d = 0; d < 3; ++d) {
        if (desc->n[d] < 2) return fail(TPT_ERR_INVALID, "need at least 2 cells per direction");
        if (!desc->faces[d]) return fail(TPT_ERR_INVALID, "faces pointer is NULL");
    }
    std::unique_ptr<tpt_plan_s> p(new tpt_plan_s());
    p->desc = *desc;
    if (p->desc.rtol <= 0.0) p->desc.rtol = 1e-12;
    if (p->desc.max_refine <= 0) p->desc.max_refine = 8;
    p->host_only = (desc->flags & TPT_FLAG_HOST_ONLY) != 0;
    p->seq_thomas = (desc->flags & TPT_FLAG_SEQ_THOMAS) != 0;
    p->check = (desc->flags & TPT_FLAG_NO_CHECK) == 0;
    p->tx = desc->implicit == TPT_IMPLICIT_XYZ;
    p->ty = desc->implicit != TPT_IMPLICIT_Z;
    if (!p->host_only && hipGetDevice(&p->device) != hipSuccess)
        return fail(TPT_ERR_HIP, "no HIP device");
    for (int d = 0; d < 3; ++d) {
        p->faces[d].assign(desc->faces[d], desc->faces[d] + desc->n[d] + 1);
        p->desc.faces[d] = p->faces[d].data();
        std::string err = build_op1d(desc->n[d], p->faces[d].data(), desc->bc[d][0], desc->bc[d][1], desc->loc[d],
                                     p->op[d]);
        if (!err.empty()) return fail(TPT_ERR_INVALID, "direction " + std::to_string(d) + ": " + err);
        p->N[d] = p->op[d].n;
    }
    p->dof = (long long)p->N[0] * p->N[1] * p->N[2];
    std::string err;
    p->bx = basis_cache_get(desc->n[0], p->faces[0].data(), desc->bc[0][0], desc->bc[0][1], desc->loc[0],
                            p->host_only, err);
    if (!p->bx) return fail(err.find("memory") != std::string::npos ? TPT_ERR_OOM : TPT_ERR_INVALID, "x basis: " + err);
    p->by = basis_cache_get(desc->n[1], p->faces[1].data(), desc->bc[1][0], desc->bc[1][1], desc->loc[1],
                            p->host_only, err);
    if (!p->by) return fail(err.find("memory") != std::string::npos ? TPT_ERR_OOM : TPT_ERR_INVALID, "y basis: " + err);
    if (desc->kind == TPT_POISSON) {
        p->sigma = 0.0;
        p->tau = 1.0;
    } else {
        p->sigma = 1.0;
        p->tau = -desc->alpha;
    }
    // the null line: lambda_x = lambda_y = 0 (both exact) and a singular T_z
    if (desc->kind == TPT_POISSON && p->bx->eig.null_index >= 0 && p->by->eig.null_index >= 0 &&
        p->op[2].null_mode)
        p->null_line = p->bx->eig.null_index + p->N[0] * p->by->eig.null_index;
    p->info.null_line = p->null_line;
    p->run_check = p->check || (desc->precision != TPT_FP64 && p->null_line >= 0);
    {
        double ax = 0.0, ay = 0.0;
        for (double v : p->op[0].vol) ax += v;
        for (double v : p->op[1].vol) ay += v;
        p->last_area_inv = 1.0 / (ax * ay * p->op[2].vol[p->N[2] - 1]);
    }
    if (!p->host_only) {
        if (p->bx->fast_kind >= 0 && !(desc->flags & TPT_FLAG_DENSE_X)) p->fast[0] = p->bx->fast_kind;
        if (p->by->fast_kind >= 0 && !(desc->flags & TPT_FLAG_DENSE_Y)) p->fast[1] = p->by->fast_kind;
        // one pass for the x transform and the y GEMM (FP64; x rows of 128 or
        // 256 points, whole 128-row tiles of y)
        p->fuse_xy = p->tx && p->ty && desc->precision == TPT_FP64 && (desc->flags & TPT_FLAG_FUSE_XY) && p->fast[0] >= 0 &&
                     p->fast[1] < 0 && (p->N[0] == 128 || p->N[0] == 256) && p->N[1] % 128 == 0;
    }
    p->info.rel_residual = -1.0;
    p->info.compat_defect = p->check ? 0.0 : -1.0;
    p->info.nonfinite = p->check ? 0 : -1;
    if (!p->host_only) {
        const size_t nx = p->N[0], ny = p->N[1], nz = p->N[2];
        const size_t nstat = (size_t)TPT_STATS * p->desc.nrhs;
        const size_t doubles = 5 * (nx + ny + nz) + ny * nz + std::max(nx, ny) + nstat + 64;
        void* blk = nullptr;
        if (hipMalloc(&blk, doubles * 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(TPT_ERR_OOM, "out of device memory for plan coefficients");
        }
        p->buf.block = blk;
        std::vector<double> h(doubles, 0.0);
        double* w = h.data();
        auto put = [&](const std::vector<double>& v) {
            std::memcpy(w, v.data(), 8 * v.size());
            w += v.size();
        };
        put(p->op[0].a); put(p->op[0].b); put(p->op[0].c);
        put(p->op[1].a); put(p->op[1].b); put(p->op[1].c);
        put(p->op[2].a); put(p->op[2].b); put(p->op[2].c);
        put(p->op[0].vol); put(p->op[1].vol); put(p->op[2].vol);
        for (size_t k = 0; k < nz; ++k)
            for (size_t j = 0; j < ny; ++j) *w++ = p->op[1].vol[j] * p->op[2].vol[k];
        w += std::max(nx, ny);  // zeros
        for (int d = 0; d < 3; ++d) {
            // centre distances, half the sum of the two cell widths (as the
            // operator's couplings use them, so that D G is its Laplacian)
            const std::vector<double>& fc = p->faces[d];
            const size_t nc = fc.size() - 1, n = p->N[d];
            for (size_t m = 0; m < n; ++m) {
                const double wm = fc[m + 1] - fc[m];
                const double wn = m + 1 < nc ? fc[m + 2] - fc[m + 1] : fc[1] - fc[0];
                *w++ = 0.5 * (wm + wn);
            }
        }
        TPT_HIP(hipMemcpy(blk, h.data(), doubles * 8, hipMemcpyHostToDevice));
        double* d = (double*)blk;
        p->buf.ax = d; d += nx; p->buf.bx = d; d += nx; p->buf.cx = d; d += nx;
        p->buf.ay = d; d += ny; p->buf.by = d; d += ny; p->buf.cy = d; d += ny;
        p->buf.az = d; d += nz; p->buf.bz = d; d += nz; p->buf.cz = d; d += nz;
        p->buf.vx = d; d += nx; p->buf.vy = d; d += ny; p->buf.vz = d; d += nz;
        p->buf.vyz = d; d += ny * nz;
        p->buf.zeros = d; d += std::max(nx, ny);
        p->buf.dcx = d; d += nx; p->buf.dcy = d; d += ny; p->buf.dcz = d; d += nz;
        p->buf.norms = d;
        if (hipHostMalloc((void**)&p->h_norms, (nstat + 8) * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            p->h_norms = nullptr;
            return fail(TPT_ERR_OOM, "pinned host allocation failed");
        }
    }
    *out = p.release();
    return TPT_OK;
}

int tpt_plan_destroy(tpt_plan plan) {
    delete plan;
    return TPT_OK;
}

int tpt_plan_shape(tpt_plan p, int shape[3]) {
    if (!p || !shape) return fail(TPT_ERR_INVALID, "NULL argument");
    for (int d = 0; d < 3; ++d) shape[d] = p->N[d];
    return TPT_OK;
}

int tpt_plan_workspace_bytes(tpt_plan p, size_t* bytes) {
    if (!p || !bytes) return fail(TPT_ERR_INVALID, "NULL argument");
    *bytes = plan_workspace_bytes(p);
    return TPT_OK;
}

int tpt_plan_eigen(tpt_plan p, int dir, double* lam, double* Qt) {
    if (!p || !lam || dir < 0 || dir > 1) return fail(TPT_ERR_INVALID, "bad argument");
    const Eig1D& e = (dir == 0 ? p->bx : p->by)->eig;
    std::memcpy(lam, e.lam.data(), sizeof(double) * e.n);
    if (Qt) std::memcpy(Qt, e.Qt.data(), sizeof(double) * (size_t)e.n * e.n);
    return TPT_OK;
}

int tpt_plan_operator(tpt_plan p, int dir, double* a, double* b, double* c, double* vol) {
    if (!p || dir < 0 || dir > 2) return fail(TPT_ERR_INVALID, "bad argument");
    const Op1D& op = p->op[dir];
    const size_t n = sizeof(double) * op.n;
    if (a) std::memcpy(a, op.a.data(), n);
    if (b) std::memcpy(b, op.b.data(), n);
    if (c) std::memcpy(c, op.c.data(), n);
    if (vol) std::memcpy(vol, op.vol.data(), n);
    return TPT_OK;
}

int tpt_plan_transforms(tpt_plan p, int kinds[2]) {
    if (!p || !kinds) return fail(TPT_ERR_INVALID, "NULL argument");
    for (int d = 0; d < 2; ++d) kinds[d] = p->fast[d] < 0 ? TPT_XFORM_GEMM : TPT_XFORM_FFT + p->fast[d];
    if (!p->tx) kinds[0] = TPT_XFORM_NONE;
    if (!p->ty) kinds[1] = TPT_XFORM_NONE;
    return TPT_OK;
}

int tpt_plan_fused(tpt_plan p, int* fused) {
    if (!p || !fused) return fail(TPT_ERR_INVALID, "NULL argument");
    *fused = p->fuse_xy ? 1 : 0;
    return TPT_OK;
}

const char* tpt_last_error(void) { return tpt::last_error_cstr(); }
const char* tpt_version(void) { return "tpt 0.1 (gfx950)"; }

}  // extern "C"
