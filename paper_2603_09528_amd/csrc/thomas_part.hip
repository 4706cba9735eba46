// Partitioned batched Thomas along z (§2.2.2 step 2.3) for non-periodic
// lines: single- and multi-problem launches over a table of (lines per
// block, segments, planes per segment) configurations.
#include "device_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace tpt {

// ---------------------------------------------------------------------------
// Partitioned Thomas (non-periodic lines): each line is split into P
// segments of L planes, one lane per (line, segment), LB lines per block
// (lane t holds segment t / LB of line t % LB, so every load and store of a
// plane touches LB consecutive lines).  The segment's planes stay in
// registers: f is read once and x written once (16 B per unknown against 24 B
// for the sequential kernel), and the dependent chain per lane is P times
// shorter.
//
// Segment s owns rows k0 = sL .. k0+L-1; rows k0 .. k0+L-2 are its interior,
// row k0+L-1 its interface unknown z_s.  With the neighbouring interface
// values Xl = z_{s-1} and Xr = z_s taken as known, every interior unknown is
// affine in them, x_r = U_r + V_r Xr + W_r Xl.  Pass 1 finds these responses
// at the two ends of the interior: a downward elimination gives the last
// interior row (U, V, W at r = L-2), an upward one the first (r = 0), no
// back substitution needed.  Substituted into the interface rows they give a
// tridiagonal system of P unknowns per line,
//   (D + A Vd_s + C Wu_{s+1}) z_s + A Wd_s z_{s-1} + C Vu_{s+1} z_{s+1}
//       = f - A Ud_s - C Uu_{s+1},
// (A, D, C, f of row k0+L-1; Ud.. of segment s at its last interior row, Uu..
// of segment s+1 at its first), which the P lanes of the line solve by
// parallel cyclic reduction through LDS.
// Pass 2 folds Xl and Xr into the interior's first and last right-hand side
// and runs the interior Thomas with the pivots kept from pass 1.
//
// Rows k >= nz are identity rows (f = 0), so P L may exceed nz.  The pinned
// line (singular Poisson) has its row nz-1 replaced by the identity with
// f = 0: x_{nz-1} = 0 and rows 0..nz-2 unchanged, the gauge of §3.  Without
// pivoting the elimination relies, as the sequential one does, on the
// diagonal dominance of D + tau lambda.
// ---------------------------------------------------------------------------
template <int LB, int P, int L>
struct ThomasPartLds {
    static constexpr int NT = LB * P, CS = L + 1;  // CS: segment stride of cf (one row of bank padding)
    // (A, C, D, E) per row, E = 1 where the line shift applies (0 on identity
    // rows); segment s at s CS, then the pinned line's copy of segment
    // (nz-1)/L with row nz-1 made the identity
    double4 cf[(P + 1) * CS];
    double pcr[2][4][NT];  // interface rows (a, c, d, 1/b) by level; first the up-sweep responses
    double zz[P][LB];      // interface solution
};

// One block of LB lines (block index blk of the problem t with nlines lines).
template <int LB, int P, int L, typename TF, typename TX>
__device__ __forceinline__ void thomas_part_block(const ThomasDesc& t, long long nlines, long long blk,
                                                  ThomasPartLds<LB, P, L>& sh) {
    constexpr int NT = LB * P, M = L - 1, CS = L + 1, PIN = P * CS;
    constexpr int NE = (P + 1) * L, SI = (NE + NT - 1) / NT;  // staged rows, per thread
    static_assert(L >= 4, "segments need interior rows");
    const int nz = t.nz;
    const int sp = (nz - 1) / L;  // segment of row nz-1

    // Prologue, two forms.  EAGER: every global load of the block is issued
    // before any is waited for (at clamped, valid addresses, without
    // branches): the raw coefficients of its staged rows, the lambdas, the
    // segment's planes of f; the block then waits one memory latency and
    // pass 1 can start as the first planes arrive.  Otherwise the staging
    // loop waits for its coefficient loads before the planes are requested
    // (up to three latencies in a row), but the block needs about ten fewer
    // registers.  With L = 16 those ten registers cross the 128 that keep
    // four waves per SIMD, and the lazy form measured faster there (32-line
    // blocks at 1024^2 x 256: 0.98 against 1.06 ms); at L = 8 and 32 the
    // occupancy does not change and the eager form is faster (1024^2 x 512:
    // 2.19 against 2.34 ms; 1024^2 x 64: 0.214 against 0.228 ms).
    constexpr bool EAGER = L != 16;
    [[maybe_unused]] double za[SI], zb[SI], zc[SI];
    // (A, C, D, E) of staged row e; the pinned copy (seg == P) has its row
    // nz-1 as the identity
    auto stage_row = [&](int e, double a, double b, double c) {
        const int seg = e / L, r = e - seg * L;
        const int k = (seg < P ? seg : sp) * L + r;
        double4 v = make_double4(0.0, 0.0, 1.0, 0.0);
        if (k < nz && !(seg == P && k == nz - 1)) {
            v.x = k > 0 ? t.tau * a : 0.0;
            v.y = k < nz - 1 ? t.tau * c : 0.0;
            v.z = t.sigma + t.tau * b;
            v.w = 1.0;
        }
        sh.cf[seg * CS + r] = v;
    };
    if constexpr (EAGER) {
#pragma unroll
        for (int q = 0; q < SI; ++q) {
            const int e = threadIdx.x + q * NT, seg = e / L;
            const int k = min((seg < P ? seg : sp) * L + (e - seg * L), nz - 1);
            za[q] = t.az[k];
            zb[q] = t.bz[k];
            zc[q] = t.cz[k];
        }
    } else {
        for (int e = threadIdx.x; e < NE; e += NT) {
            const int seg = e / L;
            const int k = min((seg < P ? seg : sp) * L + (e - seg * L), nz - 1);
            stage_row(e, t.az[k], t.bz[k], t.cz[k]);
        }
    }
    const int l = threadIdx.x % LB, s = threadIdx.x / LB;
    const long long S = (long long)t.nx * t.ny;
    const long long glr = blk * LB + l;
    const bool live = glr < nlines;
    const long long gl = live ? glr : nlines - 1;
    const int sys = (int)(gl / S);
    const long long line = gl - (long long)sys * S;
    const int i = (int)(line % t.nx), j = (int)(line / t.nx);
    const double tl = t.tau * (t.lamx[i] + t.lamy[j]);
    const bool pinned = line == t.pin_line;
    const int k0 = s * L;
    const long long base = (long long)sys * S * nz + line;
    const TF* f = (const TF*)t.f + base;
    TX* x = (TX*)t.x + base;
    const bool full = k0 + L <= nz;

    double fv[L];
    if constexpr (EAGER) {
#pragma unroll
        for (int r = 0; r < L; ++r) fv[r] = (double)f[(long long)min(k0 + r, nz - 1) * S];
#pragma unroll
        for (int q = 0; q < SI; ++q)
            if (threadIdx.x + q * NT < NE) stage_row(threadIdx.x + q * NT, za[q], zb[q], zc[q]);
    } else {
        if (live && full) {
#pragma unroll
            for (int r = 0; r < L; ++r) fv[r] = (double)f[(long long)(k0 + r) * S];
        } else {
#pragma unroll
            for (int r = 0; r < L; ++r) fv[r] = live && k0 + r < nz ? (double)f[(long long)(k0 + r) * S] : 0.0;
        }
        if (pinned && s == sp) {
#pragma unroll
            for (int r = 0; r < L; ++r)
                if (k0 + r == nz - 1) fv[r] = 0.0;
        }
    }
    __syncthreads();
    const double4* cb = sh.cf + ((pinned && s == sp) ? PIN : s * CS);
    if constexpr (EAGER) {
        // identity rows (beyond nz, and the pinned row) carry no data: E = 0
        // there and 1 elsewhere.  (A select on the row index instead was
        // scheduled before the barrier, making it wait for the loads.)
#pragma unroll
        for (int r = 0; r < L; ++r) fv[r] *= cb[r].w;
    }

    // ---- pass 1: end responses of the interior rows 0 .. M-1 ----
    double ip[M];
    double Ud, Vd, Wd, Uu, Vu, Wu;
    {
        double4 v = cb[0];
        ip[0] = recip(__builtin_fma(v.w, tl, v.z));
        double Fd = fv[0] * ip[0], Gd = v.x * ip[0], cprev = v.y;
#pragma unroll
        for (int r = 1; r < M; ++r) {
            v = cb[r];
            ip[r] = recip(__builtin_fma(v.w, tl, v.z) - v.x * cprev * ip[r - 1]);
            Fd = (fv[r] - v.x * Fd) * ip[r];
            Gd = -v.x * Gd * ip[r];
            cprev = v.y;
        }
        Ud = Fd;
        Vd = -cprev * ip[M - 1];
        Wd = -Gd;
        // re-read the coefficients rather than keep the down sweep's in
        // registers
        asm volatile("" ::: "memory");
        v = cb[M - 1];
        double jp = recip(__builtin_fma(v.w, tl, v.z));
        double Fu = fv[M - 1] * jp, Hu = v.y * jp, anext = v.x;
#pragma unroll
        for (int r = M - 2; r >= 0; --r) {
            v = cb[r];
            jp = recip(__builtin_fma(v.w, tl, v.z) - v.y * anext * jp);
            Fu = (fv[r] - v.y * Fu) * jp;
            Hu = -v.y * Hu * jp;
            anext = v.x;
        }
        Uu = Fu;
        Vu = -Hu;
        Wu = -anext * jp;
    }
    // materialise the responses here: left to the compiler, the products
    // behind Wd and Vd sink past the barrier below with every factor kept
    // in registers
    asm volatile("" : "+v"(Ud), "+v"(Vd), "+v"(Wd), "+v"(Uu), "+v"(Vu), "+v"(Wu));
    // ---- interface system: parallel cyclic reduction over the P rows ----
    // Lane s forms row s (a z_{s-1} + b z_s + c z_{s+1} = d) from its own
    // down-sweep responses and the up-sweep responses of segment s+1; each
    // level h = 1, 2, 4, .. eliminates the couplings to rows s -+ h with the
    // rows there, so after log2 P levels row s reads b z_s = d.  Rows are
    // exchanged through two LDS buffers used alternately (one barrier per
    // level); rows outside 0..P-1 are the identity.
    const int me = threadIdx.x;
    sh.pcr[1][0][me] = Uu;
    sh.pcr[1][1][me] = Vu;
    sh.pcr[1][2][me] = Wu;
    __syncthreads();
    double ra, rb, rc, rd;
    {
        const double4 v = cb[M];  // the interface row (pinned copy on the pinned line)
        const double A = v.x, C = v.y;
        ra = A * Wd;
        rb = __builtin_fma(v.w, tl, v.z) + A * Vd;
        rc = 0.0;
        rd = fv[M] - A * Ud;
        if (s + 1 < P) {
            const int nb = me + LB;
            rb += C * sh.pcr[1][2][nb];
            rc = C * sh.pcr[1][1][nb];
            rd -= C * sh.pcr[1][0][nb];
        }
    }
    double ib = recip(rb);
#pragma unroll 1
    for (int h = 1, lvl = 0; h < P; h *= 2, ++lvl) {
        double (*R)[NT] = sh.pcr[lvl & 1];
        R[0][me] = ra;
        R[1][me] = rc;
        R[2][me] = rd;
        R[3][me] = ib;
        __syncthreads();
        double na = 0.0, nc = 0.0, nb = rb, nd = rd;
        if (s >= h) {
            const int u = me - h * LB;
            const double k1 = ra * R[3][u];
            na = -R[0][u] * k1;
            nb -= R[1][u] * k1;
            nd -= R[2][u] * k1;
        }
        if (s + h < P) {
            const int u = me + h * LB;
            const double k2 = rc * R[3][u];
            nc = -R[1][u] * k2;
            nb -= R[0][u] * k2;
            nd -= R[2][u] * k2;
        }
        ra = na;
        rb = nb;
        rc = nc;
        rd = nd;
        ib = recip(rb);
    }
    sh.zz[s][l] = rd * ib;
    __syncthreads();

    // ---- pass 2: interior Thomas with the interface values folded in ----
    const double Xr = sh.zz[s][l], Xl = s > 0 ? sh.zz[s - 1][l] : 0.0;
    fv[0] -= cb[0].x * Xl;
    fv[M - 1] -= cb[M - 1].y * Xr;
    fv[0] *= ip[0];
#pragma unroll
    for (int r = 1; r < M; ++r) fv[r] = (fv[r] - cb[r].x * fv[r - 1]) * ip[r];
#pragma unroll
    for (int r = M - 2; r >= 0; --r) fv[r] -= cb[r].y * ip[r] * fv[r + 1];
    fv[M] = Xr;
    if (live && full) {
#pragma unroll
        for (int r = 0; r < L; ++r) x[(long long)(k0 + r) * S] = (TX)fv[r];
    } else if (live) {
#pragma unroll
        for (int r = 0; r < L; ++r)
            if (k0 + r < nz) x[(long long)(k0 + r) * S] = (TX)fv[r];
    }
}

template <int LB, int P, int L, typename TF, typename TX>
__global__ __launch_bounds__(LB * P) void thomas_part_kernel(ThomasDesc t, long long nlines) {
    __shared__ ThomasPartLds<LB, P, L> sh;
    thomas_part_block<LB, P, L, TF, TX>(t, nlines, blockIdx.x, sh);
}

// Multi-problem: block_begin counts blocks of LB lines per problem; every
// problem of the list has the same storage types and P L >= nz.
template <int LB, int P, int L, typename TF, typename TX>
__global__ __launch_bounds__(LB * P) void thomas_part_multi_kernel(const ThomasDesc* __restrict__ work, int nwork,
                                                                   long long total_blocks) {
    __shared__ ThomasPartLds<LB, P, L> sh;
    for (long long blk = blockIdx.x; blk < total_blocks; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const ThomasDesc t = work[lo];
        thomas_part_block<LB, P, L, TF, TX>(t, (long long)t.nx * t.ny * t.nsys, blk - t.block_begin, sh);
        __syncthreads();
    }
}

// Configurations (lines per block LB, segments P, planes per segment L); a
// line of nz planes needs P L >= nz.  Blocks of LB P lanes; the register
// count grows with L (about 122 at L = 16, 246 at L = 32), which with the
// block size sets how many blocks share a compute unit.
struct ThomasPart {
    int LB, P, L;
};
#define TPT_THOMAS_PARTS(X) \
    X(64, 4, 8)             \
    X(64, 8, 8)             \
    X(32, 8, 8)             \
    X(64, 8, 16)            \
    X(32, 8, 16)            \
    X(16, 8, 16)            \
    X(64, 16, 16)           \
    X(32, 16, 16)           \
    X(16, 16, 16)           \
    X(64, 8, 32)            \
    X(32, 8, 32)            \
    X(16, 8, 32)            \
    X(16, 32, 16)           \
    X(32, 16, 32)           \
    X(16, 16, 32)           \
    X(16, 64, 16)           \
    X(16, 32, 32)
#define TPT_TP_ROW(XLB, XP, XL) {XLB, XP, XL},
constexpr ThomasPart THOMAS_PARTS[] = {TPT_THOMAS_PARTS(TPT_TP_ROW)};
#undef TPT_TP_ROW
static_assert(sizeof(THOMAS_PARTS) / sizeof(THOMAS_PARTS[0]) == THOMAS_NPART, "configuration count");

void thomas_part_shape(int v, int* lb, int* p, int* l) {
    *lb = THOMAS_PARTS[v].LB;
    *p = THOMAS_PARTS[v].P;
    *l = THOMAS_PARTS[v].L;
}

// Automatic choice by nz and line count (the autotuner's measurement on the
// plan's own lines takes precedence): the configuration measured fastest on
// lines of 32, 64, 128, 256, 512 and 1024 planes (FP64, 16 K - 1 M lines).
// Small blocks win: with the barriers of each block, several blocks per
// compute unit keep its loads going while one block computes; from about
// 256 K lines, 32-line blocks (256-byte plane segments) overtake 16-line ones
// (1024^2 x 256: 0.98 against 1.22 ms; 256^3: 55 against 54 us).  Lines of
// more than 512 planes need 1024-lane blocks (one per compute unit); with
// many lines the sequential kernel then has parallelism enough and is faster
// (1024^3: 5.2 against 6.9 ms), with few it is not (32 K lines of 1024
// planes: 0.24 against 0.17 ms).
static int thomas_part_auto(int nz, long long lines) {
    if (nz > 512 && lines >= 131072) return -1;
    const bool many = lines >= 262144;
    const int want[][2] = {{32, 0}, {64, 2}, {128, 4}, {256, many ? 7 : 8}, {512, many ? 13 : 12}, {1024, 15}};
    for (const auto& w : want)
        if (nz <= w[0]) return w[1];
    return -1;
}

int thomas_variant(const ThomasDesc& t) {
    const bool same = t.tf == t.tx;
    if (t.variant == THOMAS_SEQ) return THOMAS_SEQ;
    if (t.variant == THOMAS_AUTO) {
        if (t.periodic || !same || t.nz < 16) return THOMAS_SEQ;
        const int v = thomas_part_auto(t.nz, (long long)t.nx * t.ny * t.nsys);
        return v < 0 ? THOMAS_SEQ : THOMAS_PART + v;
    }
    const int v = t.variant - THOMAS_PART;
    if (v < 0 || v >= THOMAS_NPART || t.periodic || !same || THOMAS_PARTS[v].P * THOMAS_PARTS[v].L < t.nz)
        return -1;
    return t.variant;
}

long long thomas_part_blocks(const ThomasDesc& t, int v) {
    const long long lb = THOMAS_PARTS[v].LB;
    return ((long long)t.nx * t.ny * t.nsys + lb - 1) / lb;
}

template <typename T>
static hipError_t launch_part_t(const ThomasDesc& t, int v, hipStream_t s) {
    const long long n = (long long)t.nx * t.ny * t.nsys;
    const dim3 gr((unsigned)thomas_part_blocks(t, v));
#define TPT_TP_CASE(XLB, XP, XL)                                                           \
    if (THOMAS_PARTS[v].LB == XLB && THOMAS_PARTS[v].P == XP && THOMAS_PARTS[v].L == XL) { \
        TPT_KLAUNCH((thomas_part_kernel<XLB, XP, XL, T, T>), gr, dim3(XLB * XP), 0, s, t, n); \
        return hipGetLastError();                                                       \
    }
    TPT_THOMAS_PARTS(TPT_TP_CASE)
#undef TPT_TP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_thomas_part(const ThomasDesc& t, int v, hipStream_t s) {
    if (v < 0 || v >= THOMAS_NPART || t.tf != t.tx) return hipErrorInvalidValue;
    return t.tf == DT_F64 ? launch_part_t<double>(t, v, s) : launch_part_t<float>(t, v, s);
}

template <typename T>
static hipError_t launch_part_multi_t(const ThomasDesc* d_work, int nwork, long long total_blocks, int v,
                                      hipStream_t s) {
    const dim3 gr((unsigned)std::min(total_blocks, 8 * PERSISTENT_BLOCKS));
#define TPT_TP_CASE(XLB, XP, XL)                                                                          \
    if (THOMAS_PARTS[v].LB == XLB && THOMAS_PARTS[v].P == XP && THOMAS_PARTS[v].L == XL) {                \
        TPT_KLAUNCH((thomas_part_multi_kernel<XLB, XP, XL, T, T>), gr, dim3(XLB * XP), 0, s, d_work, nwork, \
                    total_blocks);                                                                     \
        return hipGetLastError();                                                                      \
    }
    TPT_THOMAS_PARTS(TPT_TP_CASE)
#undef TPT_TP_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_thomas_part_multi(const ThomasDesc* d_work, int nwork, long long total_blocks, int v, int dtype,
                                    hipStream_t s) {
    if (total_blocks <= 0) return hipSuccess;
    if (v < 0 || v >= THOMAS_NPART) return hipErrorInvalidValue;
    return dtype == DT_F64 ? launch_part_multi_t<double>(d_work, nwork, total_blocks, v, s)
                           : launch_part_multi_t<float>(d_work, nwork, total_blocks, v, s);
}

}  // namespace tpt
