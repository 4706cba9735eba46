// HIP kernels for gfx950 (CDNA4): eigenbasis-transform GEMMs on MFMA,
// lane-per-line batched Thomas, FP64 7-point residual, reductions.
//
// Layout of every field: u[k][j][i], x fastest.  The x transform is a GEMM
// whose rows are the N_y N_z x-lines (A = field, K = N_x contiguous) and whose
// B is the basis (end of §2.2.2: all lines stacked into one GEMM).  The y
// transform is a strided batch over z slabs of a left multiplication by the
// basis (A = basis, B = slab with x contiguous), so no transpose is needed.
#include "device_common.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace tpt {

const char* tile_variant_name(int v) {
    static const char* names[TV_COUNT] = {"128x128", "64x128", "128x64", "64x64", "32x64", "128x128k32", "128x128p",
                                          "128x128p8", "128x128w8"};
    return (v >= 0 && v < TV_COUNT) ? names[v] : "?";
}

void tile_variant_shape(int v, int* bm, int* bn) {
    static const int s[TV_COUNT][2] = {{128, 128}, {64, 128}, {128, 64}, {64, 64}, {32, 64}, {128, 128}, {128, 128},
                                       {128, 128}, {128, 128}};
    *bm = s[v][0];
    *bn = s[v][1];
}

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

long long persistent_gemm_grid(long long tiles) {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cus[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    long long grid = 2LL * cus[dev];
    grid -= grid % 8;
    if (grid < 8) grid = 8;
    return tiles < grid ? tiles : grid;
}

long long gemm_blocks(const GemmDesc& g, int variant) {
    int bm, bn;
    tile_variant_shape(variant, &bm, &bn);
    return (long long)cdiv(g.M, bm) * cdiv(g.N, bn) * g.batch;
}

hipError_t launch_gemm(GemmDesc g, int prec, int variant, hipStream_t s) {
    int bm, bn;
    if (variant < 0 || variant >= TV_COUNT) return hipErrorInvalidValue;
    tile_variant_shape(variant, &bm, &bn);
    g.tiles_m = cdiv(g.M, bm);
    g.tiles_n = cdiv(g.N, bn);
    g.block_begin = 0;
    const long long blocks = (long long)g.tiles_m * g.tiles_n * g.batch;
    switch (prec) {
        case GP_F64: return launch_gemm_f64(g, nullptr, 0, blocks, variant, s);
        case GP_F32: return launch_gemm_f32(g, nullptr, 0, blocks, variant, s);
        case GP_BF16X3: return launch_gemm_bf16(g, nullptr, 0, blocks, variant, s);
    }
    return hipErrorInvalidValue;
}

void worklist_shape(GemmDesc& g) {
    if (g.b_nk) {
        g.tiles_m = cdiv(g.M, 128);
        g.tiles_n = cdiv((long long)g.N * g.batch, 64);
    } else {
        g.tiles_m = cdiv(g.M, 64);
        g.tiles_n = cdiv((long long)g.N * g.batch, 128);
    }
}

long long worklist_tiles(const GemmDesc& g) {
    GemmDesc t = g;
    worklist_shape(t);
    return (long long)t.tiles_m * t.tiles_n;
}

bool worklist_ok(const GemmDesc& g, int prec) {
    if (prec == GP_BF16X3) return false;
    const long long es = prec == GP_F64 ? 8 : 4;
    const long long lim = 0x7ffffff0LL;
    if (g.b_nk) {
        // x pass: one problem, no batch; a tile's A rows and the basis
        return g.batch == 1 && 128LL * g.lda * 8 < lim && (long long)g.N * g.ldb * es < lim;
    }
    // y pass: slab-folded columns and the B offsets of a tile's slabs
    const long long ntot = (long long)g.N * g.batch;
    return ntot < 0x7fffffffLL && (long long)g.M * g.lda * es < lim && g.sB * es * (128 / g.N + 3) < lim &&
           g.sB < 0x7fffffffLL;
}

hipError_t launch_gemm_worklist(const GemmDesc& rep, const GemmDesc* d_work, int nwork, long long tiles, int prec,
                                hipStream_t s) {
    switch (prec) {
        case GP_F64: return launch_gemm_worklist_f64(rep, d_work, nwork, tiles, s);
        case GP_F32: return launch_gemm_worklist_f32(rep, d_work, nwork, tiles, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gemm_multi(const GemmDesc& rep, const GemmDesc* d_work, int nwork, long long total_blocks,
                             int prec, int variant, hipStream_t s) {
    switch (prec) {
        case GP_F64: return launch_gemm_f64(rep, d_work, nwork, total_blocks, variant, s);
        case GP_F32: return launch_gemm_f32(rep, d_work, nwork, total_blocks, variant, s);
        case GP_BF16X3: return launch_gemm_bf16(rep, d_work, nwork, total_blocks, variant, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched Thomas along z, one lane per (i, j) line (§2.2.2 step 2.3): at each
// k the lanes of a wave touch consecutive addresses (stride N_x N_y between k
// planes).  Arithmetic in FP64 whatever the storage type of f and x.
//
// Traffic: the forward elimination keeps c' and d' in registers and stores
// only a checkpoint (c', d') every THOMAS_KC planes; the back substitution
// walks the chunks from the top, re-reads the chunk of f, recomputes its c'
// and d' from the checkpoint and substitutes.  So f is read twice and x
// written once (no per-unknown scratch), and x may alias f.  Loads of the
// next chunk are issued before the current chunk is computed.
//
// The line-independent coefficients A_k = tau a_k, D_k = sigma + tau b_k,
// C_k = tau c_k are staged in LDS once per block: the elimination is one
// dependent chain per line, and a coefficient fetched from memory inside it
// would also wait for the prefetched chunk.
//
// The line pin_line is the null line of a singular Poisson problem: its final
// pivot vanishes and its last unknown is set to zero (§3).
// ---------------------------------------------------------------------------
constexpr int THOMAS_KC = 16;
constexpr int THOMAS_NT = 256;

long long thomas_scratch_doubles(int nx, int ny, int nz, int nsys, int periodic) {
    const long long lines = (long long)nx * ny * nsys;
    const long long nck = (nz + THOMAS_KC - 1) / THOMAS_KC;
    return (periodic ? 4 : 2) * lines * nck;
}

// Stage the coefficients of one problem in LDS as planes of nz doubles:
// A_k (0 at k = 0), D_k, C_k (0 at k = nz-1) and AC_k = A_{k+1} C_k (the
// coupling of pivot k+1 to pivot k; 0 at k = nz-1).
constexpr int THOMAS_LDS_PLANES = 4;
__device__ __forceinline__ void thomas_stage(const ThomasDesc& t, double* lds) {
    const int nz = t.nz;
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        const double a = k > 0 ? t.tau * t.az[k] : 0.0;
        const double c = k < nz - 1 ? t.tau * t.cz[k] : 0.0;
        lds[k] = a;
        lds[nz + k] = t.sigma + t.tau * t.bz[k];
        lds[2 * nz + k] = c;
        lds[3 * nz + k] = k < nz - 1 ? t.tau * t.az[k + 1] * c : 0.0;
    }
}

// The elimination carries the inverse pivot: pivot k is
// q_k = D_k + tau lambda - AC_{k-1} / q_{k-1} and d'_k = (f_k - A_k d'_{k-1}) / q_k,
// so the dependent chain per step is one FMA and the reciprocal; c'_k = C_k / q_k
// is only needed by the back substitution.
template <typename TF, typename TX>
__device__ __forceinline__ void thomas_line(const ThomasDesc& t, long long gl, const double* __restrict__ cf) {
    constexpr int KC = THOMAS_KC;
    const long long S = (long long)t.nx * t.ny;
    const int sys = (int)(gl / S);
    const long long line = gl - (long long)sys * S;
    const int i = (int)(line % t.nx), j = (int)(line / t.nx);
    const int nz = t.nz;
    const int nc = (nz + KC - 1) / KC;
    const long long lines = S * t.nsys;
    const double tl = t.tau * (t.lamx[i] + t.lamy[j]);
    const long long base = (long long)sys * S * nz + line;
    const TF* f = (const TF*)t.f + base;
    TX* x = (TX*)t.x + base;
    double2* ck = (double2*)t.scratch + gl;  // ck[c * lines]: (1/q, d') entering chunk c
    const bool pinned = line == t.pin_line;
    const double* __restrict__ cA = cf;
    const double* __restrict__ cD = cf + nz;
    const double* __restrict__ cC = cf + 2 * nz;
    const double* __restrict__ cAC = cf + 3 * nz;

    // step k below the top plane: (ip, dp) <- (1/q_k, d'_k)
    auto step = [&](int k, double fk, double& ip, double& dp) {
        const double acp = k > 0 ? cAC[k - 1] : 0.0;
        ip = recip(cD[k] + tl - acp * ip);
        dp = (fk - cA[k] * dp) * ip;
    };
    // any step, including the top plane (pinned line: last unknown zero)
    auto step_top = [&](int k, double fk, double& ip, double& dp) {
        step(k, fk, ip, dp);
        if (k == nz - 1 && pinned) {
            ip = 0.0;
            dp = 0.0;
        }
    };

    // ---- forward elimination ----
    // (chunks below the top run without guards, so the coefficient reads of a
    // chunk can be issued ahead of its dependent chain)
    double ip = 0.0, dp = 0.0;
    double fb[KC], fn[KC];
#pragma unroll
    for (int e = 0; e < KC; ++e) fb[e] = e < nz ? (double)f[(long long)e * S] : 0.0;
    for (int c = 0; c < nc; ++c) {
        const int k0 = c * KC;
        ck[(long long)c * lines] = make_double2(ip, dp);
        if (k0 + 2 * KC <= nz) {
#pragma unroll
            for (int e = 0; e < KC; ++e) fn[e] = (double)f[(long long)(k0 + KC + e) * S];
        } else {
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const int k = k0 + KC + e;
                fn[e] = k < nz ? (double)f[(long long)k * S] : 0.0;
            }
        }
        if (k0 + KC < nz) {
            // coefficients read one step ahead of the chain that uses them
            double nA = cA[k0], nD = cD[k0], nAC = k0 > 0 ? cAC[k0 - 1] : 0.0;
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const double a = nA, d = nD, acp = nAC;
                if (e + 1 < KC) {
                    nA = cA[k0 + e + 1];
                    nD = cD[k0 + e + 1];
                    nAC = cAC[k0 + e];
                }
                ip = recip(d + tl - acp * ip);
                dp = (fb[e] - a * dp) * ip;
            }
        } else {
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const int k = k0 + e;
                if (k < nz) step_top(k, fb[e], ip, dp);
            }
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) fb[e] = fn[e];
    }

    // ---- back substitution chunk by chunk from the top ----
    double xv = 0.0;  // x_{k+1} entering each step from above
    {
        const int k0 = (nc - 1) * KC;
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + e;
            fb[e] = k < nz ? (double)f[(long long)k * S] : 0.0;
        }
    }
    for (int c = nc - 1; c >= 0; --c) {
        const int k0 = c * KC;
        if (c > 0) {
#pragma unroll
            for (int e = 0; e < KC; ++e) fn[e] = (double)f[(long long)(k0 - KC + e) * S];
        }
        const double2 c0 = ck[(long long)c * lines];
        double cb[KC];
        double ipr = c0.x, dpr = c0.y;
        if (k0 + KC < nz) {
            // a whole chunk below the top plane: no guards; recompute the
            // chunk (c' into cb, d' replaces f in fb)
            double nA = cA[k0], nD = cD[k0], nAC = k0 > 0 ? cAC[k0 - 1] : 0.0;
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const double a = nA, d = nD, acp = nAC;
                if (e + 1 < KC) {
                    nA = cA[k0 + e + 1];
                    nD = cD[k0 + e + 1];
                    nAC = cAC[k0 + e];
                }
                ipr = recip(d + tl - acp * ipr);
                dpr = (fb[e] - a * dpr) * ipr;
                cb[e] = cC[k0 + e] * ipr;
                fb[e] = dpr;
            }
#pragma unroll
            for (int e = KC - 1; e >= 0; --e) {
                xv = fb[e] - cb[e] * xv;
                x[(long long)(k0 + e) * S] = (TX)xv;
            }
        } else {
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const int k = k0 + e;
                if (k < nz) step_top(k, fb[e], ipr, dpr);
                cb[e] = k < nz ? cC[k] * ipr : 0.0;
                fb[e] = dpr;
            }
#pragma unroll
            for (int e = KC - 1; e >= 0; --e) {
                const int k = k0 + e;
                if (k < nz) {
                    xv = (k == nz - 1) ? fb[e] : fb[e] - cb[e] * xv;  // top: x = d' (0 on the pinned line)
                    x[(long long)k * S] = (TX)xv;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) fb[e] = fn[e];
    }
}

// Periodic z: every line is cyclic, with corners tau az[0] (row 0, column
// nz-1) and tau cz[nz-1] (row nz-1, column 0).  Eliminating the last unknown
// leaves the tridiagonal system of rows 0..nz-2,
//   A' x' = f' - x_{nz-1} e,  e = tau az[0] e_0 + tau cz[nz-2] e_{nz-2},
// so x' = y - x_{nz-1} v with A' y = f', A' v = e (one forward elimination
// for both right-hand sides), and the last row gives
//   x_{nz-1} = (f_{nz-1} - tau cz[nz-1] y_0 - tau az[nz-1] y_{nz-2})
//            / (d_{nz-1} - tau cz[nz-1] v_0 - tau az[nz-1] v_{nz-2}).
// Passes: forward elimination (checkpoints of c', d'_y, d'_v), a back
// substitution that only finds y_0 and v_0, and a second one that writes
// x = y - x_{nz-1} v.  On the pinned line (singular Poisson) x_{nz-1} = 0 and
// the last equation is dropped, the gauge of §3.  nz >= 2.
template <typename TF, typename TX>
__device__ __forceinline__ void thomas_line_cyclic(const ThomasDesc& t, long long gl, const double* __restrict__ cf) {
    constexpr int KC = THOMAS_KC;
    const long long S = (long long)t.nx * t.ny;
    const int sys = (int)(gl / S);
    const long long line = gl - (long long)sys * S;
    const int i = (int)(line % t.nx), j = (int)(line / t.nx);
    const int nz = t.nz, nr = nz - 1;  // reduced system rows 0 .. nr-1
    const int nc = (nr + KC - 1) / KC;
    const long long lines = S * t.nsys;
    const double tl = t.tau * (t.lamx[i] + t.lamy[j]);
    const long long base = (long long)sys * S * nz + line;
    const TF* f = (const TF*)t.f + base;
    TX* x = (TX*)t.x + base;
    double2* ck = (double2*)t.scratch + gl;  // ck[2 c lines]: (c', d'_y), ck[(2c+1) lines]: (d'_v, -)
    const bool pinned = line == t.pin_line;
    const double tau = t.tau;
    const double* __restrict__ cA = cf;
    const double* __restrict__ cD = cf + nz;
    const double* __restrict__ cC = cf + 2 * nz;
    // coupling of rows 0 and nr-1 of the reduced system to x_{nz-1}
    const double e0 = tau * t.az[0], e1 = tau * t.cz[nr - 1];
    auto step = [&](int k, double fk, double& cp, double& dy, double& dv) {
        const double a = cA[k];
        const double den = cD[k] + tl - a * cp;
        const double inv = recip(den);
        const double ek = (k == 0 ? e0 : 0.0) + (k == nr - 1 ? e1 : 0.0);
        cp = k < nr - 1 ? cC[k] * inv : 0.0;
        dy = (fk - a * dy) * inv;
        dv = (ek - a * dv) * inv;
    };
    double fb[KC], fn[KC];
    // ---- forward elimination of the reduced system ----
    double cp = 0.0, dy = 0.0, dv = 0.0;
#pragma unroll
    for (int e = 0; e < KC; ++e) fb[e] = e < nr ? (double)f[(long long)e * S] : 0.0;
    for (int c = 0; c < nc; ++c) {
        const int k0 = c * KC;
        ck[(long long)(2 * c) * lines] = make_double2(cp, dy);
        ck[(long long)(2 * c + 1) * lines] = make_double2(dv, 0.0);
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + KC + e;
            fn[e] = k < nr ? (double)f[(long long)k * S] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + e;
            if (k < nr) step(k, fb[e], cp, dy, dv);
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) fb[e] = fn[e];
    }
    const double ytop = dy, vtop = dv;  // y_{nr-1}, v_{nr-1}
    const double flast = (double)f[(long long)nr * S];
    // ---- back substitutions from the top: pass 0 finds y_0, v_0; pass 1 writes ----
    double xlast = 0.0;
    for (int pass = pinned ? 1 : 0; pass < 2; ++pass) {
        if (pass == 1) x[(long long)nr * S] = (TX)xlast;
        double yv = 0.0, vv = 0.0;  // y_{k+1}, v_{k+1}
        {
            const int k0 = (nc - 1) * KC;
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const int k = k0 + e;
                fb[e] = k < nr ? (double)f[(long long)k * S] : 0.0;
            }
        }
        for (int c = nc - 1; c >= 0; --c) {
            const int k0 = c * KC;
            if (c > 0) {
#pragma unroll
                for (int e = 0; e < KC; ++e) fn[e] = (double)f[(long long)(k0 - KC + e) * S];
            }
            const double2 c0 = ck[(long long)(2 * c) * lines];
            const double2 c1 = ck[(long long)(2 * c + 1) * lines];
            double cb[KC], db[KC];
            double cpr = c0.x, dyr = c0.y, dvr = c1.x;
#pragma unroll
            for (int e = 0; e < KC; ++e) {
                const int k = k0 + e;
                if (k < nr) step(k, fb[e], cpr, dyr, dvr);
                cb[e] = cpr;
                fb[e] = dyr;
                db[e] = dvr;
            }
#pragma unroll
            for (int e = KC - 1; e >= 0; --e) {
                const int k = k0 + e;
                if (k < nr) {
                    yv = (k == nr - 1) ? fb[e] : fb[e] - cb[e] * yv;
                    vv = (k == nr - 1) ? db[e] : db[e] - cb[e] * vv;
                    if (pass == 1) x[(long long)k * S] = (TX)(yv - xlast * vv);
                }
            }
#pragma unroll
            for (int e = 0; e < KC; ++e) fb[e] = fn[e];
        }
        if (pass == 0) {
            // yv, vv now hold y_0, v_0
            const double cl = tau * t.cz[nz - 1], al = tau * t.az[nz - 1];
            const double dl = cD[nz - 1] + tl;
            xlast = (flast - cl * yv - al * ytop) * recip(dl - cl * vv - al * vtop);
        }
    }
}

template <typename TF, typename TX>
__device__ __forceinline__ void thomas_any(const ThomasDesc& t, long long gl, const double* cf) {
    if (t.periodic) thomas_line_cyclic<TF, TX>(t, gl, cf);
    else thomas_line<TF, TX>(t, gl, cf);
}

__device__ __forceinline__ void thomas_dispatch(const ThomasDesc& t, long long gl, const double* cf) {
    if (t.tf == DT_F64 && t.tx == DT_F64) thomas_any<double, double>(t, gl, cf);
    else if (t.tf == DT_F32 && t.tx == DT_F32) thomas_any<float, float>(t, gl, cf);
    else if (t.tf == DT_F64) thomas_any<double, float>(t, gl, cf);
    else thomas_any<float, double>(t, gl, cf);
}

// Single-problem launches: one kernel per storage-type pair and line kind,
// so each keeps only its own registers.  Dynamic LDS: 3 nz doubles.
template <typename TF, typename TX, bool CYC>
__global__ __launch_bounds__(THOMAS_NT) void thomas_kernel(ThomasDesc t, long long nlines) {
    extern __shared__ double th_lds[];
    thomas_stage(t, th_lds);
    __syncthreads();
    const long long gl = (long long)blockIdx.x * THOMAS_NT + threadIdx.x;
    if (gl >= nlines) return;
    if constexpr (CYC) thomas_line_cyclic<TF, TX>(t, gl, th_lds);
    else thomas_line<TF, TX>(t, gl, th_lds);
}

// Multi-problem: blocks never straddle problems (block_begin counts blocks of
// THOMAS_NT lines per problem), so each block stages one problem's
// coefficients.
__global__ __launch_bounds__(THOMAS_NT) void thomas_multi_kernel(const ThomasDesc* __restrict__ work, int nwork,
                                                                 long long total_blocks) {
    extern __shared__ double th_lds[];
    for (long long blk = blockIdx.x; blk < total_blocks; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const ThomasDesc t = work[lo];
        thomas_stage(t, th_lds);
        __syncthreads();
        const long long gl = (blk - t.block_begin) * THOMAS_NT + threadIdx.x;
        if (gl < (long long)t.nx * t.ny * t.nsys) thomas_dispatch(t, gl, th_lds);
        __syncthreads();
    }
}

long long thomas_blocks(const ThomasDesc& t) {
    return ((long long)t.nx * t.ny * t.nsys + THOMAS_NT - 1) / THOMAS_NT;
}

hipError_t launch_thomas(const ThomasDesc& t, hipStream_t s) {
    const long long n = (long long)t.nx * t.ny * t.nsys;
    if (n <= 0) return hipSuccess;
    const int variant = thomas_variant(t);
    if (variant < 0) return hipErrorInvalidValue;
    if (variant >= THOMAS_PART) return launch_thomas_part(t, variant - THOMAS_PART, s);
    const long long blocks = thomas_blocks(t);
    const dim3 gr((unsigned)blocks), bl(THOMAS_NT);
    const size_t sm = THOMAS_LDS_PLANES * sizeof(double) * (size_t)t.nz;
#define TPT_THOMAS_LAUNCH(TF, TX)                                                                    \
    do {                                                                                           \
        if (t.periodic) TPT_KLAUNCH((thomas_kernel<TF, TX, true>), gr, bl, sm, s, t, n);     \
        else TPT_KLAUNCH((thomas_kernel<TF, TX, false>), gr, bl, sm, s, t, n);               \
    } while (0)
    if (t.tf == DT_F64 && t.tx == DT_F64) TPT_THOMAS_LAUNCH(double, double);
    else if (t.tf == DT_F32 && t.tx == DT_F32) TPT_THOMAS_LAUNCH(float, float);
    else if (t.tf == DT_F64) TPT_THOMAS_LAUNCH(double, float);
    else TPT_THOMAS_LAUNCH(float, double);
#undef TPT_THOMAS_LAUNCH
    return hipGetLastError();
}

hipError_t launch_thomas_multi(const ThomasDesc* d_work, int nwork, long long total_blocks, int nz_max,
                               hipStream_t s) {
    if (total_blocks <= 0) return hipSuccess;
    const long long grid = std::min(total_blocks, 4 * PERSISTENT_BLOCKS);
    const size_t sm = THOMAS_LDS_PLANES * sizeof(double) * (size_t)nz_max;
    TPT_KLAUNCH(thomas_multi_kernel, dim3((unsigned)grid), dim3(THOMAS_NT), sm, s, d_work, nwork,
                       total_blocks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 residual of the 7-point operator (the Kronecker sum of §2.2.2 with the
// same boundary rows as the plan), r = f - A x, A = L or I - alpha L, with
// partial sums of r^2 and f^2 per block.
// ---------------------------------------------------------------------------
constexpr int RES_NT = 256;
constexpr int RES_RZ = 32;  // z planes per thread

// Blocks: 256 consecutive (i, j) columns times one chunk of RES_RZ planes.
int residual_blocks(const StencilDesc& st) {
    const int bc = st.pair ? 2 * RES_NT : RES_NT;
    const long long ncb = ((long long)st.nx * st.ny + bc - 1) / bc;
    const long long nzc = (st.nz + RES_RZ - 1) / RES_RZ;
    return (int)(ncb * nzc);
}

// Each thread marches up one column through RES_RZ planes, keeping the z
// neighbours in registers: per unknown it loads the next plane's value, f and
// the four x / y neighbours (cache hits), with the x / y coefficients of its
// column held in registers.  A missing neighbour (a wall) gets coefficient 0
// and offset 0, so the stencil needs no branches.
__device__ __forceinline__ void residual_block(const StencilDesc& st, long long lb, double* red, double* zco) {
    const int nx = st.nx, ny = st.ny, nz = st.nz;
    const long long sxy = (long long)nx * ny;
    const long long ncb = (sxy + RES_NT - 1) / RES_NT;
    const long long zc = lb / ncb, cbk = lb - zc * ncb;
    const long long c = cbk * RES_NT + threadIdx.x;  // column i + nx j
    // the z coefficients of the block's planes, staged in LDS once (read
    // inside the march, where a memory load per plane would wait each step)
    {
        const int k0 = (int)zc * RES_RZ;
        for (int t = threadIdx.x; t < 3 * RES_RZ; t += RES_NT) {
            const int q = t / RES_RZ, k = k0 + t % RES_RZ;
            double v = 0.0;
            if (k < nz) {
                if (q == 0) v = (k > 0 || st.perz) ? st.az[k] : 0.0;
                else if (q == 1) v = st.bz[k];
                else v = (k < nz - 1 || st.perz) ? st.cz[k] : 0.0;
            }
            zco[t] = v;
        }
        __syncthreads();
    }
    double sr = 0.0, sf = 0.0;
    if (c < sxy) {
        const int j = (int)(c / nx), i = (int)(c - (long long)j * nx);
        const double* __restrict__ x = st.x;
        // x / y neighbours: offsets (elements) and coefficients, 0 where absent
        long long oxm = 0, oxp = 0, oym = 0, oyp = 0;
        double axm = 0.0, axp = 0.0, aym = 0.0, ayp = 0.0;
        if (i > 0) { oxm = -1; axm = st.ax[i]; } else if (st.perx) { oxm = nx - 1; axm = st.ax[0]; }
        if (i < nx - 1) { oxp = 1; axp = st.cx[i]; } else if (st.perx) { oxp = -(long long)(nx - 1); axp = st.cx[nx - 1]; }
        if (j > 0) { oym = -nx; aym = st.ay[j]; } else if (st.pery) { oym = (long long)(ny - 1) * nx; aym = st.ay[0]; }
        if (j < ny - 1) { oyp = nx; ayp = st.cy[j]; } else if (st.pery) { oyp = -(long long)(ny - 1) * nx; ayp = st.cy[ny - 1]; }
        const double bxy = st.bx[i] + st.by[j];
        const int k0 = (int)zc * RES_RZ, k1 = min(nz, k0 + RES_RZ);
        // the incompatible part of f, removed from the last plane
        const double fshift = (st.wsum && k1 == nz) ? *st.wsum * st.wscale : 0.0;
        // z window: the value below k0 (or its periodic image) and at k0
        double xm = 0.0;
        if (k0 > 0) xm = x[(long long)(k0 - 1) * sxy + c];
        else if (st.perz) xm = x[(long long)(nz - 1) * sxy + c];
        double xc = x[(long long)k0 * sxy + c];
        for (int k = k0; k < k1; ++k) {
            const long long idx = (long long)k * sxy + c;
            double xp = 0.0;
            if (k + 1 < nz) xp = x[idx + sxy];
            else if (st.perz) xp = x[c];
            const double azk = zco[k - k0], czk = zco[2 * RES_RZ + k - k0];
            double lap = (bxy + zco[RES_RZ + k - k0]) * xc + azk * xm + czk * xp;
            lap += axm * x[idx + oxm] + axp * x[idx + oxp] + aym * x[idx + oym] + ayp * x[idx + oyp];
            const double ax = st.helmholtz ? xc - st.alpha * lap : lap;
            const double fv = st.f[idx] - (k == nz - 1 ? fshift : 0.0);
            const double r = fv - ax;
            st.r[idx] = (float)r;
            sr += r * r;
            sf += fv * fv;
            xm = xc;
            xc = xp;
        }
    }
    block_sum2<RES_NT>(sr, sf, red);
    if (threadIdx.x == 0 && st.partials) {
        st.partials[2 * lb] = sr;
        st.partials[2 * lb + 1] = sf;
    }
}

// Paired form (even nx, 16-byte aligned x and f, planes under 2 GB): each
// thread owns two neighbouring columns of one row, so its plane reads are
// 16-byte loads and a wave covers 128 columns.  The x neighbours inside the
// wave come from the neighbouring lanes' registers (the current plane's x is
// already held for the z stencil); only the lanes at a wave's ends or a row's
// ends load them.  Per plane a wave then issues four full-width loads (x one
// plane up, f, and the two y neighbours) instead of six half-width ones per
// 64 columns: the scalar march is bound by that load issue rate, not by HBM.
// Loads go through per-plane buffer descriptors (uniform) with 32-bit
// per-thread offsets.  Every lane runs the march (lanes past the last column
// work on the last pair and store nothing), so the cross-lane reads always
// find their source lane active.
typedef unsigned int res_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 res_ld2(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
__device__ __forceinline__ double res_ld1(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

__device__ __forceinline__ void residual_pair_block(const StencilDesc& st, long long lb, double* red, double* zco) {
    const int nx = st.nx, ny = st.ny, nz = st.nz;
    const long long sxy = (long long)nx * ny;
    constexpr int BC = 2 * RES_NT;  // columns per block
    const long long ncb = (sxy + BC - 1) / BC;
    const long long zc = lb / ncb, cbk = lb - zc * ncb;
    const int k0 = (int)zc * RES_RZ, k1 = min(nz, k0 + RES_RZ);
    {
        for (int t = threadIdx.x; t < 3 * RES_RZ; t += RES_NT) {
            const int q = t / RES_RZ, k = k0 + t % RES_RZ;
            double v = 0.0;
            if (k < nz) {
                if (q == 0) v = (k > 0 || st.perz) ? st.az[k] : 0.0;
                else if (q == 1) v = st.bz[k];
                else v = (k < nz - 1 || st.perz) ? st.cz[k] : 0.0;
            }
            zco[t] = v;
        }
        __syncthreads();
    }
    const long long c_raw = cbk * BC + 2 * (long long)threadIdx.x;
    const bool live = c_raw < sxy;
    const int c = (int)(live ? c_raw : sxy - 2);  // column of the pair's first element (sxy < 2^28 here)
    const int j = c / nx, i0 = c - j * nx, i1 = i0 + 1;
    const int lane = threadIdx.x & 63;
    // x neighbours outside the pair: from the neighbouring lane, or loaded at
    // a wave end or a row end (the wrap of a periodic row; a wall has
    // coefficient 0 and re-reads the own column)
    const double axm0 = i0 > 0 ? st.ax[i0] : (st.perx ? st.ax[0] : 0.0);
    const double axp0 = st.cx[i0];
    const double axm1 = st.ax[i1];
    const double axp1 = i1 < nx - 1 ? st.cx[i1] : (st.perx ? st.cx[nx - 1] : 0.0);
    const bool loadL = lane == 0 || i0 == 0, loadR = lane == 63 || i1 == nx - 1 || c_raw + 2 >= sxy;
    const int colL = i0 > 0 ? c - 1 : (st.perx ? c + nx - 1 : c);
    const int colR = i1 < nx - 1 ? c + 2 : (st.perx ? c + 2 - nx : c + 1);
    int cym = c, cyp = c;
    double aym = 0.0, ayp = 0.0;
    if (j > 0) { cym = c - nx; aym = st.ay[j]; } else if (st.pery) { cym = c + (ny - 1) * nx; aym = st.ay[0]; }
    if (j < ny - 1) { cyp = c + nx; ayp = st.cy[j]; } else if (st.pery) { cyp = c - (ny - 1) * nx; ayp = st.cy[ny - 1]; }
    const double bxy0 = st.bx[i0] + st.by[j], bxy1 = st.bx[i1] + st.by[j];
    const double fshift = (st.wsum && k1 == nz) ? *st.wsum * st.wscale : 0.0;
    const int pbytes = (int)(sxy * 8);
    auto rsrc = [&](const void* base, int bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
    };
    const unsigned oc = (unsigned)c * 8u, ocym = (unsigned)cym * 8u, ocyp = (unsigned)cyp * 8u;
    const unsigned oL = (unsigned)colL * 8u, oR = (unsigned)colR * 8u;
    // z window: the pair below k0 (or its periodic image, or 0) and at k0
    double2 xm = make_double2(0.0, 0.0);
    if (k0 > 0) xm = res_ld2(rsrc(st.x + (long long)(k0 - 1) * sxy, pbytes), oc);
    else if (st.perz) xm = res_ld2(rsrc(st.x + (long long)(nz - 1) * sxy, pbytes), oc);
    double2 xc = res_ld2(rsrc(st.x + (long long)k0 * sxy, pbytes), oc);
    double sr = 0.0, sf = 0.0;
    for (int k = k0; k < k1; ++k) {
        const double* xk = st.x + (long long)k * sxy;
        const __amdgpu_buffer_rsrc_t rx = rsrc(xk, pbytes);
        const double2 xq = res_ld2(rsrc(k + 1 < nz ? xk + sxy : st.x, pbytes), oc);
        const double2 fv = res_ld2(rsrc(st.f + (long long)k * sxy, pbytes), oc);
        const double2 ym = res_ld2(rx, ocym), yp = res_ld2(rx, ocyp);
        double xl = __shfl_up(xc.y, 1, 64), xr = __shfl_down(xc.x, 1, 64);
        if (loadL) xl = res_ld1(rx, oL);
        if (loadR) xr = res_ld1(rx, oR);
        const double2 xp = (k + 1 < nz || st.perz) ? xq : make_double2(0.0, 0.0);
        const double azk = zco[k - k0], bzk = zco[RES_RZ + k - k0], czk = zco[2 * RES_RZ + k - k0];
        double lap0 = (bxy0 + bzk) * xc.x + azk * xm.x + czk * xp.x;
        lap0 += axm0 * xl + axp0 * xc.y + aym * ym.x + ayp * yp.x;
        double lap1 = (bxy1 + bzk) * xc.y + azk * xm.y + czk * xp.y;
        lap1 += axm1 * xc.x + axp1 * xr + aym * ym.y + ayp * yp.y;
        const double ax0 = st.helmholtz ? xc.x - st.alpha * lap0 : lap0;
        const double ax1 = st.helmholtz ? xc.y - st.alpha * lap1 : lap1;
        const double sh = k == nz - 1 ? fshift : 0.0;
        const double f0 = fv.x - sh, f1 = fv.y - sh;
        const double r0 = f0 - ax0, r1 = f1 - ax1;
        if (live) {
            const float2 rv = make_float2((float)r0, (float)r1);
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(res_u32x2, rv),
                                                  rsrc(st.r + (long long)k * sxy, pbytes / 2), (int)(oc / 2u), 0, 0);
            sr += r0 * r0 + r1 * r1;
            sf += f0 * f0 + f1 * f1;
        }
        xm = xc;
        xc = xp;
    }
    block_sum2<RES_NT>(sr, sf, red);
    if (threadIdx.x == 0 && st.partials) {
        st.partials[2 * lb] = sr;
        st.partials[2 * lb + 1] = sf;
    }
}

__global__ __launch_bounds__(RES_NT) void residual_kernel(StencilDesc st) {
    __shared__ double red[2 * RES_NT / 64];
    __shared__ double zco[3 * RES_RZ];
    // consecutive logical blocks (neighbouring rows of one z chunk, whose y
    // neighbours they read) share one XCD's L2
    residual_block(st, xcd_block(blockIdx.x, gridDim.x), red, zco);
}

__global__ __launch_bounds__(RES_NT) void residual_pair_kernel(StencilDesc st) {
    __shared__ double red[2 * RES_NT / 64];
    __shared__ double zco[3 * RES_RZ];
    residual_pair_block(st, xcd_block(blockIdx.x, gridDim.x), red, zco);
}

__global__ __launch_bounds__(RES_NT) void residual_multi_kernel(const StencilDesc* __restrict__ work, int nwork,
                                                                long long total) {
    __shared__ double red[2 * RES_NT / 64];
    __shared__ double zco[3 * RES_RZ];
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const StencilDesc st = work[lo];
        const long long lb = blk - st.block_begin;
        if (st.pair) residual_pair_block(st, lb, red, zco);
        else residual_block(st, lb, red, zco);
        __syncthreads();
    }
}

bool residual_pairs_ok(const StencilDesc& st) {
    const long long sxy = (long long)st.nx * st.ny;
    return st.nx % 2 == 0 && sxy >= 2 && sxy * 8 < (1LL << 31) && ((uintptr_t)st.x % 16) == 0 &&
           ((uintptr_t)st.f % 16) == 0 && ((uintptr_t)st.r % 8) == 0;
}

hipError_t launch_residual(const StencilDesc& st, hipStream_t s) {
    const int nb = residual_blocks(st);
    if (nb <= 0) return hipSuccess;
    if (st.pair) TPT_KLAUNCH(residual_pair_kernel, dim3(nb), dim3(RES_NT), 0, s, st);
    else TPT_KLAUNCH(residual_kernel, dim3(nb), dim3(RES_NT), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_residual_multi(const StencilDesc* d_work, int nwork, long long total_blocks, hipStream_t s) {
    if (total_blocks <= 0) return hipSuccess;
    TPT_KLAUNCH(residual_multi_kernel, dim3((unsigned)std::min(total_blocks, 4 * PERSISTENT_BLOCKS)),
                       dim3(RES_NT), 0, s, d_work, nwork, total_blocks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic pair reduction (fixed assignment of partials to threads and a
// fixed tree): one block per reduction.
// ---------------------------------------------------------------------------
constexpr int RED_NT = 1024;

__device__ __forceinline__ void reduce_pairs_block(const double* p, int n, double* out, double* red) {
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += RED_NT) {
        a += p[2 * i];
        b += p[2 * i + 1];
    }
    block_sum2<RED_NT>(a, b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

__global__ __launch_bounds__(RED_NT) void reduce_pairs_kernel(const double* p, int n, double* out) {
    __shared__ double red[2 * RED_NT / 64];
    reduce_pairs_block(p, n, out, red);
}

__global__ __launch_bounds__(RED_NT) void reduce_pairs_multi_kernel(const ReduceDesc* work, int nwork) {
    __shared__ double red[2 * RED_NT / 64];
    const ReduceDesc d = work[blockIdx.x];
    reduce_pairs_block(d.partials, d.n, d.out, red);
}

hipError_t launch_reduce_pairs(const double* partials, int n, double* out, hipStream_t s) {
    TPT_KLAUNCH(reduce_pairs_kernel, dim3(1), dim3(RED_NT), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_reduce_pairs_multi(const ReduceDesc* d_work, int nwork, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    TPT_KLAUNCH(reduce_pairs_multi_kernel, dim3(nwork), dim3(RED_NT), 0, s, d_work, nwork);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Right-hand-side check: volume-weighted sums (for the compatibility defect
// of a singular problem) and the count of non-finite values.  A block covers
// CHK_ROWS consecutive x-lines (rows (j, k)) of one field as 64 columns x 4
// row lanes: lane (c, r) visits columns i = c + 64 a and rows r + 4 b, so a
// wave reads 512 contiguous bytes of one row per access, holds vx_i in a
// register across its rows and forms vy_j vz_k once per row; the CHK_ROWS / 4
// loads of a column are independent and issued together.
// ---------------------------------------------------------------------------
constexpr int CHK_NT = 256;
constexpr int CHK_ROWS = 32;

__host__ __device__ inline long long check_blocks_of(const CheckDesc& c) {
    const long long rows = (long long)c.ny * c.nz;
    return (rows + CHK_ROWS - 1) / CHK_ROWS;
}
long long check_blocks(const CheckDesc& c) { return check_blocks_of(c); }

__device__ __forceinline__ void check_block(const CheckDesc& c, int sys, long long lb, long long nb, double* red) {
    const int nx = c.nx, ny = c.ny;
    const long long rows = (long long)ny * c.nz;
    const double* __restrict__ f = c.f + (long long)sys * rows * nx;
    const int col = threadIdx.x & 63, rl = threadIdx.x >> 6;
    const long long r0 = lb * CHK_ROWS + rl;
    // the rows of this lane and their y-z weights (0 past the last row)
    double wyz[CHK_ROWS / 4];
    long long roff[CHK_ROWS / 4];
#pragma unroll
    for (int b = 0; b < CHK_ROWS / 4; ++b) {
        const long long row = r0 + 4 * b;
        const bool in = row < rows;
        const long long rr = in ? row : 0;
        const int k = (int)(rr / ny), j = (int)(rr - (long long)k * ny);
        wyz[b] = in ? c.vy[j] * c.vz[k] : 0.0;
        roff[b] = rr * nx;
    }
    double s = 0.0, a = 0.0, bad = 0.0;
    for (int i = col; i < nx; i += 64) {
        const double wx = c.vx[i];
        double v[CHK_ROWS / 4];
#pragma unroll
        for (int b = 0; b < CHK_ROWS / 4; ++b) v[b] = f[roff[b] + i];
#pragma unroll
        for (int b = 0; b < CHK_ROWS / 4; ++b) {
            const bool live = wyz[b] != 0.0;
            const bool fin = __builtin_isfinite(v[b]);
            const double w = wx * wyz[b];
            s += fin ? w * v[b] : 0.0;
            a += fin ? w * __builtin_fabs(v[b]) : 0.0;
            bad += (live && !fin) ? 1.0 : 0.0;
        }
    }
    double zero = 0.0;
    block_sum2<CHK_NT>(s, a, red);
    block_sum2<CHK_NT>(bad, zero, red);
    if (threadIdx.x == 0) {
        double* p = c.partials + 4 * ((long long)sys * nb + lb);
        p[0] = s;
        p[1] = a;
        p[2] = bad;
        p[3] = 0.0;
    }
}

__global__ __launch_bounds__(CHK_NT) void check_kernel(CheckDesc c, long long nb) {
    __shared__ double red[2 * CHK_NT / 64];
    check_block(c, blockIdx.y, blockIdx.x, nb, red);
}

__global__ __launch_bounds__(CHK_NT) void check_multi_kernel(const CheckDesc* __restrict__ work, int nwork,
                                                             long long total) {
    __shared__ double red[2 * CHK_NT / 64];
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const CheckDesc c = work[lo];
        check_block(c, 0, blk - c.block_begin, check_blocks_of(c), red);
        __syncthreads();
    }
}

// Fold the nb partials of field `sys` in a fixed order.
__device__ __forceinline__ void check_reduce_block(const CheckDesc& c, int sys, long long nb, double* red) {
    const double* p = c.partials + 4 * (long long)sys * nb;
    double s = 0.0, a = 0.0, bad = 0.0, zero = 0.0;
    for (long long b = threadIdx.x; b < nb; b += RED_NT) {
        s += p[4 * b];
        a += p[4 * b + 1];
        bad += p[4 * b + 2];
    }
    block_sum2<RED_NT>(s, a, red);
    block_sum2<RED_NT>(bad, zero, red);
    if (threadIdx.x == 0) {
        double* o = c.out + (long long)sys * c.out_stride;
        o[0] = s;
        o[1] = a;
        o[2] = bad;
    }
}

__global__ __launch_bounds__(RED_NT) void check_reduce_kernel(CheckDesc c, long long nb) {
    __shared__ double red[2 * RED_NT / 64];
    check_reduce_block(c, blockIdx.x, nb, red);
}

__global__ __launch_bounds__(RED_NT) void check_reduce_multi_kernel(const CheckDesc* __restrict__ work) {
    __shared__ double red[2 * RED_NT / 64];
    const CheckDesc c = work[blockIdx.x];
    check_reduce_block(c, 0, c.nblk > 0 ? c.nblk : check_blocks_of(c), red);
}

hipError_t launch_check(const CheckDesc& c, hipStream_t s) {
    const long long nb = check_blocks(c);
    if (nb <= 0 || c.nsys < 1) return hipSuccess;
    TPT_KLAUNCH(check_kernel, dim3((unsigned)nb, (unsigned)c.nsys), dim3(CHK_NT), 0, s, c, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TPT_KLAUNCH(check_reduce_kernel, dim3((unsigned)c.nsys), dim3(RED_NT), 0, s, c, nb);
    return hipGetLastError();
}

hipError_t launch_check_reduce(const CheckDesc& c, long long nb, hipStream_t s) {
    if (nb <= 0 || c.nsys < 1) return hipSuccess;
    TPT_KLAUNCH(check_reduce_kernel, dim3((unsigned)c.nsys), dim3(RED_NT), 0, s, c, nb);
    return hipGetLastError();
}

hipError_t launch_check_reduce_multi(const CheckDesc* d_work, int nwork, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    TPT_KLAUNCH(check_reduce_multi_kernel, dim3((unsigned)nwork), dim3(RED_NT), 0, s, d_work);
    return hipGetLastError();
}

hipError_t launch_check_multi(const CheckDesc* d_work, int nwork, long long total_blocks, hipStream_t s) {
    if (nwork <= 0 || total_blocks <= 0) return hipSuccess;
    TPT_KLAUNCH(check_multi_kernel, dim3((unsigned)std::min(total_blocks, 4 * PERSISTENT_BLOCKS)), dim3(CHK_NT), 0,
                s, d_work, nwork, total_blocks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    TPT_KLAUNCH(check_reduce_multi_kernel, dim3((unsigned)nwork), dim3(RED_NT), 0, s, d_work);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Elementwise conversions.
// ---------------------------------------------------------------------------
__global__ void split_bf16_kernel(const float* x, uint16_t* hi, uint16_t* lo, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        uint16_t h, l;
        split_bf16(x[i], h, l);
        hi[i] = h;
        lo[i] = l;
    }
}

__global__ void convert_kernel(const double* x, float* y, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

hipError_t launch_split_bf16(const float* x, uint16_t* hi, uint16_t* lo, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    TPT_KLAUNCH(split_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, hi, lo, n);
    return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* x, float* y, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    TPT_KLAUNCH(convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace tpt
