// HIP kernels for gfx950 (CDNA4): eigenbasis-transform GEMMs on MFMA,
// lane-per-line batched Thomas, FP64 7-point residual, reductions.
//
// Layout of every field: u[k][j][i], x fastest.  The x transform is a GEMM
// whose rows are the N_y N_z x-lines (A = field, K = N_x contiguous) and whose
// B is the basis (end of §2.2.2: all lines stacked into one GEMM).  The y
// transform is a strided batch over z slabs of a left multiplication by the
// basis (A = basis, B = slab with x contiguous), so no transpose is needed.
#include "kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace tpt {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

const char* tile_variant_name(int v) {
    static const char* names[TV_COUNT] = {"128x128", "64x128", "128x64", "64x64", "32x64"};
    return (v >= 0 && v < TV_COUNT) ? names[v] : "?";
}

void tile_variant_shape(int v, int* bm, int* bn) {
    static const int s[TV_COUNT][2] = {{128, 128}, {64, 128}, {128, 64}, {64, 64}, {32, 64}};
    *bm = s[v][0];
    *bn = s[v][1];
}

static inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

long long gemm_blocks(const GemmDesc& g, int variant) {
    int bm, bn;
    tile_variant_shape(variant, &bm, &bn);
    return (long long)cdiv(g.M, bm) * cdiv(g.N, bn) * g.batch;
}

// ---------------------------------------------------------------------------
// Wave-level helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum (a, b) over the block in a fixed order; thread 0 gets the result.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            sa += red[2 * i];
            sb += red[2 * i + 1];
        }
        a = sa;
        b = sb;
    }
}

template <typename T>
__device__ __forceinline__ T load_as(const void* p, long long i, int dtype) {
    if (dtype == DT_F64) return (T)(((const double*)p)[i]);
    return (T)(((const float*)p)[i]);
}

// ---------------------------------------------------------------------------
// FP64 / FP32 MFMA GEMM tile (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32).
// Operand fragments: lane l holds A[m0 + l%16][k0 + l/16] and
// B[k0 + l/16][n0 + l%16]; the 16x16 result of lane l is column l%16, rows
// l/16 + 4r (f64) or 4(l/16) + r (f32), r = 0..3.
// Tiles of A and B are staged through LDS (double-buffered, BK = 16).
// ---------------------------------------------------------------------------
template <typename TM> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc zero() { return (acc){0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result element r of lane l is row l/16 + 4 r (measured on gfx950)
    static __device__ __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc zero() { return (acc){0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result element r of lane l is row 4 (l/16) + r
    static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
};

template <int BM, int BN> struct TileCfg {
    static constexpr int WM = BM >= 64 ? 64 : 32;
    static constexpr int WN = BN >= 64 ? 64 : BN;
    static constexpr int WAVES_M = BM / WM;
    static constexpr int WAVES_N = BN / WN;
    static constexpr int NT = WAVES_M * WAVES_N * 64;
    static constexpr int MI = WM / 16;
    static constexpr int NI = WN / 16;
};

template <typename TM, int BM, int BN, bool BNK> struct SmemF {
    static constexpr int BK = 16;
    static constexpr int PA = BK + 1;
    static constexpr int PB = BNK ? BK + 1 : BN + 2;
    static constexpr int A_ELEMS = BM * PA;
    static constexpr int B_ELEMS = BNK ? BN * PB : BK * PB;
    static constexpr int TOTAL = 2 * (A_ELEMS + B_ELEMS);
};

// Decode a block of a descriptor into (batch, tile_m, tile_n).
__device__ __forceinline__ void decode_tile(const GemmDesc& g, long long lb, int& b, int& tm, int& tn) {
    const long long per = (long long)g.tiles_m * g.tiles_n;
    b = (int)(lb / per);
    const int rem = (int)(lb - (long long)b * per);
    tm = rem / g.tiles_n;
    tn = rem - tm * g.tiles_n;
}

template <typename TM, int BM, int BN, bool BNK>
__device__ __forceinline__ void gemm_tile_f(const GemmDesc& g, long long lb, long long gblock, TM* smem,
                                            double* red) {
    typedef TileCfg<BM, BN> C;
    typedef SmemF<TM, BM, BN, BNK> S;
    typedef Mfma<TM> MM;
    constexpr int BK = S::BK;
    constexpr int NT = C::NT;
    constexpr int LA = BM * BK / NT;  // A elements loaded per thread per K tile
    constexpr int LB = BN * BK / NT;
    TM* As = smem;
    TM* Bs = smem + 2 * S::A_ELEMS;

    int b, tm, tn;
    decode_tile(g, lb, b, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x;
    const int w = tid / 64, l = tid % 64, lr = l % 16, lg = l / 16;
    const int wm = w / C::WAVES_N, wn = w % C::WAVES_N;
    const long long offA = (long long)b * g.sA, offB = (long long)b * g.sB, offC = (long long)b * g.sC;

    typename MM::acc acc[C::MI][C::NI];
#pragma unroll
    for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::zero();

    TM ra[LA], rb[LB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int t = 0; t < LA; ++t) {
            const int e = tid + NT * t;
            const int row = e / BK, col = e % BK;
            const int m = m0 + row, k = k0 + col;
            ra[t] = (m < g.M && k < g.K) ? load_as<TM>(g.A, offA + (long long)m * g.lda + k, g.tA) : (TM)0;
        }
#pragma unroll
        for (int t = 0; t < LB; ++t) {
            const int e = tid + NT * t;
            if (BNK) {
                const int row = e / BK, col = e % BK;  // row over n, col over k
                const int n = n0 + row, k = k0 + col;
                rb[t] = (n < g.N && k < g.K) ? load_as<TM>(g.B, offB + (long long)n * g.ldb + k, g.tB) : (TM)0;
            } else {
                const int row = e / BN, col = e % BN;  // row over k, col over n
                const int n = n0 + col, k = k0 + row;
                rb[t] = (n < g.N && k < g.K) ? load_as<TM>(g.B, offB + (long long)k * g.ldb + n, g.tB) : (TM)0;
            }
        }
    };
    auto sstore = [&](int buf) {
        TM* a = As + buf * S::A_ELEMS;
        TM* bb = Bs + buf * S::B_ELEMS;
#pragma unroll
        for (int t = 0; t < LA; ++t) {
            const int e = tid + NT * t;
            a[(e / BK) * S::PA + (e % BK)] = ra[t];
        }
#pragma unroll
        for (int t = 0; t < LB; ++t) {
            const int e = tid + NT * t;
            if (BNK) bb[(e / BK) * S::PB + (e % BK)] = rb[t];
            else bb[(e / BN) * S::PB + (e % BN)] = rb[t];
        }
    };

    const int nk = (g.K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const TM* a = As + cur * S::A_ELEMS;
        const TM* bb = Bs + cur * S::B_ELEMS;
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            const int k = kk * 4 + lg;
            TM fa[C::MI], fb[C::NI];
#pragma unroll
            for (int i = 0; i < C::MI; ++i) fa[i] = a[(wm * C::WM + i * 16 + lr) * S::PA + k];
#pragma unroll
            for (int j = 0; j < C::NI; ++j)
                fb[j] = BNK ? bb[(wn * C::WN + j * 16 + lr) * S::PB + k] : bb[k * S::PB + wn * C::WN + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < C::MI; ++i)
#pragma unroll
                for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::mma(fa[i], fb[j], acc[i][j]);
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    // epilogue
    double se = 0.0, sx = 0.0;
#pragma unroll
    for (int i = 0; i < C::MI; ++i) {
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int n = n0 + wn * C::WN + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * C::WM + i * 16 + MM::row(lg, r);
                if (m < g.M && n < g.N) {
                    const long long idx = offC + (long long)m * g.ldc + n;
                    const double v = (double)acc[i][j][r];
                    if (g.epi == EPI_ACCUM_F64) {
                        double* cp = (double*)g.C;
                        const double x = cp[idx] + v;
                        cp[idx] = x;
                        se += v * v;
                        sx += x * x;
                    } else if (g.tC == DT_F64) {
                        ((double*)g.C)[idx] = v;
                    } else {
                        ((float*)g.C)[idx] = (float)acc[i][j][r];
                    }
                }
            }
        }
    }
    if (g.epi == EPI_ACCUM_F64) {
        block_sum2<NT>(se, sx, red);
        if (threadIdx.x == 0) {
            g.partials[2 * gblock] = se;
            g.partials[2 * gblock + 1] = sx;
        }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 x3 MFMA GEMM tile (v_mfma_f32_16x16x32_bf16, FP32 accumulate):
// each operand is x = hi + lo with hi = bf16(x), lo = bf16(x - hi) (round to
// nearest even); C = A_hi B_hi + A_hi B_lo + A_lo B_hi, small products first.
// Fragments: lane l holds A[m0 + l%16][k0 + 8(l/16) .. +7] and
// B[k0 + 8(l/16) .. +7][n0 + l%16]; LDS tiles are stored k-contiguous for both
// operands (As[m][k], Bs[n][k]) so each fragment is one 16-byte LDS read.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_to_f(hi));
}

template <int BM, int BN> struct SmemB {
    static constexpr int BK = 32;
    static constexpr int P = BK + 8;  // row stride in bf16 (16-byte padding)
    static constexpr int A_ELEMS = BM * P;
    static constexpr int B_ELEMS = BN * P;
    // [2 buffers][hi, lo][A | B]
    static constexpr int TOTAL = 2 * 2 * (A_ELEMS + B_ELEMS);
};

template <int BM, int BN, bool BNK>
__device__ __forceinline__ void gemm_tile_b(const GemmDesc& g, long long lb, long long gblock, uint16_t* smem,
                                            double* red) {
    typedef TileCfg<BM, BN> C;
    typedef SmemB<BM, BN> S;
    constexpr int BK = S::BK;
    constexpr int NT = C::NT;
    constexpr int P = S::P;
    // A tile: BM x BK in chunks of 8 k; B tile: BN x BK in chunks of 8 k
    constexpr int CA = BM * BK / 8 / NT;   // 8-element chunks of A per thread
    constexpr int CB = BN * BK / 8 / NT;
    static_assert(CA >= 1 && CB >= 1, "tile too small for the thread count");
    uint16_t* sm_hi = smem;                       // [2][A_ELEMS + B_ELEMS]
    uint16_t* sm_lo = smem + 2 * (S::A_ELEMS + S::B_ELEMS);

    int b, tm, tn;
    decode_tile(g, lb, b, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x;
    const int w = tid / 64, l = tid % 64, lr = l % 16, lg = l / 16;
    const int wm = w / C::WAVES_N, wn = w % C::WAVES_N;
    const long long offA = (long long)b * g.sA, offB = (long long)b * g.sB, offC = (long long)b * g.sC;

    f4 acc[C::MI][C::NI];
#pragma unroll
    for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

    // register staging: hi/lo chunks of 8 bf16 for A and B
    u16x8 rah[CA], ral[CA], rbh[CB], rbl[CB];

    // Load an 8-element k-chunk of row `row` (m or n) of an operand stored
    // [row][k] (k contiguous): either the pre-split basis or data to split.
    auto load_rowk = [&](bool is_basis, const void* data, int dtype, long long off, int ld, int nrows, int row,
                         int k, u16x8& h, u16x8& lo) {
        if (is_basis) {
            const long long base = off + (long long)row * ld + k;
            const bool full = row < nrows && k + 8 <= g.K && ((base & 7) == 0);
            if (full) {
                h = *(const u16x8*)(g.basis_hi + base);
                lo = *(const u16x8*)(g.basis_lo + base);
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const bool ok = row < nrows && k + e < g.K;
                    h[e] = ok ? g.basis_hi[base + e] : (uint16_t)0;
                    lo[e] = ok ? g.basis_lo[base + e] : (uint16_t)0;
                }
            }
        } else {
            const long long base = off + (long long)row * ld + k;
            float v[8];
            if (dtype == DT_F32 && row < nrows && k + 8 <= g.K && ((base & 3) == 0)) {
                const float4 p0 = *(const float4*)((const float*)data + base);
                const float4 p1 = *(const float4*)((const float*)data + base + 4);
                v[0] = p0.x; v[1] = p0.y; v[2] = p0.z; v[3] = p0.w;
                v[4] = p1.x; v[5] = p1.y; v[6] = p1.z; v[7] = p1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    v[e] = (row < nrows && k + e < g.K) ? load_as<float>(data, base + e, dtype) : 0.f;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                uint16_t hh, ll;
                split_bf16(v[e], hh, ll);
                h[e] = hh;
                lo[e] = ll;
            }
        }
    };

    auto gload = [&](int k0) {
        // A: BM rows x BK, chunk c -> row = c / (BK/8), kc = c % (BK/8)
#pragma unroll
        for (int t = 0; t < CA; ++t) {
            const int c = tid + NT * t;
            const int row = c / (BK / 8), kc = c % (BK / 8);
            load_rowk(g.basis_is_A != 0, g.A, g.tA, offA, g.lda, g.M, m0 + row, k0 + kc * 8, rah[t], ral[t]);
        }
        if (BNK) {
#pragma unroll
            for (int t = 0; t < CB; ++t) {
                const int c = tid + NT * t;
                const int row = c / (BK / 8), kc = c % (BK / 8);
                load_rowk(g.basis_is_A == 0, g.B, g.tB, offB, g.ldb, g.N, n0 + row, k0 + kc * 8, rbh[t], rbl[t]);
            }
        } else {
            // B stored [k][n] (data slab): chunk c covers n = c % BN, k = 8*(c / BN) .. +7
#pragma unroll
            for (int t = 0; t < CB; ++t) {
                const int c = tid + NT * t;
                const int nn = c % BN, kc = c / BN;
                const int n = n0 + nn;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = k0 + kc * 8 + e;
                    const float v = (n < g.N && k < g.K) ? load_as<float>(g.B, offB + (long long)k * g.ldb + n, g.tB) : 0.f;
                    uint16_t hh, ll;
                    split_bf16(v, hh, ll);
                    rbh[t][e] = hh;
                    rbl[t][e] = ll;
                }
            }
        }
    };
    auto sstore = [&](int buf) {
        uint16_t* ah = sm_hi + buf * (S::A_ELEMS + S::B_ELEMS);
        uint16_t* al = sm_lo + buf * (S::A_ELEMS + S::B_ELEMS);
#pragma unroll
        for (int t = 0; t < CA; ++t) {
            const int c = tid + NT * t;
            const int row = c / (BK / 8), kc = c % (BK / 8);
            *(u16x8*)(ah + row * P + kc * 8) = rah[t];
            *(u16x8*)(al + row * P + kc * 8) = ral[t];
        }
        uint16_t* bh = ah + S::A_ELEMS;
        uint16_t* bl = al + S::A_ELEMS;
#pragma unroll
        for (int t = 0; t < CB; ++t) {
            const int c = tid + NT * t;
            int row, kc;
            if (BNK) {
                row = c / (BK / 8);
                kc = c % (BK / 8);
            } else {
                row = c % BN;
                kc = c / BN;
            }
            *(u16x8*)(bh + row * P + kc * 8) = rbh[t];
            *(u16x8*)(bl + row * P + kc * 8) = rbl[t];
        }
    };

    const int nk = (g.K + BK - 1) / BK;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload((kt + 1) * BK);
        const uint16_t* ah = sm_hi + cur * (S::A_ELEMS + S::B_ELEMS);
        const uint16_t* al = sm_lo + cur * (S::A_ELEMS + S::B_ELEMS);
        const uint16_t* bh = ah + S::A_ELEMS;
        const uint16_t* bl = al + S::A_ELEMS;
        bf16x8 fah[C::MI], fal[C::MI], fbh[C::NI], fbl[C::NI];
#pragma unroll
        for (int i = 0; i < C::MI; ++i) {
            const int row = wm * C::WM + i * 16 + lr;
            fah[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)(ah + row * P + lg * 8));
            fal[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)(al + row * P + lg * 8));
        }
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int row = wn * C::WN + j * 16 + lr;
            fbh[j] = __builtin_bit_cast(bf16x8, *(const u16x8*)(bh + row * P + lg * 8));
            fbl[j] = __builtin_bit_cast(bf16x8, *(const u16x8*)(bl + row * P + lg * 8));
        }
#pragma unroll
        for (int i = 0; i < C::MI; ++i)
#pragma unroll
            for (int j = 0; j < C::NI; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], acc[i][j], 0, 0, 0);
            }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }

    double se = 0.0, sx = 0.0;
#pragma unroll
    for (int i = 0; i < C::MI; ++i) {
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int n = n0 + wn * C::WN + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * C::WM + i * 16 + 4 * lg + r;
                if (m < g.M && n < g.N) {
                    const long long idx = offC + (long long)m * g.ldc + n;
                    if (g.epi == EPI_ACCUM_F64) {
                        double* cp = (double*)g.C;
                        const double v = (double)acc[i][j][r];
                        const double x = cp[idx] + v;
                        cp[idx] = x;
                        se += v * v;
                        sx += x * x;
                    } else if (g.tC == DT_F64) {
                        ((double*)g.C)[idx] = (double)acc[i][j][r];
                    } else {
                        ((float*)g.C)[idx] = acc[i][j][r];
                    }
                }
            }
        }
    }
    if (g.epi == EPI_ACCUM_F64) {
        block_sum2<NT>(se, sx, red);
        if (threadIdx.x == 0) {
            g.partials[2 * gblock] = se;
            g.partials[2 * gblock + 1] = sx;
        }
    }
}

// ---------------------------------------------------------------------------
// GEMM kernels: one descriptor, or a work list of descriptors (one launch
// for many independent problems; a block finds its problem by binary search
// on block_begin).
// ---------------------------------------------------------------------------
template <int PREC> struct PrecT;
template <> struct PrecT<GP_F64> { typedef double T; };
template <> struct PrecT<GP_F32> { typedef float T; };

template <int PREC, int BM, int BN, bool BNK>
__device__ __forceinline__ void gemm_dispatch_tile(const GemmDesc& g, long long lb, long long gblock) {
    if constexpr (PREC == GP_BF16X3) {
        __shared__ __attribute__((aligned(16))) uint16_t smem[SmemB<BM, BN>::TOTAL];
        __shared__ double red[2 * TileCfg<BM, BN>::NT / 64];
        gemm_tile_b<BM, BN, BNK>(g, lb, gblock, smem, red);
    } else {
        typedef typename PrecT<PREC>::T T;
        __shared__ __attribute__((aligned(16))) T smem[SmemF<T, BM, BN, BNK>::TOTAL];
        __shared__ double red[2 * TileCfg<BM, BN>::NT / 64];
        gemm_tile_f<T, BM, BN, BNK>(g, lb, gblock, smem, red);
    }
}

template <int PREC, int BM, int BN, bool BNK>
__global__ __launch_bounds__((TileCfg<BM, BN>::NT)) void gemm_kernel(GemmDesc g) {
    gemm_dispatch_tile<PREC, BM, BN, BNK>(g, blockIdx.x, blockIdx.x);
}

// Persistent multi-problem kernel: blocks loop over the tiles of every work
// item; partial sums are indexed by the tile's block within its own problem.
template <int PREC, int BM, int BN, bool BNK>
__global__ __launch_bounds__((TileCfg<BM, BN>::NT)) void gemm_multi_kernel(const GemmDesc* __restrict__ work,
                                                                            int nwork, long long total) {
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {  // last work item with block_begin <= blk
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const GemmDesc g = work[lo];
        const long long lb = blk - g.block_begin;
        gemm_dispatch_tile<PREC, BM, BN, BNK>(g, lb, lb);
        __syncthreads();
    }
}

constexpr long long PERSISTENT_BLOCKS = 2048;

template <int PREC, bool BNK>
static hipError_t launch_gemm_v(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks,
                                int variant, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
#define TPT_LAUNCH(BM_, BN_)                                                                               \
    do {                                                                                                   \
        constexpr int NT_ = TileCfg<BM_, BN_>::NT;                                                         \
        if (d_work)                                                                                        \
            hipLaunchKernelGGL((gemm_multi_kernel<PREC, BM_, BN_, BNK>),                                   \
                               dim3((unsigned)std::min(blocks, PERSISTENT_BLOCKS)), dim3(NT_), 0, s, d_work, \
                               nwork, blocks);                                                             \
        else                                                                                               \
            hipLaunchKernelGGL((gemm_kernel<PREC, BM_, BN_, BNK>), dim3((unsigned)blocks), dim3(NT_), 0, s, \
                               g);                                                                         \
    } while (0)
    switch (variant) {
        case TV_128x128: TPT_LAUNCH(128, 128); break;
        case TV_64x128: TPT_LAUNCH(64, 128); break;
        case TV_128x64: TPT_LAUNCH(128, 64); break;
        case TV_64x64: TPT_LAUNCH(64, 64); break;
        case TV_32x64: TPT_LAUNCH(32, 64); break;
        default: return hipErrorInvalidValue;
    }
#undef TPT_LAUNCH
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_gemm_p(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks,
                                int variant, int b_nk, hipStream_t s) {
    return b_nk ? launch_gemm_v<PREC, true>(g, d_work, nwork, blocks, variant, s)
                : launch_gemm_v<PREC, false>(g, d_work, nwork, blocks, variant, s);
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
        case GP_F64: return launch_gemm_p<GP_F64>(g, nullptr, 0, blocks, variant, g.b_nk, s);
        case GP_F32: return launch_gemm_p<GP_F32>(g, nullptr, 0, blocks, variant, g.b_nk, s);
        case GP_BF16X3: return launch_gemm_p<GP_BF16X3>(g, nullptr, 0, blocks, variant, g.b_nk, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gemm_multi(const GemmDesc* d_work, int nwork, long long total_blocks, int prec, int variant,
                             int b_nk, hipStream_t s) {
    GemmDesc dummy{};
    switch (prec) {
        case GP_F64: return launch_gemm_p<GP_F64>(dummy, d_work, nwork, total_blocks, variant, b_nk, s);
        case GP_F32: return launch_gemm_p<GP_F32>(dummy, d_work, nwork, total_blocks, variant, b_nk, s);
        case GP_BF16X3: return launch_gemm_p<GP_BF16X3>(dummy, d_work, nwork, total_blocks, variant, b_nk, s);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched Thomas along z, one lane per (i, j) line (§2.2.2 step 2.3): at each
// k the lanes of a wave touch consecutive addresses (stride N_x N_y between k
// planes).  Arithmetic in FP64 whatever the storage type of f and x.
//
// Traffic: the forward sweep stores only d' (into x when x is FP64, else into
// an FP64 scratch) and, every THOMAS_KC planes, a checkpoint of c'; the
// backward sweep recomputes c' chunk by chunk from its checkpoint in
// registers instead of reading it back.  Loads of the next chunk are issued
// before the current chunk is computed (one lane per line leaves only one
// wave per SIMD at the workload sizes, so latency is hidden by prefetching,
// not by occupancy).
//
// The line pin_line is the null line of a singular Poisson problem: its final
// pivot vanishes and its last unknown is set to zero (§3).
// ---------------------------------------------------------------------------
constexpr int THOMAS_KC = 16;

long long thomas_scratch_doubles(int nx, int ny, int nz, int nsys, int tx) {
    const long long lines = (long long)nx * ny * nsys;
    const long long nck = (nz + THOMAS_KC - 1) / THOMAS_KC;
    return lines * nck + (tx == DT_F64 ? 0 : lines * nz);
}

template <typename TF, typename TX>
__device__ __forceinline__ void thomas_line(const ThomasDesc& t, long long gl) {
    constexpr int KC = THOMAS_KC;
    const long long S = (long long)t.nx * t.ny;
    const int sys = (int)(gl / S);
    const long long line = gl - (long long)sys * S;
    const int i = (int)(line % t.nx), j = (int)(line / t.nx);
    const int nz = t.nz;
    const int nc = (nz + KC - 1) / KC;
    const long long lines = S * t.nsys;
    const double lam = t.lamx[i] + t.lamy[j];
    const long long base = (long long)sys * S * nz + line;
    const TF* f = (const TF*)t.f + base;
    TX* x = (TX*)t.x + base;
    // checkpoints ck[c][gl] (c' entering chunk c), then (FP32 x) d' [sys][k][line]
    double* ck = t.scratch + gl;
    double* dst = sizeof(TX) == 8 ? (double*)((TX*)t.x + base) : t.scratch + lines * nc + base;
    const bool pinned = line == t.pin_line;
    const double sig = t.sigma, tau = t.tau;
    const double* __restrict__ az = t.az;
    const double* __restrict__ bz = t.bz;
    const double* __restrict__ cz = t.cz;

    // ---- forward elimination ----
    double cp = 0.0, dp = 0.0;
    double fb[KC], fn[KC];
#pragma unroll
    for (int e = 0; e < KC; ++e) fb[e] = e < nz ? (double)f[(long long)e * S] : 0.0;
    for (int c = 0; c < nc; ++c) {
        const int k0 = c * KC;
        ck[(long long)c * lines] = cp;
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + KC + e;
            fn[e] = k < nz ? (double)f[(long long)k * S] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + e;
            if (k < nz) {
                const double sub = k > 0 ? tau * az[k] : 0.0;
                const double den = sig + tau * (lam + bz[k]) - sub * cp;
                const double inv = (pinned && k == nz - 1) ? 0.0 : 1.0 / den;
                cp = k < nz - 1 ? tau * cz[k] * inv : 0.0;
                dp = (fb[e] - sub * dp) * inv;
                dst[(long long)k * S] = dp;
            }
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) fb[e] = fn[e];
    }

    // ---- back substitution, c' recomputed per chunk from its checkpoint ----
    double xv = dp;  // x_{nz-1} (0 on the pinned line: inv = 0 there)
    x[(long long)(nz - 1) * S] = (TX)xv;
    double db[KC], dn[KC];
    {
        const int k0 = (nc - 1) * KC;
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + e;
            db[e] = k < nz - 1 ? dst[(long long)k * S] : 0.0;
        }
    }
    for (int c = nc - 1; c >= 0; --c) {
        const int k0 = c * KC;
        if (c > 0) {
#pragma unroll
            for (int e = 0; e < KC; ++e) dn[e] = dst[(long long)(k0 - KC + e) * S];
        }
        double cb[KC];
        double cpr = ck[(long long)c * lines];
#pragma unroll
        for (int e = 0; e < KC; ++e) {
            const int k = k0 + e;
            if (k < nz) {
                const double sub = k > 0 ? tau * az[k] : 0.0;
                const double den = sig + tau * (lam + bz[k]) - sub * cpr;
                const double inv = (pinned && k == nz - 1) ? 0.0 : 1.0 / den;
                cpr = k < nz - 1 ? tau * cz[k] * inv : 0.0;
            }
            cb[e] = cpr;
        }
#pragma unroll
        for (int e = KC - 1; e >= 0; --e) {
            const int k = k0 + e;
            if (k < nz - 1) {
                xv = db[e] - cb[e] * xv;
                x[(long long)k * S] = (TX)xv;
            }
        }
#pragma unroll
        for (int e = 0; e < KC; ++e) db[e] = dn[e];
    }
}

__device__ __forceinline__ void thomas_dispatch(const ThomasDesc& t, long long gl) {
    if (t.tf == DT_F64 && t.tx == DT_F64) thomas_line<double, double>(t, gl);
    else if (t.tf == DT_F32 && t.tx == DT_F32) thomas_line<float, float>(t, gl);
    else if (t.tf == DT_F64) thomas_line<double, float>(t, gl);
    else thomas_line<float, double>(t, gl);
}

constexpr int THOMAS_NT = 64;

__global__ __launch_bounds__(THOMAS_NT) void thomas_kernel(ThomasDesc t, long long nlines) {
    const long long gl = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gl < nlines) thomas_dispatch(t, gl);
}

__global__ __launch_bounds__(THOMAS_NT) void thomas_multi_kernel(const ThomasDesc* __restrict__ work, int nwork,
                                                                 long long total) {
    for (long long gl = (long long)blockIdx.x * blockDim.x + threadIdx.x; gl < total;
         gl += (long long)gridDim.x * blockDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].line_begin <= gl) lo = mid;
            else hi = mid - 1;
        }
        const ThomasDesc t = work[lo];
        const long long local = gl - t.line_begin;
        if (local < (long long)t.nx * t.ny * t.nsys) thomas_dispatch(t, local);
    }
}

hipError_t launch_thomas(const ThomasDesc& t, hipStream_t s) {
    const long long n = (long long)t.nx * t.ny * t.nsys;
    if (n <= 0) return hipSuccess;
    const long long blocks = (n + THOMAS_NT - 1) / THOMAS_NT;
    hipLaunchKernelGGL(thomas_kernel, dim3((unsigned)blocks), dim3(THOMAS_NT), 0, s, t, n);
    return hipGetLastError();
}

hipError_t launch_thomas_multi(const ThomasDesc* d_work, int nwork, long long total_lines, hipStream_t s) {
    if (total_lines <= 0) return hipSuccess;
    const long long blocks = std::min((total_lines + THOMAS_NT - 1) / THOMAS_NT, 32 * PERSISTENT_BLOCKS);
    hipLaunchKernelGGL(thomas_multi_kernel, dim3((unsigned)blocks), dim3(THOMAS_NT), 0, s, d_work, nwork,
                       total_lines);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 residual of the 7-point operator (the Kronecker sum of §2.2.2 with the
// same boundary rows as the plan), r = f - A x, A = L or I - alpha L.
// One thread per unknown; partial sums of r^2 and f^2 per block.
// ---------------------------------------------------------------------------
constexpr int RES_NT = 256;

int residual_blocks(const StencilDesc& st) {
    const long long n = (long long)st.nx * st.ny * st.nz;
    return (int)((n + RES_NT - 1) / RES_NT);
}

__device__ __forceinline__ void residual_block(const StencilDesc& st, long long lb, long long gblock, double* red) {
    const long long n = (long long)st.nx * st.ny * st.nz;
    const long long idx = lb * RES_NT + threadIdx.x;
    double sr = 0.0, sf = 0.0;
    if (idx < n) {
        const int nx = st.nx, ny = st.ny, nz = st.nz;
        const long long sxy = (long long)nx * ny;
        const int i = (int)(idx % nx);
        const long long jk = idx / nx;
        const int j = (int)(jk % ny);
        const int k = (int)(jk / ny);
        const double* x = st.x;
        const double xc = x[idx];
        double lap = (st.bx[i] + st.by[j] + st.bz[k]) * xc;
        // x direction
        if (i > 0) lap += st.ax[i] * x[idx - 1];
        else if (st.perx) lap += st.ax[0] * x[idx + nx - 1];
        if (i < nx - 1) lap += st.cx[i] * x[idx + 1];
        else if (st.perx) lap += st.cx[nx - 1] * x[idx - (nx - 1)];
        // y direction
        if (j > 0) lap += st.ay[j] * x[idx - nx];
        else if (st.pery) lap += st.ay[0] * x[idx + (long long)(ny - 1) * nx];
        if (j < ny - 1) lap += st.cy[j] * x[idx + nx];
        else if (st.pery) lap += st.cy[ny - 1] * x[idx - (long long)(ny - 1) * nx];
        // z direction (never periodic)
        if (k > 0) lap += st.az[k] * x[idx - sxy];
        if (k < nz - 1) lap += st.cz[k] * x[idx + sxy];
        const double ax = st.helmholtz ? xc - st.alpha * lap : lap;
        const double fv = st.f[idx];
        const double r = fv - ax;
        st.r[idx] = (float)r;
        sr = r * r;
        sf = fv * fv;
    }
    block_sum2<RES_NT>(sr, sf, red);
    if (threadIdx.x == 0) {
        st.partials[2 * gblock] = sr;
        st.partials[2 * gblock + 1] = sf;
    }
}

__global__ __launch_bounds__(RES_NT) void residual_kernel(StencilDesc st) {
    __shared__ double red[2 * RES_NT / 64];
    residual_block(st, blockIdx.x, blockIdx.x, red);
}

__global__ __launch_bounds__(RES_NT) void residual_multi_kernel(const StencilDesc* __restrict__ work, int nwork,
                                                                long long total) {
    __shared__ double red[2 * RES_NT / 64];
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const StencilDesc st = work[lo];
        const long long lb = blk - st.block_begin;
        residual_block(st, lb, lb, red);
        __syncthreads();
    }
}

hipError_t launch_residual(const StencilDesc& st, hipStream_t s) {
    const int nb = residual_blocks(st);
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(RES_NT), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_residual_multi(const StencilDesc* d_work, int nwork, long long total_blocks, hipStream_t s) {
    if (total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(residual_multi_kernel, dim3((unsigned)std::min(total_blocks, 4 * PERSISTENT_BLOCKS)),
                       dim3(RES_NT), 0, s, d_work, nwork, total_blocks);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic pair reduction (fixed assignment of partials to threads and a
// fixed tree): one block per reduction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void reduce_pairs_block(const double* p, int n, double* out, double* red) {
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        a += p[2 * i];
        b += p[2 * i + 1];
    }
    block_sum2<256>(a, b, red);
    if (threadIdx.x == 0) {
        out[0] = a;
        out[1] = b;
    }
}

__global__ __launch_bounds__(256) void reduce_pairs_kernel(const double* p, int n, double* out) {
    __shared__ double red[8];
    reduce_pairs_block(p, n, out, red);
}

__global__ __launch_bounds__(256) void reduce_pairs_multi_kernel(const ReduceDesc* work, int nwork) {
    __shared__ double red[8];
    const ReduceDesc d = work[blockIdx.x];
    reduce_pairs_block(d.partials, d.n, d.out, red);
}

hipError_t launch_reduce_pairs(const double* partials, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(reduce_pairs_kernel, dim3(1), dim3(256), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_reduce_pairs_multi(const ReduceDesc* d_work, int nwork, hipStream_t s) {
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_pairs_multi_kernel, dim3(nwork), dim3(256), 0, s, d_work, nwork);
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
    hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, hi, lo, n);
    return hipGetLastError();
}

hipError_t launch_convert_f64_f32(const double* x, float* y, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, y, n);
    return hipGetLastError();
}

}  // namespace tpt
