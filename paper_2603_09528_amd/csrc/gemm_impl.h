// MFMA GEMM tiles for the eigenbasis transforms (x pass: C = A B^T with A the
// field's x-lines and B the basis; y pass: C_k = A B_k with A the basis and
// B_k one z slab).  Included by the per-precision translation units.
#pragma once
#include <type_traits>

#include "device_common.h"

namespace tpt {

// ---------------------------------------------------------------------------
// FP64 / FP32 MFMA (v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x4f32).
// Operand fragments: lane l holds A[m0 + l%16][k0 + l/16] and
// B[k0 + l/16][n0 + l%16]; the 16x16 result of lane l is column l%16, rows
// l/16 + 4r (f64, measured on gfx950) or 4(l/16) + r (f32), r = 0..3.
// ---------------------------------------------------------------------------
template <typename TM> struct Mfma;
template <> struct Mfma<double> {
    typedef d4 acc;
    static __device__ __forceinline__ acc zero() { return (acc){0.0, 0.0, 0.0, 0.0}; }
    static __device__ __forceinline__ acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
};
template <> struct Mfma<float> {
    typedef f4 acc;
    static __device__ __forceinline__ acc zero() { return (acc){0.f, 0.f, 0.f, 0.f}; }
    static __device__ __forceinline__ acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
};

// Work decomposition of a BM x BN tile: waves of WM x WN.
template <int BM, int BN, int WM_ = (BM >= 64 ? 64 : 32), int WN_ = (BN >= 64 ? 64 : BN)> struct TileCfg {
    static constexpr int WM = WM_;
    static constexpr int WN = WN_;
    static constexpr int WAVES_M = BM / WM;
    static constexpr int WAVES_N = BN / WN;
    static constexpr int NT = WAVES_M * WAVES_N * 64;
    static constexpr int MI = WM / 16;
    static constexpr int NI = WN / 16;
};

// LDS layout of the FP64/FP32 tile: A as [m][k], B as [n][k] (x pass) or
// [k][n] (y pass), rows padded against bank conflicts.  NBUF = 2: double
// buffered (one barrier per K tile); NBUF = 1: single buffer, two barriers
// per K tile, room for a deeper K tile.
template <typename TM, int BM, int BN, bool BNK, int BK_ = 16, int NBUF_ = 2> struct SmemF {
    static constexpr int BK = BK_;
    static constexpr int NBUF = NBUF_;
    static constexpr int PA = BK + 1;
    static constexpr int PB = BNK ? BK + 1 : BN + 2;
    static constexpr int A_ELEMS = BM * PA;
    static constexpr int B_ELEMS = BNK ? BN * PB : BK * PB;
    static constexpr int TOTAL = NBUF * (A_ELEMS + B_ELEMS);
};

__device__ __forceinline__ void decode_tile(const GemmDesc& g, long long lb, int& b, int& tm, int& tn) {
    const long long per = (long long)g.tiles_m * g.tiles_n;
    b = (int)(lb / per);
    const int rem = (int)(lb - (long long)b * per);
    tm = rem / g.tiles_n;
    tn = rem - tm * g.tiles_n;
}

// Epilogue store of one result element.
template <typename TC, int EPI>
__device__ __forceinline__ void epi_store(TC* __restrict__ C, long long idx, double v, double& se, double& sx) {
    if constexpr (EPI == EPI_ACCUM_F64) {
        const double x = C[idx] + v;
        C[idx] = x;
        se += v * v;
        sx += x * x;
    } else {
        C[idx] = (TC)v;
    }
}

template <typename TM, typename TA, typename TB, typename TC, int EPI, int BM, int BN, bool BNK, int BK_ = 16,
          int NBUF = 2, int WN_ = (BN >= 64 ? 64 : BN)>
__device__ __forceinline__ void gemm_tile_f(const GemmDesc& g, long long lb, TM* smem, double* red) {
    typedef TileCfg<BM, BN, (BM >= 64 ? 64 : 32), WN_> C;
    typedef SmemF<TM, BM, BN, BNK, BK_, NBUF> S;
    typedef Mfma<TM> MM;
    constexpr int BK = S::BK;
    constexpr int NT = C::NT;
    constexpr int LA = BM * BK / NT;
    constexpr int LB = BN * BK / NT;
    static_assert(NT % BK == 0, "thread count must be a multiple of BK");
    TM* As = smem;
    TM* Bs = smem + S::NBUF * S::A_ELEMS;

    int b, tm, tn;
    decode_tile(g, lb, b, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x;
    const int w = tid / 64, l = tid % 64, lr = l % 16, lg = l / 16;
    const int wm = w / C::WAVES_N, wn = w % C::WAVES_N;
    const int mrem = g.M - m0, nrem = g.N - n0, K = g.K;
    const int lda = g.lda, ldb = g.ldb;
    const TA* __restrict__ Ab = (const TA*)g.A + (long long)b * g.sA + (long long)m0 * lda;
    const TB* __restrict__ Bb =
        BNK ? (const TB*)g.B + (long long)b * g.sB + (long long)n0 * ldb : (const TB*)g.B + (long long)b * g.sB + n0;

    typename MM::acc acc[C::MI][C::NI];
#pragma unroll
    for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::zero();

    // fixed per-thread load geometry: A slot t covers row tid/BK + t*(NT/BK), column tid%BK
    const int arow = tid / BK, acol = tid % BK;
    // interior tiles (whole tile inside M x N) load without predicates; a K
    // that is not a multiple of BK takes the guarded loads in its last K step
    const bool full = mrem >= BM && nrem >= BN;
    TM ra[LA], rb[LB];
    // FULL is a compile-time copy of `full`: the K loop is instantiated once
    // per case, so the interior loop has no divergent loads and the loads of
    // tile k+1 stay in flight while tile k is multiplied
    auto gload = [&](int k0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        if constexpr (FULL) {
            // offsets within the tile are small and non-negative: 32-bit
            // unsigned offsets from the block's (uniform) operand bases
#pragma unroll
            for (int t = 0; t < LA; ++t) ra[t] = (TM)Ab[(unsigned)((arow + t * (NT / BK)) * lda + k0 + acol)];
#pragma unroll
            for (int t = 0; t < LB; ++t) {
                if constexpr (BNK) {
                    rb[t] = (TM)Bb[(unsigned)((arow + t * (NT / BK)) * ldb + k0 + acol)];
                } else {
                    const int e = tid + NT * t;
                    rb[t] = (TM)Bb[(unsigned)((k0 + e / BN) * ldb + e % BN)];
                }
            }
            return;
        } else {
        const bool kok = k0 + acol < K;
#pragma unroll
        for (int t = 0; t < LA; ++t) {
            const int row = arow + t * (NT / BK);
            ra[t] = (kok && row < mrem) ? (TM)Ab[row * lda + k0 + acol] : (TM)0;
        }
#pragma unroll
        for (int t = 0; t < LB; ++t) {
            if constexpr (BNK) {
                const int row = arow + t * (NT / BK);  // over n
                rb[t] = (kok && row < nrem) ? (TM)Bb[row * ldb + k0 + acol] : (TM)0;
            } else {
                const int e = tid + NT * t;
                const int row = e / BN, col = e % BN;  // row over k, col over n
                rb[t] = (k0 + row < K && col < nrem) ? (TM)Bb[(k0 + row) * ldb + col] : (TM)0;
            }
        }
        }
    };
    auto sstore = [&](int buf) {
        TM* a = As + buf * S::A_ELEMS;
        TM* bb = Bs + buf * S::B_ELEMS;
#pragma unroll
        for (int t = 0; t < LA; ++t) a[(arow + t * (NT / BK)) * S::PA + acol] = ra[t];
#pragma unroll
        for (int t = 0; t < LB; ++t) {
            if constexpr (BNK) {
                bb[(arow + t * (NT / BK)) * S::PB + acol] = rb[t];
            } else {
                const int e = tid + NT * t;
                bb[(e / BN) * S::PB + (e % BN)] = rb[t];
            }
        }
    };

    const int nk = (K + BK - 1) / BK;
    // loop forms: 0 guarded loads, 1 interior (no predicates), 2 interior
    // with a ragged K, whose last K step takes the guarded loads (its own
    // instantiation, so the interior loop keeps its single basic block)
    const bool ktail = (K % BK) != 0;
    auto gload_step = [&](int kt, auto mode) {
        constexpr int MODE = decltype(mode)::value;
        if constexpr (MODE == 0) {
            gload(kt * BK, std::false_type{});
        } else if constexpr (MODE == 1) {
            gload(kt * BK, std::true_type{});
        } else {
            if (kt == nk - 1) gload(kt * BK, std::false_type{});
            else gload(kt * BK, std::true_type{});
        }
    };
    auto kloop = [&](auto mode) {
    gload_step(0, mode);
    if constexpr (NBUF == 2) {
        sstore(0);
        __syncthreads();
    }
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = NBUF == 2 ? (kt & 1) : 0;
        if constexpr (NBUF == 1) {
            if (kt > 0) __syncthreads();  // every wave is done with the previous tile
            sstore(0);
            __syncthreads();
        }
        if (kt + 1 < nk) gload_step(kt + 1, mode);
        const TM* a = As + cur * S::A_ELEMS + (wm * C::WM + lr) * S::PA + lg;
        const TM* bb = Bs + cur * S::B_ELEMS;
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            TM fa[C::MI], fb[C::NI];
#pragma unroll
            for (int i = 0; i < C::MI; ++i) fa[i] = a[i * 16 * S::PA + kk * 4];
#pragma unroll
            for (int j = 0; j < C::NI; ++j) {
                if constexpr (BNK) fb[j] = bb[(wn * C::WN + j * 16 + lr) * S::PB + kk * 4 + lg];
                else fb[j] = bb[(kk * 4 + lg) * S::PB + wn * C::WN + j * 16 + lr];
            }
#pragma unroll
            for (int i = 0; i < C::MI; ++i)
#pragma unroll
                for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::mma(fa[i], fb[j], acc[i][j]);
            // stage the next K tile before the last MFMA group (see the
            // persistent form)
            if constexpr (NBUF == 2)
                if (kk == BK / 4 - 2 && kt + 1 < nk) sstore(cur ^ 1);
        }
        if constexpr (NBUF == 2) __syncthreads();
    }
    };
    if (!full) kloop(std::integral_constant<int, 0>{});
    else if (!ktail) kloop(std::integral_constant<int, 1>{});
    else kloop(std::integral_constant<int, 2>{});
    if constexpr (NBUF == 1) __syncthreads();

    double se = 0.0, sx = 0.0;
    TC* __restrict__ Cb = (TC*)g.C + (long long)b * g.sC + (long long)m0 * g.ldc + n0;
#pragma unroll
    for (int i = 0; i < C::MI; ++i) {
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int n = wn * C::WN + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = wm * C::WM + i * 16 + MM::row(lg, r);
                if (full || (m < mrem && n < nrem))
                    epi_store<TC, EPI>(Cb, (long long)m * g.ldc + n, (double)acc[i][j][r], se, sx);
            }
        }
    }
    if constexpr (EPI == EPI_ACCUM_F64) {
        block_sum2<NT>(se, sx, red);
        if (threadIdx.x == 0) {
            g.partials[2 * lb] = se;
            g.partials[2 * lb + 1] = sx;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent form of the FP64/FP32 tile.  Edge tiles (M or N not a multiple
// of 128) read their operands through buffer resources that end at the
// operand's last row, so rows past it read zero, and store only inside M x N;
// a K that is not a multiple of 16 zeroes the elements past K in its last K
// step (both operands, so that nothing else meets a zero).  Each block walks
// tiles v = blockIdx.x, + gridDim.x, ... (numbered per XCD as in gemm_kernel)
// and, during the last K step of a tile, already loads the first K tile of
// its next tile, which it stores to the free LDS buffer before writing the
// finished tile out: the load latency at the start of a tile and the result
// stores at its end overlap the multiplications (a 256-deep K has only 16 K
// steps per tile, so these ends are a large share of a tile).  Operands are
// read and results written through buffer resources (base in scalar
// registers, 32-bit per-thread offsets, block-uniform K steps as scalar
// offsets), which keeps the address state small enough for two blocks per CU.
// Within a K step the next K tile is written to the free LDS buffer before the
// last group of MFMAs rather than after all of them: the wait for its loads
// and the LDS writes then overlap MFMAs still in the queue (measured 7-8 %
// faster at 256^3 x 256, 512^3 x 64 and 768 x 1024 x 768 x 64).
// ---------------------------------------------------------------------------
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int BUF_RSRC_WORD3 = 0x00020000;  // raw 32-bit buffer (gfx9 family)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, BUF_RSRC_WORD3);
}
// buffer resource over [base, base + bytes), bytes clamped to the 31-bit range
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc_n(const void* base, long long bytes) {
    const int n = bytes <= 0 ? 0 : (bytes > 0x7ffffff0LL ? 0x7ffffff0 : (int)bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, n, BUF_RSRC_WORD3);
}
template <typename T> struct BufIO;
template <> struct BufIO<double> {
    static __device__ __forceinline__ double ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
    }
    static __device__ __forceinline__ void st(double v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)vo, (int)so, 0);
    }
};
template <> struct BufIO<float> {
    static __device__ __forceinline__ float ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
    }
    static __device__ __forceinline__ void st(float v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)vo, (int)so, 0);
    }
};

template <typename TM, typename TA, typename TB, typename TC, int EPI, bool BNK, int WN = 64, bool EDGE = false>
__device__ __forceinline__ void gemm_tiles_persist_f(const GemmDesc& g, long long ntiles, TM* smem, double* red) {
    constexpr int BM = 128, BN = 128, BK = 16;
    typedef TileCfg<BM, BN, 64, WN> C;
    typedef SmemF<TM, BM, BN, BNK, BK, 2> S;
    typedef Mfma<TM> MM;
    constexpr int NT = C::NT;
    constexpr int LA = BM * BK / NT;
    constexpr int LB = BN * BK / NT;
    TM* As = smem;
    TM* Bs = smem + 2 * S::A_ELEMS;
    const int tid = threadIdx.x;
    const int w = tid / 64, l = tid % 64, lr = l % 16, lg = l / 16;
    const int wm = w / C::WAVES_N, wn = w % C::WAVES_N;
    const int arow = tid / BK, acol = tid % BK;
    const int lda = g.lda, ldb = g.ldb, ldc = g.ldc;
    const int M = g.M, N = g.N, K = g.K;
    // EDGE: M, N or K ragged (the launcher picks it); else every tile is
    // interior and none of the edge handling below is compiled in
    const int nk = EDGE ? (K + BK - 1) / BK : K / BK;
    const bool ktail = EDGE && (K % BK) != 0;
    const long long grid = gridDim.x;
    // K-step scalar offsets (bytes) of the A and B tiles
    const unsigned kstepA = BK * (unsigned)sizeof(TA);
    const unsigned kstepB = BNK ? BK * (unsigned)sizeof(TB) : (unsigned)(BK * ldb) * (unsigned)sizeof(TB);

    // a tile's operand and result resources: each ends where its operand's
    // rows of this batch entry end (A: rows past M; B: rows past N (x pass)
    // or past K (y pass); C: rows past M), so edge tiles read zeros there and
    // nothing past them is ever touched; mrem / nrem bound the stores
    auto tile_rsrc = [&](long long v, __amdgpu_buffer_rsrc_t& rA, __amdgpu_buffer_rsrc_t& rB,
                         __amdgpu_buffer_rsrc_t& rC, int& mrem, int& nrem) {
        int b, tm, tn;
        decode_tile(g, xcd_block(v, ntiles), b, tm, tn);
        const int m0 = tm * BM, n0 = tn * BN;
        mrem = M - m0;
        nrem = N - n0;
        const TA* a = (const TA*)g.A + (long long)b * g.sA + (long long)m0 * lda;
        const TB* bp = BNK ? (const TB*)g.B + (long long)b * g.sB + (long long)n0 * ldb
                           : (const TB*)g.B + (long long)b * g.sB + n0;
        TC* c = (TC*)g.C + (long long)b * g.sC + (long long)m0 * ldc + n0;
        if constexpr (EDGE) {
            rA = buf_rsrc_n(a, (long long)mrem * lda * (long long)sizeof(TA));
            rB = BNK ? buf_rsrc_n(bp, (long long)nrem * ldb * (long long)sizeof(TB))
                     : buf_rsrc_n(bp, ((long long)K * ldb - n0) * (long long)sizeof(TB));
            rC = buf_rsrc_n(c, ((long long)mrem * ldc - n0) * (long long)sizeof(TC));
        } else {
            rA = buf_rsrc(a);
            rB = buf_rsrc(bp);
            rC = buf_rsrc(c);
        }
    };
    TM ra[LA], rb[LB];
    auto gload = [&](__amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rB, int kt) {
#pragma unroll
        for (int q = 0; q < LA; ++q)
            ra[q] = (TM)BufIO<TA>::ld(rA, (unsigned)(((arow + q * (NT / BK)) * lda + acol) * (int)sizeof(TA)),
                                      kt * kstepA);
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            unsigned vo;
            if constexpr (BNK) {
                vo = (unsigned)(((arow + q * (NT / BK)) * ldb + acol) * (int)sizeof(TB));
            } else {
                const int e = tid + NT * q;
                vo = (unsigned)(((e / BN) * ldb + e % BN) * (int)sizeof(TB));
            }
            rb[q] = (TM)BufIO<TB>::ld(rB, vo, kt * kstepB);
        }
        // the last K step of a K that is not a multiple of BK: elements past
        // K (the next row's or slab's values) are zero in both operands
        if (ktail && kt == nk - 1) {
            const bool kin = kt * BK + acol < K;
#pragma unroll
            for (int q = 0; q < LA; ++q) ra[q] = kin ? ra[q] : (TM)0;
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                if constexpr (BNK) rb[q] = kin ? rb[q] : (TM)0;
                else rb[q] = kt * BK + (tid + NT * q) / BN < K ? rb[q] : (TM)0;
            }
        }
    };
    auto sstore = [&](int buf) {
        TM* a = As + buf * S::A_ELEMS;
        TM* bb = Bs + buf * S::B_ELEMS;
#pragma unroll
        for (int q = 0; q < LA; ++q) a[(arow + q * (NT / BK)) * S::PA + acol] = ra[q];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            if constexpr (BNK) {
                bb[(arow + q * (NT / BK)) * S::PB + acol] = rb[q];
            } else {
                const int e = tid + NT * q;
                bb[(e / BN) * S::PB + (e % BN)] = rb[q];
            }
        }
    };

    long long v = blockIdx.x;
    if (v >= ntiles) return;
    __amdgpu_buffer_rsrc_t rA, rB, rC;
    int mrem, nrem;
    tile_rsrc(v, rA, rB, rC, mrem, nrem);
    gload(rA, rB, 0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    const unsigned tbase = (unsigned)(((wm * C::WM + MM::row(lg, 0)) * ldc + wn * C::WN + lr) * (int)sizeof(TC));
    for (; v < ntiles; v += grid) {
        const bool more = v + grid < ntiles;
        typename MM::acc acc[C::MI][C::NI];
#pragma unroll
        for (int i = 0; i < C::MI; ++i)
#pragma unroll
            for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::zero();
        __amdgpu_buffer_rsrc_t rAn = rA, rBn = rB, rCn = rC;
        int mremn = mrem, nremn = nrem;
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) {
                gload(rA, rB, kt + 1);
            } else if (more) {
                tile_rsrc(v + grid, rAn, rBn, rCn, mremn, nremn);
                gload(rAn, rBn, 0);
            }
            const TM* a = As + buf * S::A_ELEMS + (wm * C::WM + lr) * S::PA + lg;
            const TM* bb = Bs + buf * S::B_ELEMS;
            const bool stage = kt + 1 < nk || more;
#pragma unroll
            for (int kk = 0; kk < BK / 4; ++kk) {
                TM fa[C::MI], fb[C::NI];
#pragma unroll
                for (int i = 0; i < C::MI; ++i) fa[i] = a[i * 16 * S::PA + kk * 4];
#pragma unroll
                for (int j = 0; j < C::NI; ++j) {
                    if constexpr (BNK) fb[j] = bb[(wn * C::WN + j * 16 + lr) * S::PB + kk * 4 + lg];
                    else fb[j] = bb[(kk * 4 + lg) * S::PB + wn * C::WN + j * 16 + lr];
                }
#pragma unroll
                for (int i = 0; i < C::MI; ++i)
#pragma unroll
                    for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::mma(fa[i], fb[j], acc[i][j]);
                // stage the next K tile (or the next tile's first) into the
                // other buffer before the last MFMA group, so that waiting for
                // its loads and writing it overlap the MFMAs still queued
                if (kk == BK / 4 - 2 && stage) sstore(buf ^ 1);
            }
            if (kt + 1 < nk) {
                __syncthreads();
                buf ^= 1;
            }
        }
        double se = 0.0, sx = 0.0;
        // edge tiles store only the rows below M and the columns below N
        const bool edge = EDGE && (mrem < BM || nrem < BN);
        const int wrow = wm * C::WM + MM::row(lg, 0), wcol = wn * C::WN + lr;
#pragma unroll
        for (int i = 0; i < C::MI; ++i) {
#pragma unroll
            for (int j = 0; j < C::NI; ++j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const unsigned so = (unsigned)(((i * 16 + MM::row(0, r)) * ldc + j * 16) * (int)sizeof(TC));
                    const double val = (double)acc[i][j][r];
                    if (edge && (wrow + i * 16 + MM::row(0, r) >= mrem || wcol + j * 16 >= nrem)) continue;
                    if constexpr (EPI == EPI_ACCUM_F64) {
                        const double x = BufIO<double>::ld(rC, tbase, so) + val;
                        BufIO<double>::st(x, rC, tbase, so);
                        se += val * val;
                        sx += x * x;
                    } else {
                        BufIO<TC>::st((TC)val, rC, tbase, so);
                    }
                }
            }
        }
        if constexpr (EPI == EPI_ACCUM_F64) {
            const long long lt = xcd_block(v, ntiles);
            block_sum2<NT>(se, sx, red);
            if (threadIdx.x == 0) {
                g.partials[2 * lt] = se;
                g.partials[2 * lt + 1] = sx;
            }
        }
        __syncthreads();
        buf ^= 1;
        rA = rAn;
        rB = rBn;
        rC = rCn;
        mrem = mremn;
        nrem = nremn;
    }
}

// ---------------------------------------------------------------------------
// Work-list form of the FP64/FP32 tile for many uneven problems (batches,
// serving): a persistent grid walks the tiles of every problem of the list
// (tile v = blockIdx.x, + gridDim.x, ...; its problem by binary search on
// block_begin) and, as the single-problem persistent tile does, loads and
// stages the first K tile of its next tile during the last K step of the
// current one, so a short K loop (K = 48..192 in the batches) does not pay a
// load latency and a store phase per tile.  Uneven shapes are handled without
// per-element predicates on the loads: operands are read through buffer
// resources whose range ends at the problem's data, so rows past M (x pass)
// or columns past the last slab (y pass) read zero, and only the last K step
// of a K that is not a multiple of 16 masks the elements past K (in both
// operands, so that no stray value meets a zero).
//
// Tile shapes follow the problems: the x pass (M = Ny Nz rows, N = K = Nx)
// takes 128 x 64 tiles; the y pass folds the z slabs into N (column
// n' = slab Nx + i, N' = Nz Nx) and takes 64 x 128 tiles over M = Ny, so a
// small slab does not leave most of a 128-wide tile empty.  Four waves of
// (BM/2) x (BN/2).  Every output element accumulates its K products in the
// same order as in the single-problem tiles, so results are bitwise those of
// the single solves.
// ---------------------------------------------------------------------------
template <int BM, int BN> struct WlCfg {
    static constexpr int BK = 16, NT = 256, WM = BM / 2, WN = BN / 2, MI = WM / 16, NI = WN / 16;
    static constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
};


// One tile of a work list: its problem's operands and its position.
struct WlTile {
    const char* A;
    const char* B;
    char* C;
    double* partials;
    long long sB, sC, Ntot, n0, lb;
    int M, N, K, lda, ldb, ldc, m0, batch;
};

template <int BM, int BN, bool BNK>
__device__ __forceinline__ void wl_find(const GemmDesc* __restrict__ work, int nwork, long long v, WlTile& t) {
    int lo = 0, hi = nwork - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (work[mid].block_begin <= v) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc& g = work[lo];
    t.A = (const char*)g.A;
    t.B = (const char*)g.B;
    t.C = (char*)g.C;
    t.partials = g.partials;
    t.M = g.M;
    t.N = g.N;
    t.K = g.K;
    t.lda = g.lda;
    t.ldb = g.ldb;
    t.ldc = g.ldc;
    t.sB = g.sB;
    t.sC = g.sC;
    t.batch = BNK ? 1 : g.batch;
    t.Ntot = (long long)g.N * t.batch;
    t.lb = v - g.block_begin;
    const long long tm = t.lb / g.tiles_n;
    t.m0 = (int)(tm * BM);
    t.n0 = (t.lb - tm * g.tiles_n) * BN;
}

template <typename TM, typename TA, typename TB, typename TC, int EPI, bool BNK, int BM, int BN>
__device__ __forceinline__ void gemm_worklist_f(const GemmDesc* __restrict__ work, int nwork, long long total,
                                                TM* smem, double* red) {
    typedef WlCfg<BM, BN> W;
    constexpr int BK = W::BK, NT = W::NT, LA = W::LA, LB = W::LB, MI = W::MI, NI = W::NI;
    typedef SmemF<TM, BM, BN, BNK, BK, 2> S;
    typedef Mfma<TM> MM;
    TM* As = smem;
    TM* Bs = smem + 2 * S::A_ELEMS;
    const int tid = threadIdx.x;
    const int w = tid / 64, l = tid % 64, lr = l % 16, lg = l / 16;
    const int wm = w / 2, wn = w % 2;
    const int arow = tid / BK, acol = tid % BK;
    constexpr int ea = (int)sizeof(TA), eb = (int)sizeof(TB);

    // operand resources of a tile, and (y pass) the column part of each B
    // load's offset: slab (relative to the tile's first) and index in it
    auto setup = [&](const WlTile& t, __amdgpu_buffer_rsrc_t& rA, __amdgpu_buffer_rsrc_t& rB, unsigned* boff) {
        rA = buf_rsrc_n(t.A + (long long)t.m0 * t.lda * ea, (long long)(t.M - t.m0) * t.lda * ea);
        if constexpr (BNK) {
            rB = buf_rsrc_n(t.B + t.n0 * t.ldb * eb, (t.N - t.n0) * (long long)t.ldb * eb);
        } else {
            // column indices fit 32 bits (the launcher checks N' and the extents)
            const unsigned N = (unsigned)t.N, b0 = (unsigned)t.n0 / N;
            rB = buf_rsrc_n(t.B + (long long)b0 * t.sB * eb, (t.batch - (long long)b0) * t.sB * eb);
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const int e = tid + NT * q;
                const unsigned nn = (unsigned)t.n0 + (unsigned)(e % BN);
                const unsigned bq = nn / N;
                boff[q] = (bq - b0) * (unsigned)t.sB + (nn - bq * N);
            }
        }
    };
    TM ra[LA], rb[LB];
    auto gload = [&](const WlTile& t, __amdgpu_buffer_rsrc_t rA, __amdgpu_buffer_rsrc_t rB, const unsigned* boff,
                     int kt) {
        const int k0 = kt * BK;
        const bool tail = k0 + BK > t.K;
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const unsigned vo = (unsigned)(((arow + q * (NT / BK)) * t.lda + k0 + acol) * ea);
            ra[q] = (TM)BufIO<TA>::ld(rA, vo, 0);
        }
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            unsigned vo;
            if constexpr (BNK) vo = (unsigned)(((arow + q * (NT / BK)) * t.ldb + k0 + acol) * eb);
            else vo = (boff[q] + (unsigned)((k0 + (tid + NT * q) / BN) * t.ldb)) * (unsigned)eb;
            rb[q] = (TM)BufIO<TB>::ld(rB, vo, 0);
        }
        if (tail) {
            const bool ka = k0 + acol < t.K;
#pragma unroll
            for (int q = 0; q < LA; ++q) ra[q] = ka ? ra[q] : (TM)0;
#pragma unroll
            for (int q = 0; q < LB; ++q) {
                const bool kb = BNK ? ka : (k0 + (tid + NT * q) / BN < t.K);
                rb[q] = kb ? rb[q] : (TM)0;
            }
        }
    };
    auto sstore = [&](int buf) {
        TM* a = As + buf * S::A_ELEMS;
        TM* bb = Bs + buf * S::B_ELEMS;
#pragma unroll
        for (int q = 0; q < LA; ++q) a[(arow + q * (NT / BK)) * S::PA + acol] = ra[q];
#pragma unroll
        for (int q = 0; q < LB; ++q) {
            if constexpr (BNK) {
                bb[(arow + q * (NT / BK)) * S::PB + acol] = rb[q];
            } else {
                const int e = tid + NT * q;
                bb[(e / BN) * S::PB + (e % BN)] = rb[q];
            }
        }
    };

    const long long grid = gridDim.x;
    long long v = blockIdx.x;
    if (v >= total) return;
    WlTile cur, nxt;
    __amdgpu_buffer_rsrc_t rA, rB, nA, nB;
    unsigned boff[BNK ? 1 : LB], nboff[BNK ? 1 : LB];
    wl_find<BM, BN, BNK>(work, nwork, v, cur);
    setup(cur, rA, rB, boff);
    gload(cur, rA, rB, boff, 0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (; v < total; v += grid) {
        const bool more = v + grid < total;
        const int nk = (cur.K + BK - 1) / BK;
        typename MM::acc acc[MI][NI];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < NI; ++j) acc[i][j] = MM::zero();
        for (int kt = 0; kt < nk; ++kt) {
            if (kt + 1 < nk) {
                gload(cur, rA, rB, boff, kt + 1);
            } else if (more) {
                wl_find<BM, BN, BNK>(work, nwork, v + grid, nxt);
                setup(nxt, nA, nB, nboff);
                gload(nxt, nA, nB, nboff, 0);
            }
            const bool stage = kt + 1 < nk || more;
            const TM* a = As + buf * S::A_ELEMS + (wm * W::WM + lr) * S::PA + lg;
            const TM* bb = Bs + buf * S::B_ELEMS;
#pragma unroll
            for (int kk = 0; kk < BK / 4; ++kk) {
                TM fa[MI], fb[NI];
#pragma unroll
                for (int i = 0; i < MI; ++i) fa[i] = a[i * 16 * S::PA + kk * 4];
#pragma unroll
                for (int j = 0; j < NI; ++j) {
                    if constexpr (BNK) fb[j] = bb[(wn * W::WN + j * 16 + lr) * S::PB + kk * 4 + lg];
                    else fb[j] = bb[(kk * 4 + lg) * S::PB + wn * W::WN + j * 16 + lr];
                }
#pragma unroll
                for (int i = 0; i < MI; ++i)
#pragma unroll
                    for (int j = 0; j < NI; ++j) acc[i][j] = MM::mma(fa[i], fb[j], acc[i][j]);
                if (kk == BK / 4 - 2 && stage) sstore(buf ^ 1);
            }
            if (kt + 1 < nk) {
                __syncthreads();
                buf ^= 1;
            }
        }
        // results: rows m < M, columns n' < N' (y pass: slab n' / N, index n' % N)
        double se = 0.0, sx = 0.0;
        TC* __restrict__ C = (TC*)cur.C;
        long long coff[NI];
        bool cok[NI];
#pragma unroll
        for (int j = 0; j < NI; ++j) {
            const long long nn = cur.n0 + wn * W::WN + j * 16 + lr;
            cok[j] = nn < cur.Ntot;
            if constexpr (BNK) {
                coff[j] = nn;
            } else {
                const unsigned bq = (unsigned)nn / (unsigned)cur.N;
                coff[j] = (long long)bq * cur.sC + ((unsigned)nn - bq * (unsigned)cur.N);
            }
        }
#pragma unroll
        for (int i = 0; i < MI; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = cur.m0 + wm * W::WM + i * 16 + MM::row(lg, r);
                const long long ro = (long long)m * cur.ldc;
#pragma unroll
                for (int j = 0; j < NI; ++j)
                    if (m < cur.M && cok[j]) epi_store<TC, EPI>(C, ro + coff[j], (double)acc[i][j][r], se, sx);
            }
        }
        if constexpr (EPI == EPI_ACCUM_F64) {
            block_sum2<NT>(se, sx, red);
            if (threadIdx.x == 0) {
                cur.partials[2 * cur.lb] = se;
                cur.partials[2 * cur.lb + 1] = sx;
            }
        }
        __syncthreads();
        buf ^= 1;
        if (more) {
            cur = nxt;
            rA = nA;
            rB = nB;
            if constexpr (!BNK)
#pragma unroll
                for (int q = 0; q < LB; ++q) boff[q] = nboff[q];
        }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 x3 (v_mfma_f32_16x16x32_bf16, FP32 accumulate): each operand is
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi), round to nearest even) and
// C = A_lo B_hi + A_hi B_lo + A_hi B_hi, small products first.  Fragments:
// lane l holds A[m0 + l%16][k0 + 8(l/16) .. +7] and B[k0 + 8(l/16) .. +7][n0 + l%16];
// result rows 4(l/16) + r.  Both LDS tiles are k-contiguous (As[m][k],
// Bs[n][k]) so each fragment is one 16-byte LDS read.  The basis operand
// arrives pre-split (bf16 planes); the data operand is split on the fly.
// ---------------------------------------------------------------------------
template <int BM, int BN, int BK_ = 32> struct SmemB {
    static constexpr int BK = BK_;
    static constexpr int P = BK + 8;  // row stride in bf16 (16-byte padding)
    static constexpr int A_ELEMS = BM * P;
    static constexpr int B_ELEMS = BN * P;
    static constexpr int TOTAL = 2 * (A_ELEMS + B_ELEMS);  // [hi, lo][A | B], single buffer
};

// 8 consecutive k of one row of pre-split bf16 planes (row start ph / pl);
// zeros outside [0, nrows) x [0, K).
__device__ __forceinline__ void load8_planes(const uint16_t* __restrict__ ph, const uint16_t* __restrict__ pl,
                                             bool rowok, int k, int K, u16x8& h, u16x8& lo) {
    if (rowok && k + 8 <= K && ((((uintptr_t)(ph + k)) & 15) == 0)) {
        h = *(const u16x8*)(ph + k);
        lo = *(const u16x8*)(pl + k);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const bool ok = rowok && k + e < K;
            h[e] = ok ? ph[k + e] : (uint16_t)0;
            lo[e] = ok ? pl[k + e] : (uint16_t)0;
        }
    }
}

template <typename TD, typename TC, int EPI, int BM, int BN, bool BNK, int BK_ = 32>
__device__ __forceinline__ void gemm_tile_b(const GemmDesc& g, long long lb, uint16_t* smem, double* red) {
    typedef TileCfg<BM, BN> C;
    typedef SmemB<BM, BN, BK_> S;
    constexpr int BK = S::BK;
    constexpr int NT = C::NT;
    constexpr int P = S::P;
    constexpr int CA = BM * BK / 8 / NT;  // 8-element chunks of A per thread
    constexpr int CB = BN * BK / 8 / NT;
    static_assert(CA >= 1 && CB >= 1, "tile too small for the thread count");
    uint16_t* sm_hi = smem;
    uint16_t* sm_lo = smem + (S::A_ELEMS + S::B_ELEMS);

    int b, tm, tn;
    decode_tile(g, lb, b, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    const int tid = threadIdx.x;
    const int w = tid / 64, l = tid % 64, lr = l % 16, lg = l / 16;
    const int wm = w / C::WAVES_N, wn = w % C::WAVES_N;
    const int mrem = g.M - m0, nrem = g.N - n0, K = g.K;
    const int lda = g.lda, ldb = g.ldb;
    // x pass (BNK): A = data [m][k], B = basis planes [n][k]
    // y pass:       A = basis planes [m][k], B = data [k][n]
    const long long offA = (long long)b * g.sA + (long long)m0 * lda;
    const long long offB = BNK ? (long long)b * g.sB + (long long)n0 * ldb : (long long)b * g.sB + n0;
    // the basis planes' rows: their own stride where given (padded to 16 bytes)
    const int ldpl = g.ldp ? g.ldp : (BNK ? ldb : lda);
    const long long offP = BNK ? (long long)b * g.sB + (long long)n0 * ldpl : (long long)b * g.sA + (long long)m0 * ldpl;

    f4 acc[C::MI][C::NI];
#pragma unroll
    for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j) acc[i][j] = (f4){0.f, 0.f, 0.f, 0.f};

    // Registers between the load of a K tile and its store to LDS: the basis
    // operand arrives pre-split (bf16 planes); the data operand is kept as
    // raw FP32 values and split into hi/lo only when stored, so the loads of
    // tile k+1 stay in flight while tile k is multiplied.
    u16x8 rph[BNK ? CB : CA], rpl[BNK ? CB : CA];  // basis planes (x pass: B, y pass: A)
    float rd[BNK ? CA : CB][8];                     // data (x pass: A rows, y pass: B column pairs)
    static_assert(BNK || CB % 2 == 0, "pair chunks need an even chunk count");
    // interior tiles with aligned rows load without predicates, as vectors
    const bool aligned_data = BNK ? ((lda % 8) == 0 && (offA % 8) == 0 && ((((uintptr_t)g.A) & 31) == 0))
                                  : ((ldb % 2) == 0 && (offB % 2) == 0 &&
                                     ((((uintptr_t)g.B) & (2 * sizeof(TD) - 1)) == 0));
    const bool aligned_planes = (ldpl % 8) == 0 && (offP % 8) == 0;
    // interior tiles load without predicates; a K that is not a multiple of
    // BK takes the guarded loads in its last K step only
    const bool full = mrem >= BM && nrem >= BN && aligned_data && aligned_planes;
    auto gload = [&](int k0, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        // basis planes
#pragma unroll
        for (int t = 0; t < (BNK ? CB : CA); ++t) {
            const int c = tid + NT * t;
            const int row = c / (BK / 8), kc = c % (BK / 8);
            const long long off = offP + (long long)row * ldpl + k0 + kc * 8;
            if constexpr (FULL) {
                rph[t] = *(const u16x8*)(g.basis_hi + off);
                rpl[t] = *(const u16x8*)(g.basis_lo + off);
            } else {
                const bool rok = row < (BNK ? nrem : mrem);
                load8_planes(g.basis_hi + off - (k0 + kc * 8), g.basis_lo + off - (k0 + kc * 8), rok, k0 + kc * 8, K,
                             rph[t], rpl[t]);
            }
        }
        if constexpr (BNK) {
            // x pass: A data [m][k], 8 consecutive k of one row per chunk
#pragma unroll
            for (int t = 0; t < CA; ++t) {
                const int c = tid + NT * t;
                const int row = c / (BK / 8), kc = c % (BK / 8);
                const TD* pa = (const TD*)g.A + offA + (long long)row * lda + k0 + kc * 8;
                if constexpr (FULL) {
                    if constexpr (sizeof(TD) == 4) {
                        const float4 p0 = *(const float4*)pa, p1 = *(const float4*)(pa + 4);
                        rd[t][0] = p0.x; rd[t][1] = p0.y; rd[t][2] = p0.z; rd[t][3] = p0.w;
                        rd[t][4] = p1.x; rd[t][5] = p1.y; rd[t][6] = p1.z; rd[t][7] = p1.w;
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; e += 2) {
                            const double2 q = *(const double2*)(pa + e);
                            rd[t][e] = (float)q.x;
                            rd[t][e + 1] = (float)q.y;
                        }
                    }
                } else {
                    const bool rok = row < mrem;
#pragma unroll
                    for (int e = 0; e < 8; ++e) rd[t][e] = (rok && k0 + kc * 8 + e < K) ? (float)pa[e] : 0.f;
                }
            }
        } else {
            // y pass: B data [k][n]; pair chunk c covers columns 2 (c % (BN/2)) + {0, 1}
            // and k = 8 (c / (BN/2)) .. +7
#pragma unroll
            for (int t = 0; t < CB / 2; ++t) {
                const int c = tid + NT * t;
                const int np = c % (BN / 2), kc = c / (BN / 2);
                const int nn = 2 * np;
                const TD* pb = (const TD*)g.B + offB + nn;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = k0 + kc * 8 + e;
                    if constexpr (FULL) {
                        if constexpr (sizeof(TD) == 4) {
                            const float2 q = *(const float2*)(pb + (long long)k * ldb);
                            rd[2 * t][e] = q.x;
                            rd[2 * t + 1][e] = q.y;
                        } else {
                            const double2 q = *(const double2*)(pb + (long long)k * ldb);
                            rd[2 * t][e] = (float)q.x;
                            rd[2 * t + 1][e] = (float)q.y;
                        }
                    } else {
                        rd[2 * t][e] = (nn < nrem && k < K) ? (float)pb[(long long)k * ldb] : 0.f;
                        rd[2 * t + 1][e] = (nn + 1 < nrem && k < K) ? (float)pb[(long long)k * ldb + 1] : 0.f;
                    }
                }
            }
        }
    };
    auto sstore = [&]() {
        uint16_t* ah = sm_hi;
        uint16_t* al = sm_lo;
        uint16_t* bh = ah + S::A_ELEMS;
        uint16_t* bl = al + S::A_ELEMS;
        // basis planes as loaded
#pragma unroll
        for (int t = 0; t < (BNK ? CB : CA); ++t) {
            const int c = tid + NT * t;
            const int row = c / (BK / 8), kc = c % (BK / 8);
            *(u16x8*)((BNK ? bh : ah) + row * P + kc * 8) = rph[t];
            *(u16x8*)((BNK ? bl : al) + row * P + kc * 8) = rpl[t];
        }
        // data split into hi / lo planes
#pragma unroll
        for (int t = 0; t < (BNK ? CA : CB); ++t) {
            int row, kc;
            if constexpr (BNK) {
                const int c = tid + NT * t;
                row = c / (BK / 8);
                kc = c % (BK / 8);
            } else {
                const int c = tid + NT * (t / 2);
                row = 2 * (c % (BN / 2)) + (t & 1);
                kc = c / (BN / 2);
            }
            u32x4_t hw, lw;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t hh, ll;
                split_bf16x2(rd[t][2 * e], rd[t][2 * e + 1], hh, ll);
                hw[e] = hh;
                lw[e] = ll;
            }
            const u16x8 h = __builtin_bit_cast(u16x8, hw), lo = __builtin_bit_cast(u16x8, lw);
            *(u16x8*)((BNK ? ah : bh) + row * P + kc * 8) = h;
            *(u16x8*)((BNK ? al : bl) + row * P + kc * 8) = lo;
        }
    };

    // single LDS buffer (keeps the tile small enough for two or three
    // workgroups per CU); the next tile is prefetched into registers while
    // the current one is multiplied
    const int nk = (K + BK - 1) / BK;
    // loop forms: 0 guarded loads, 1 interior (no predicates), 2 interior
    // with a ragged K, whose last K step takes the guarded loads (its own
    // instantiation, so the interior loop keeps its single basic block)
    const bool ktail = (K % BK) != 0;
    auto gload_step = [&](int kt, auto mode) {
        constexpr int MODE = decltype(mode)::value;
        if constexpr (MODE == 0) {
            gload(kt * BK, std::false_type{});
        } else if constexpr (MODE == 1) {
            gload(kt * BK, std::true_type{});
        } else {
            if (kt == nk - 1) gload(kt * BK, std::false_type{});
            else gload(kt * BK, std::true_type{});
        }
    };
    auto kloop = [&](auto mode) {
    gload_step(0, mode);
    for (int kt = 0; kt < nk; ++kt) {
        if (kt > 0) __syncthreads();  // every wave is done reading the previous tile
        sstore();
        __syncthreads();
        if (kt + 1 < nk) gload_step(kt + 1, mode);
        const uint16_t* ah = sm_hi;
        const uint16_t* al = sm_lo;
        const uint16_t* bh = ah + S::A_ELEMS;
        const uint16_t* bl = al + S::A_ELEMS;
        // one MFMA K of 32 per sub-step; a 64-deep tile runs two, in the
        // order two 32-deep tiles would, so every accumulator sees the same
        // sequence of products (not unrolled: one set of fragments live)
#pragma unroll 1
        for (int kk = 0; kk < BK / 32; ++kk) {
        bf16x8 fah[C::MI], fal[C::MI], fbh[C::NI], fbl[C::NI];
#pragma unroll
        for (int i = 0; i < C::MI; ++i) {
            const int row = wm * C::WM + i * 16 + lr;
            fah[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)(ah + row * P + kk * 32 + lg * 8));
            fal[i] = __builtin_bit_cast(bf16x8, *(const u16x8*)(al + row * P + kk * 32 + lg * 8));
        }
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int row = wn * C::WN + j * 16 + lr;
            fbh[j] = __builtin_bit_cast(bf16x8, *(const u16x8*)(bh + row * P + kk * 32 + lg * 8));
            fbl[j] = __builtin_bit_cast(bf16x8, *(const u16x8*)(bl + row * P + kk * 32 + lg * 8));
        }
        // each product over every accumulator in turn: an accumulator's
        // three MFMAs (small products first) are MI x NI instructions apart
        // instead of back to back, so none waits for the previous result
#pragma unroll
        for (int i = 0; i < C::MI; ++i)
#pragma unroll
            for (int j = 0; j < C::NI; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::MI; ++i)
#pragma unroll
            for (int j = 0; j < C::NI; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl[j], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < C::MI; ++i)
#pragma unroll
            for (int j = 0; j < C::NI; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh[j], acc[i][j], 0, 0, 0);
        }
    }
    };
    if (!full) kloop(std::integral_constant<int, 0>{});
    else if (!ktail) kloop(std::integral_constant<int, 1>{});
    else kloop(std::integral_constant<int, 2>{});
    __syncthreads();

    double se = 0.0, sx = 0.0;
    TC* __restrict__ Cb = (TC*)g.C + (long long)b * g.sC + (long long)m0 * g.ldc + n0;
#pragma unroll
    for (int i = 0; i < C::MI; ++i) {
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int n = wn * C::WN + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = wm * C::WM + i * 16 + 4 * lg + r;
                if (m < mrem && n < nrem)
                    epi_store<TC, EPI>(Cb, (long long)m * g.ldc + n, (double)acc[i][j][r], se, sx);
            }
        }
    }
    if constexpr (EPI == EPI_ACCUM_F64) {
        block_sum2<NT>(se, sx, red);
        if (threadIdx.x == 0) {
            g.partials[2 * lb] = se;
            g.partials[2 * lb + 1] = sx;
        }
    }
}

// ---------------------------------------------------------------------------
// Kernels: one descriptor, or a persistent loop over a work list (a block
// finds its problem by binary search on block_begin).
// ---------------------------------------------------------------------------
// PREC: GP_F64 / GP_F32 / GP_BF16X3; TA: data type of the x-pass A (or of A
// for a plain GEMM), TB: data type of the y-pass B, TC output type.
// DEEP = 1: a deep K tile in a single LDS buffer (32 for FP64/FP32, 64 for
// BF16X3).
// Threads of the plain tile kernels: DEEP 2 splits the tile over waves of
// 64 x 32 (FP64 / FP32 only).
template <int BM, int BN, int DEEP>
struct GemmThreads {
    static constexpr int NT = TileCfg<BM, BN, (BM >= 64 ? 64 : 32), (DEEP == 2 ? 32 : (BN >= 64 ? 64 : BN))>::NT;
};

template <int PREC, typename TA, typename TB, typename TC, int EPI, int BM, int BN, bool BNK, int DEEP>
struct GemmKernel {
    static __device__ __forceinline__ void tile(const GemmDesc& g, long long lb) {
        if constexpr (PREC == GP_BF16X3) {
            // DEEP 1: a 64-deep K tile (two MFMA K steps per LDS fill)
            constexpr int BKb = DEEP == 1 ? 64 : 32;
            __shared__ __attribute__((aligned(16))) uint16_t smem[SmemB<BM, BN, BKb>::TOTAL];
            __shared__ double red[2 * TileCfg<BM, BN>::NT / 64];
            if constexpr (BNK) gemm_tile_b<TA, TC, EPI, BM, BN, true, BKb>(g, lb, smem, red);
            else gemm_tile_b<TB, TC, EPI, BM, BN, false, BKb>(g, lb, smem, red);
        } else {
            typedef typename std::conditional<PREC == GP_F64, double, float>::type T;
            // DEEP 1: 32-deep K tile, single buffer; DEEP 2: waves of 64 x 32
            constexpr int BKd = DEEP == 1 ? 32 : 16, NB = DEEP == 1 ? 1 : 2;
            constexpr int WNd = DEEP == 2 ? 32 : (BN >= 64 ? 64 : BN);
            __shared__ __attribute__((aligned(16))) T smem[SmemF<T, BM, BN, BNK, BKd, NB>::TOTAL];
            __shared__ double red[2 * GemmThreads<BM, BN, DEEP>::NT / 64];
            gemm_tile_f<T, TA, TB, TC, EPI, BM, BN, BNK, BKd, NB, WNd>(g, lb, smem, red);
        }
    }
};

#define TPT_GEMM_ATTR __launch_bounds__((GemmThreads<BM, BN, DEEP>::NT))

template <int PREC, typename TA, typename TB, typename TC, int EPI, int BM, int BN, bool BNK, int DEEP>
__global__ TPT_GEMM_ATTR void gemm_kernel(GemmDesc g) {
    // neighbouring tiles share an operand (the same data rows in the x pass,
    // the same slab in the y pass): keep them on one XCD
    GemmKernel<PREC, TA, TB, TC, EPI, BM, BN, BNK, DEEP>::tile(g, xcd_block(blockIdx.x, gridDim.x));
}

// Persistent single-problem kernel (FP64 / FP32): four
// waves of 64 x 64 (WN = 64, 256 threads) or eight of 64 x 32 (WN = 32).
template <int PREC, typename TA, typename TB, typename TC, int EPI, bool BNK, int WN = 64, bool EDGE = false>
__global__ __launch_bounds__((TileCfg<128, 128, 64, WN>::NT)) void gemm_persist_kernel(GemmDesc g, long long ntiles) {
    typedef typename std::conditional<PREC == GP_F64, double, float>::type T;
    __shared__ __attribute__((aligned(16))) T smem[SmemF<T, 128, 128, BNK, 16, 2>::TOTAL];
    __shared__ double red[2 * (TileCfg<128, 128, 64, WN>::NT / 64)];
    gemm_tiles_persist_f<T, TA, TB, TC, EPI, BNK, WN, EDGE>(g, ntiles, smem, red);
}

template <int PREC, typename TA, typename TB, typename TC, int EPI, int BM, int BN, bool BNK, int DEEP>
__global__ TPT_GEMM_ATTR void gemm_multi_kernel(const GemmDesc* __restrict__ work,
                                                                            int nwork, long long total) {
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const GemmDesc g = work[lo];
        GemmKernel<PREC, TA, TB, TC, EPI, BM, BN, BNK, DEEP>::tile(g, blk - g.block_begin);
        __syncthreads();
    }
}

// Work-list kernel (FP64 / FP32): x pass 128 x 64 tiles, y pass 64 x 128
// tiles over slab-folded columns.
template <int PREC, typename TA, typename TB, typename TC, int EPI, bool BNK>
__global__ __launch_bounds__(256) void gemm_worklist_kernel(const GemmDesc* __restrict__ work, int nwork,
                                                            long long total) {
    typedef typename std::conditional<PREC == GP_F64, double, float>::type T;
    constexpr int BM = BNK ? 128 : 64, BN = BNK ? 64 : 128;
    __shared__ __attribute__((aligned(16))) T smem[SmemF<T, BM, BN, BNK, 16, 2>::TOTAL];
    __shared__ double red[2 * (256 / 64)];
    gemm_worklist_f<T, TA, TB, TC, EPI, BNK, BM, BN>(work, nwork, total, smem, red);
}

template <int PREC, typename TA, typename TB, typename TC, int EPI, bool BNK>
hipError_t launch_worklist_typed(const GemmDesc* d_work, int nwork, long long tiles, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    // three blocks per CU (the kernel's registers and 50 KB of LDS allow
    // three), a multiple of 8 so a block keeps its XCD, at most the tiles
    long long grid = persistent_gemm_grid(1LL << 40) / 2 * 3;
    grid -= grid % 8;
    if (grid > tiles) grid = tiles;
    if (grid < 1) grid = 1;
    TPT_KLAUNCH((gemm_worklist_kernel<PREC, TA, TB, TC, EPI, BNK>), dim3((unsigned)grid), dim3(256), 0, s, d_work,
                nwork, tiles);
    return hipGetLastError();
}

template <int PREC, typename TA, typename TB, typename TC, int EPI, bool BNK>
hipError_t launch_gemm_typed(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks, int variant,
                             hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
#define TPT_LAUNCH(BM_, BN_, DEEP_)                                                                              \
    do {                                                                                                         \
        constexpr int NT_ = GemmThreads<BM_, BN_, DEEP_>::NT;                                                    \
        if (d_work)                                                                                              \
            TPT_KLAUNCH((gemm_multi_kernel<PREC, TA, TB, TC, EPI, BM_, BN_, BNK, DEEP_>),                 \
                               dim3((unsigned)(blocks < PERSISTENT_BLOCKS ? blocks : PERSISTENT_BLOCKS)),        \
                               dim3(NT_), 0, s, d_work, nwork, blocks);                                          \
        else                                                                                                     \
            TPT_KLAUNCH((gemm_kernel<PREC, TA, TB, TC, EPI, BM_, BN_, BNK, DEEP_>),                       \
                               dim3((unsigned)blocks), dim3(NT_), 0, s, g);                                      \
    } while (0)
    switch (variant) {
        case TV_128x128:
            // work lists (FP64 / FP32) run the 128 x 128 tile over eight waves:
            // the work-list kernel's extra registers leave the four-wave form
            // one wave per SIMD; every output sees the same MFMA sequence, so
            // the results are those of the single-problem launch
            if constexpr (PREC != GP_BF16X3) {
                if (d_work) {
                    TPT_LAUNCH(128, 128, 2);
                    break;
                }
            }
            TPT_LAUNCH(128, 128, 0);
            break;
        case TV_64x128: TPT_LAUNCH(64, 128, 0); break;
        case TV_128x64: TPT_LAUNCH(128, 64, 0); break;
        case TV_64x64: TPT_LAUNCH(64, 64, 0); break;
        case TV_32x64: TPT_LAUNCH(32, 64, 0); break;
        case TV_128x128_K32:
            TPT_LAUNCH(128, 128, 1);
            break;
        case TV_128x128_W8:
            if constexpr (PREC == GP_BF16X3) return hipErrorInvalidValue;
            else TPT_LAUNCH(128, 128, 2);
            break;
        case TV_128x128_P:
        case TV_128x128_P8:
            if constexpr (PREC == GP_BF16X3) {
                return hipErrorInvalidValue;
            } else {
                if (d_work) {  // work lists run the plain 128 x 128 tile (eight waves)
                    TPT_LAUNCH(128, 128, 2);
                    break;
                }
                if (g.K < 1) return hipErrorInvalidValue;
                const long long grid = persistent_gemm_grid(blocks);
                const bool edge = g.M % 128 || g.N % 128 || g.K % 16;
#define TPT_PERSIST(WN_, EDGE_)                                                                        \
    TPT_KLAUNCH((gemm_persist_kernel<PREC, TA, TB, TC, EPI, BNK, WN_, EDGE_>), dim3((unsigned)grid), \
                dim3(TileCfg<128, 128, 64, WN_>::NT), 0, s, g, blocks)
                if (variant == TV_128x128_P) {
                    if (edge) TPT_PERSIST(64, true);
                    else TPT_PERSIST(64, false);
                } else {
                    if (edge) TPT_PERSIST(32, true);
                    else TPT_PERSIST(32, false);
                }
#undef TPT_PERSIST
            }
            break;
        default: return hipErrorInvalidValue;
    }
#undef TPT_LAUNCH
    return hipGetLastError();
}

}  // namespace tpt
