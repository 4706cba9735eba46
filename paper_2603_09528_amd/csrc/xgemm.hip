// Fused x transform + y GEMM (FP64).  When x is a uniform direction (fast
// transform) and y a dense eigenbasis, steps 2.1 and 2.2 of §2.2.2 (and 2.4
// and 2.5 of the inverse) touch every unknown twice in HBM if run as separate
// passes.  Here the y GEMM's operand loader applies the x transform to the
// rows it brings in, so the field is read once and the result written once:
//   forward  C_k = A (F_k Q_x^{-T})      (rows of slab k transformed, then y)
//   inverse  C_k = A (F_k Q_x^T)         (the x inverse first: the x and y
//                                         operators act on different indices
//                                         and commute)
// with A the y operator of the plan (128-row tiles of M = N_y) and F_k the
// N_y x N_x slab k.  A block computes a 128 x N_x tile (all x modes of its
// rows, so that every row it transforms is complete): 2 x N_x/64 waves of
// 64 x 64 FP64 MFMA accumulators, K steps of 16 rows.  For the next K step
// each wave transforms its own rows (16 per step over all waves) in a
// private LDS scratch with wave-level synchronisation only, using the same
// radix-2 passes as the line kernels (four points per lane), and writes them
// into the free half of the double-buffered B tile; the block synchronises
// once per K step.
//
// Measured on gfx950 (256^3, N_x = N_y = 256) the fused pass takes longer than
// the two separate passes (about 0.22 against 0.05 + 0.14 ms): the matrix
// unit is busy about half the time, as the row transforms' chains of LDS round
// trips are not hidden behind the MFMAs with eight waves per CU (the
// stand-alone transform kernel runs sixteen).  Plans use it only on request.
#include "fft_core.h"
#include "gemm_impl.h"

namespace tpt {

namespace {

using namespace fftc;

constexpr int XG_BM = 128;
constexpr int XG_BK = 16;
constexpr int XG_Q = 2;  // radix-2 stages per pass in the row transforms (four points per lane)

template <int BN> struct XgCfg {
    typedef TileCfg<XG_BM, BN> C;
    static constexpr int NT = C::NT;          // 2 BN threads
    static constexpr int NW = NT / 64;        // waves
    static constexpr int M = BN / 2;          // complex points per row
    static constexpr int MLOG = BN == 256 ? 7 : 6;
    static constexpr int T = M >> XG_Q;       // lanes per row
    static constexpr int RPW = 64 / T;        // rows per wave per K step
    static_assert(RPW * NW == XG_BK, "the waves transform the 16 rows of a K step");
    static constexpr int LS = M + M / 16 + 3;  // scratch row stride (complex points)
    static constexpr int PA = XG_BK + 1;
    static constexpr int PB = BN + 2;
    static constexpr int A_ELEMS = XG_BM * PA;  // doubles per A buffer
    static constexpr int B_ELEMS = XG_BK * PB;  // doubles per B buffer
    static constexpr int SCR = NW * RPW * LS;   // complex points of scratch
    static constexpr int LA = XG_BM * XG_BK / NT;
    static constexpr int PPL = M / T;           // row pairs loaded per lane
    static constexpr size_t LDS_BYTES =
        (size_t)(2 * A_ELEMS + 2 * B_ELEMS) * 8 + (size_t)SCR * 16 + (size_t)(2 * M + 1) * 16;
};

template <int BN, bool INV>
__global__ __launch_bounds__(2 * BN) void xgemm_kernel(GemmDesc g, FftDesc xf, long long ntiles) {
    typedef XgCfg<BN> X;
    typedef typename X::C C;
    typedef Mfma<double> MM;
    constexpr int NT = X::NT, M = X::M, N = BN, T = X::T;
    extern __shared__ __attribute__((aligned(16))) double xg_smem[];
    double* As = xg_smem;                    // [2][BM][PA]
    double* Bs = As + 2 * X::A_ELEMS;        // [2][BK][PB]
    double2* scr = (double2*)(Bs + 2 * X::B_ELEMS);
    double2* W = scr + X::SCR;               // W^k, k < M
    double2* Qt = W + M;                     // e^{-i pi k/2N}, k <= M

    const long long v = xcd_block(blockIdx.x, ntiles);
    int b, tm, tn;
    decode_tile(g, v, b, tm, tn);
    const int tid = threadIdx.x;
    const int w = tid / 64, lane = tid % 64, lr = lane % 16, lg = lane / 16;
    const int wm = w / C::WAVES_N, wn = w % C::WAVES_N;
    const int lda = g.lda, ldb = g.ldb;
    const double* __restrict__ Ab = (const double*)g.A + (long long)tm * XG_BM * lda;
    const double* __restrict__ Bb = (const double*)g.B + (long long)b * g.sB;
    const int arow = tid / XG_BK, acol = tid % XG_BK;
    // this lane's row of the K step and its index within the row
    const int rw = w * X::RPW + lane / T, t = lane % T;
    double2* sr = scr + (size_t)(w * X::RPW + lane / T) * X::LS;  // the row's scratch
    double* srd = (double*)sr;
    const int kind = xf.kind;
    const double s = xf.scale;

    for (int k = tid; k < M; k += NT) W[k] = xf.twiddle[k];
    if (kind != UT_FOURIER)
        for (int k = tid; k <= M; k += NT) Qt[k] = xf.qtw[k];

    double ra[X::LA];
    double2 rp[X::PPL];  // row pairs (2c, 2c+1), c = t + j T
    auto gload_a = [&](int kt) {
#pragma unroll
        for (int q = 0; q < X::LA; ++q)
            ra[q] = Ab[(unsigned)((arow + q * (NT / XG_BK)) * lda + kt * XG_BK + acol)];
    };
    auto gload_rows = [&](int kt) {
        const double* row = Bb + (long long)(kt * XG_BK + rw) * ldb;
#pragma unroll
        for (int j = 0; j < X::PPL; ++j) rp[j] = *(const double2*)(row + 2 * (t + j * T));
    };
    auto store_a = [&](int buf) {
        double* a = As + buf * X::A_ELEMS;
#pragma unroll
        for (int q = 0; q < X::LA; ++q) a[(arow + q * (NT / XG_BK)) * X::PA + acol] = ra[q];
    };
    // transform this wave's rows of the loaded K step into B buffer `buf`
    auto transform = [&](int buf) {
        double* brow = Bs + buf * X::B_ELEMS + rw * X::PB;
        if constexpr (!INV) {
            // v in natural order (DCT: v_c = f_2c, v_{N-1-c} = f_2c+1; DST: odd entries negated)
#pragma unroll
            for (int j = 0; j < X::PPL; ++j) {
                const int c = t + j * T;
                if (kind == UT_FOURIER) {
                    sr[pad16(c)] = rp[j];
                } else {
                    const int c2 = N - 1 - c;
                    srd[2 * pad16(c >> 1) + (c & 1)] = rp[j].x;
                    srd[2 * pad16(c2 >> 1) + (c2 & 1)] = kind == UT_DST ? -rp[j].y : rp[j].y;
                }
            }
            SyncWave::sync();
            ut_cfft_line<XG_Q, false, SyncWave>(sr, t, X::MLOG, W);
            if (kind == UT_FOURIER) {
                // outputs from the pairs (m, M-m), m < M/2: with
                // e = (Z_m + conj Z_{M-m})/2 and t = W^m (Z_m - conj Z_{M-m})/2,
                // V_m = e - i t and V_{M-m} = conj(e) - i conj(t); m = 0 gives
                // V_0, V_M (from Z_0) and the self-paired V_{M/2}
                const double c0 = s / sqrt((double)N), c1 = s * sqrt(2.0 / N);
#pragma unroll
                for (int j = 0; j < X::PPL / 2; ++j) {
                    const int m = t + j * T;
                    if (m == 0) {
                        const double2 z0 = sr[0];
                        brow[0] = c0 * (z0.x + z0.y);
                        brow[N - 1] = c0 * (z0.x - z0.y);
                        const double2 zh = sr[pad16(M / 2)];
                        const double2 e = make_double2(zh.x, 0.0);
                        const double2 tt = cmul(W[M / 2], make_double2(0.0, zh.y));
                        brow[M - 1] = c1 * (e.x + tt.y);
                        brow[M] = -c1 * (e.y - tt.x);
                    } else {
                        const double2 zm = sr[pad16(m)], zc = conj2(sr[pad16(M - m)]);
                        const double2 e = cscale(cadd(zm, zc), 0.5);
                        const double2 tt = cmul(W[m], cscale(csub(zm, zc), 0.5));
                        brow[2 * m - 1] = c1 * (e.x + tt.y);
                        brow[2 * m] = -c1 * (e.y - tt.x);
                        brow[2 * (M - m) - 1] = c1 * (e.x - tt.y);
                        brow[2 * (M - m)] = c1 * (e.y + tt.x);
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < X::PPL; ++j) {
                    const int p = t + j * T;
                    // item p gives X_p and X_{N-p} (p = 0: X_0 and X_M); DST reverses
                    const double ca = s * sqrt(1.0 / N), cb = s * sqrt(2.0 / N);
                    const bool rev = kind == UT_DST;
                    const double2 z0 = sr[0];
                    if (p == 0) {
                        brow[rev ? N - 1 : 0] = ca * (z0.x + z0.y);
                        brow[rev ? N - 1 - M : M] = cb * sqrt(0.5) * (z0.x - z0.y);
                    } else {
                        const double2 zm = sr[pad16(p)], zc = conj2(sr[pad16(M - p)]);
                        const double2 e = cscale(cadd(zm, zc), 0.5);
                        const double2 tt = cmul(W[p], cscale(csub(zm, zc), 0.5));
                        const double2 r = cmul(Qt[p], make_double2(e.x + tt.y, e.y - tt.x));
                        brow[rev ? N - 1 - p : p] = cb * r.x;
                        brow[rev ? p - 1 : N - p] = -cb * r.y;
                    }
                }
            }
        } else {
            // half spectrum F_m in natural order, F_M in the imaginary part of slot 0
            if (kind == UT_FOURIER) {
                const double cN = s * sqrt((double)N), cH = s * sqrt(0.5 * N);
#pragma unroll
                for (int j = 0; j < X::PPL; ++j) {
                    const int p = t + j * T;
                    if (p == 0) srd[0] = cN * rp[j].x;
                    else srd[2 * pad16(p) + 1] = -cH * rp[j].x;
                    if (p == M - 1) srd[1] = cN * rp[j].y;
                    else srd[2 * pad16(p + 1)] = cH * rp[j].y;
                }
            } else {
                // X_k = s c_k phihat_k (DST: read reversed), X_0 doubled; the
                // raw row goes to the scratch first (positions k), then F_m =
                // e^{i pi m/2N} (X_m - i X_{N-m}), V_0 = X_0, V_M = sqrt(2) X_M
                const bool rev = kind == UT_DST;
                const double ca = s * sqrt(1.0 / N), cb = s * sqrt(2.0 / N);
#pragma unroll
                for (int j = 0; j < X::PPL; ++j) {
                    const int c = t + j * T;
                    srd[2 * c] = rp[j].x;
                    srd[2 * c + 1] = rp[j].y;
                }
                SyncWave::sync();
                double x0[X::PPL], x1[X::PPL];
#pragma unroll
                for (int j = 0; j < X::PPL; ++j) {
                    const int m = t + j * T;
                    const int k0 = m, k1 = m == 0 ? M : N - m;
                    x0[j] = srd[rev ? N - 1 - k0 : k0];
                    x1[j] = srd[rev ? N - 1 - k1 : k1];
                }
                SyncWave::sync();
#pragma unroll
                for (int j = 0; j < X::PPL; ++j) {
                    const int m = t + j * T;
                    sr[pad16(m)] = m == 0 ? make_double2(2.0 * ca * x0[j], sqrt(2.0) * cb * x1[j])
                                          : cmul(conj2(Qt[m]), make_double2(cb * x0[j], -cb * x1[j]));
                }
            }
            SyncWave::sync();
            ut_cfft_line<XG_Q, true, SyncWave>(sr, t, X::MLOG, W);
            const double post = kind == UT_FOURIER ? 1.0 / M : 1.0;
#pragma unroll
            for (int j = 0; j < X::PPL; ++j) {
                const int c = t + j * T;
                if (kind == UT_FOURIER) {  // v_2c, v_2c+1 = z_c
                    *(double2*)(brow + 2 * c) = cscale(sr[pad16(c)], post);
                    continue;
                }
                auto vat = [&](int e) {
                    const int jj = kind == UT_FOURIER ? e : ((e & 1) ? N - 1 - (e >> 1) : (e >> 1));
                    return srd[2 * pad16(jj >> 1) + (jj & 1)] * post;
                };
                double v0 = vat(2 * c), v1 = vat(2 * c + 1);
                if (kind == UT_DST) v1 = -v1;
                *(double2*)(brow + 2 * c) = make_double2(v0, v1);
            }
        }
        SyncWave::sync();  // the scratch is rewritten by the next K step
    };

    typename MM::acc acc[C::MI][C::NI];
#pragma unroll
    for (int i = 0; i < C::MI; ++i)
#pragma unroll
        for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::zero();

    auto mfma_step = [&](int cur) {
        const double* a = As + cur * X::A_ELEMS + (wm * C::WM + lr) * X::PA + lg;
        const double* bb = Bs + cur * X::B_ELEMS;
#pragma unroll
        for (int kk = 0; kk < XG_BK / 4; ++kk) {
            double fa[C::MI], fb[C::NI];
#pragma unroll
            for (int i = 0; i < C::MI; ++i) fa[i] = a[i * 16 * X::PA + kk * 4];
#pragma unroll
            for (int j = 0; j < C::NI; ++j) fb[j] = bb[(kk * 4 + lg) * X::PB + wn * C::WN + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < C::MI; ++i)
#pragma unroll
                for (int j = 0; j < C::NI; ++j) acc[i][j] = MM::mma(fa[i], fb[j], acc[i][j]);
        }
    };

    const int nk = g.K / XG_BK;
    gload_a(0);
    gload_rows(0);
    __syncthreads();  // twiddle tables
    store_a(0);
    transform(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int cur = kt & 1;
        const bool more = kt + 1 < nk;
        if (more) {
            gload_a(kt + 1);
            gload_rows(kt + 1);
        }
        mfma_step(cur);
        if (more) {
            store_a(cur ^ 1);
            transform(cur ^ 1);
        }
        __syncthreads();
    }

    double* __restrict__ Cb = (double*)g.C + (long long)b * g.sC + (long long)tm * XG_BM * g.ldc;
#pragma unroll
    for (int i = 0; i < C::MI; ++i) {
#pragma unroll
        for (int j = 0; j < C::NI; ++j) {
            const int n = wn * C::WN + j * 16 + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = wm * C::WM + i * 16 + MM::row(lg, r);
                Cb[(long long)m * g.ldc + n] = (double)acc[i][j][r];
            }
        }
    }
}

template <int BN, bool INV>
hipError_t launch_xgemm_t(GemmDesc g, const FftDesc& xf, hipStream_t s) {
    typedef XgCfg<BN> X;
    g.tiles_m = g.M / XG_BM;
    g.tiles_n = 1;
    const long long tiles = (long long)g.tiles_m * g.batch;
    const size_t sm = X::LDS_BYTES;
    hipError_t e = hipFuncSetAttribute((const void*)xgemm_kernel<BN, INV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sm);
    if (e != hipSuccess) return e;
    TPT_KLAUNCH((xgemm_kernel<BN, INV>), dim3((unsigned)tiles), dim3(X::NT), sm, s, g, xf, tiles);
    return hipGetLastError();
}

}  // namespace

bool xgemm_supported(const GemmDesc& g, const FftDesc& xf) {
    if (xf.ylines || xf.n != g.N || (g.N != 128 && g.N != 256)) return false;
    if (xf.kind < UT_FOURIER || xf.kind > UT_DST) return false;
    if (g.M % XG_BM || g.K % XG_BK || g.b_nk || g.sA != 0) return false;
    if (g.tA != DT_F64 || g.tB != DT_F64 || g.tC != DT_F64 || g.epi != EPI_STORE) return false;
    if (g.ldb != g.N || g.ldc != g.N || g.batch <= 0 || (long long)g.M / XG_BM * g.batch > 0x7fffffffLL) return false;
    if (((uintptr_t)g.B & 15) || ((uintptr_t)g.C & 15)) return false;
    return true;
}

hipError_t launch_xgemm(const GemmDesc& g, const FftDesc& xf, hipStream_t s) {
    if (!xgemm_supported(g, xf)) return hipErrorInvalidValue;
    if (g.N == 256) return xf.inverse ? launch_xgemm_t<256, true>(g, xf, s) : launch_xgemm_t<256, false>(g, xf, s);
    return xf.inverse ? launch_xgemm_t<128, true>(g, xf, s) : launch_xgemm_t<128, false>(g, xf, s);
}

}  // namespace tpt
