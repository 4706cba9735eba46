// Fast transforms for uniform directions.  On a uniform grid the eigenbases
// of §2.2.1 are known in closed form: the real Fourier basis (periodic), the
// cosine basis DCT-II (Neumann-Neumann, cell centres) and the sine basis
// DST-II (Dirichlet-Dirichlet, cell centres); §3 lets such a direction use
// FFT-based transforms in place of the dense eigenbasis product.
//
// Bases (orthonormal; the column order of the plan's analytic bases):
//   Fourier: column 0 = 1/sqrt(N); columns 2m-1, 2m (m = 1 .. N/2-1) =
//            sqrt(2/N) cos(2 pi m i/N), sqrt(2/N) sin(2 pi m i/N); column N-1
//            = (-1)^i / sqrt(N).
//   DCT-II:  column k = c_k cos(pi k (i + 1/2)/N), c_0 = sqrt(1/N), else sqrt(2/N).
//   DST-II:  column k-1 = c_k sin(pi k (i + 1/2)/N), k = 1..N, c_N = sqrt(1/N).
// Forward fhat = Q^{-1} f = sqrt(h) Q~^T f; inverse phi = Q phihat = Q~ phihat / sqrt(h).
//
// Each transform is one real length-N FFT (N a power of two) done as an
// N/2-point complex FFT of z_n = v_2n + i v_2n+1 in LDS, with the half
// spectrum V_m = (Z_m + conj Z_{M-m})/2 - i W^m (Z_m - conj Z_{M-m})/2
// (W = e^{-2 pi i/N}, M = N/2):
//   Fourier: v = f; the outputs are the real and imaginary parts of V_m.
//   DCT-II (Makhoul's reordering): v_n = f_2n, v_{N-1-n} = f_2n+1; then
//            X_k = Re(e^{-i pi k/2N} V_k) and X_{N-k} = -Im(e^{-i pi k/2N} V_k).
//   DST-II:  the DCT-II of (-1)^i f_i with the output order reversed, since
//            sin(pi k (2i+1)/2N) = (-1)^i cos(pi (N-k) (2i+1)/2N).
// The inverses run the same steps backwards: build the half spectrum, fold it
// into Z, inverse complex FFT (decimation in frequency: natural order in,
// bit-reversed out), unpack.  Arithmetic is FP64 whatever the storage types.
//
// Lines are either contiguous (x direction, element stride 1) or strided (y
// direction: the lines of one z slab are its Nx columns, element stride Nx).
// A block of 256 threads holds LPB lines in LDS (8N bytes each; 16 KB per
// block for x lines, 32 KB for y lines).  Loads and stores walk the lines so that consecutive
// lanes touch consecutive addresses: along a line for x, across lines for y.
// The pass is memory-bound: 16 B per unknown in FP64.
#include "device_common.h"

namespace tpt {

namespace {

constexpr int UT_NT = 256;
// Lines per block: 16 KB of line data for contiguous lines, so that several
// blocks per CU overlap their load, butterfly and store phases; 32 KB for
// strided lines, whose loads and stores run across the lines of the block
// (16 lines = 128-byte runs at N = 256).  At most 64 lines; one line at
// N = 2048, whose twiddle tables take 32 KB.
__host__ __device__ inline int ut_lines_per_block(int n, int ylines) {
    if (n >= 2048) return 1;
    const int l = (ylines ? 4096 : 2048) / n;
    return l > 64 ? 64 : l;
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }
__device__ __forceinline__ int bitrev(int v, int bits) { return (int)(__brev((unsigned)v) >> (32 - bits)); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// Block geometry.  All sizes are powers of two, so work items map to (line,
// index) with shifts and masks.  Strided (y) lines: a thread always serves
// the same line (lpb divides the block size), whose start is computed once.
struct UtGeom {
    int N, M, nlog, mlog, lpb, llog;
    long long line0;
    int ly;          // y lines: this thread's line in the block
    long long ybase; // y lines: offset of element 0 of that line
    bool yvalid;
};

__device__ __forceinline__ UtGeom ut_geom(const FftDesc& d, long long blk) {
    UtGeom g;
    g.N = d.n;
    g.M = d.n >> 1;
    g.nlog = ilog2(g.N);
    g.mlog = g.nlog - 1;
    g.lpb = ut_lines_per_block(g.N, d.ylines);
    g.llog = ilog2(g.lpb);
    g.line0 = blk << g.llog;
    g.ly = threadIdx.x & (g.lpb - 1);
    g.ybase = 0;
    g.yvalid = false;
    if (d.ylines) {
        const long long line = g.line0 + g.ly;
        g.yvalid = line < d.lines;
        if (g.yvalid) {
            const long long slab = line / d.inner;
            g.ybase = slab * d.s_outer + (line - slab * d.inner);
        }
    }
    return g;
}

// Work item idx with 2^clog items per line -> line in block l and index e:
// the index runs fastest for contiguous lines, the line for strided lines.
__device__ __forceinline__ void ut_item(const FftDesc& d, const UtGeom& g, int clog, int idx, int& l, int& e) {
    if (d.ylines) {
        l = idx & (g.lpb - 1);
        e = idx >> g.llog;
    } else {
        l = idx >> clog;
        e = idx & ((1 << clog) - 1);
    }
}

__device__ __forceinline__ bool ut_valid(const FftDesc& d, const UtGeom& g, int l) {
    return d.ylines ? g.yvalid : (g.line0 + l) < d.lines;
}

// Offset of element e of block line l.
__device__ __forceinline__ long long ut_off(const FftDesc& d, const UtGeom& g, int l, int e) {
    if (d.ylines) return g.ybase + (long long)e * d.s_elem;
    return ((g.line0 + l) << g.nlog) + e;
}

// Position in v (the sequence whose real FFT is taken) of line element e.
__device__ __forceinline__ int ut_vpos(int kind, int n, int e) {
    if (kind == UT_FOURIER) return e;
    return (e & 1) ? n - 1 - (e >> 1) : (e >> 1);
}

// Forward decimation in time over M points per line (bit-reversed in,
// natural out).  Radix-2 stages are taken in pairs: a thread owns the four
// points that stages L and 2L combine (one LDS round trip and one barrier per
// pair); an odd stage count starts with one plain radix-2 stage (L = 2,
// twiddle 1).
__device__ __forceinline__ void ut_dit(double2* lds, const UtGeom& g, const double2* __restrict__ W) {
    const int glog = 8 - g.llog;  // threads per line: 256 / lpb
    const int l = threadIdx.x >> glog, t = threadIdx.x & ((1 << glog) - 1);
    double2* a = lds + ((size_t)l << g.mlog);
    int hlog = 0;
    if (g.mlog & 1) {
#pragma unroll 4
        for (int b = t; b < (g.M >> 1); b += (1 << glog)) {
            const double2 u = a[2 * b], v = a[2 * b + 1];
            a[2 * b] = cadd(u, v);
            a[2 * b + 1] = csub(u, v);
        }
        __syncthreads();
        hlog = 1;
    }
    for (; hlog < g.mlog; hlog += 2) {
        const int half = 1 << hlog, L = half << 1;
        const int s1 = g.nlog - hlog - 1;  // twiddle stride N / L
        const int s2 = s1 - 1;             // N / 2L
#pragma unroll 2
        for (int b = t; b < (g.M >> 2); b += (1 << glog)) {
            const int p = b & (half - 1);
            const int i0 = ((b >> hlog) << (hlog + 2)) + p, i1 = i0 + half, i2 = i0 + L, i3 = i2 + half;
            double2 x0 = a[i0], x1 = a[i1], x2 = a[i2], x3 = a[i3];
            const double2 w1 = W[p << s1], w2 = W[p << s2], w3 = W[(p + half) << s2];
            double2 u = cmul(x1, w1);
            x1 = csub(x0, u);
            x0 = cadd(x0, u);
            u = cmul(x3, w1);
            x3 = csub(x2, u);
            x2 = cadd(x2, u);
            u = cmul(x2, w2);
            x2 = csub(x0, u);
            x0 = cadd(x0, u);
            u = cmul(x3, w3);
            x3 = csub(x1, u);
            x1 = cadd(x1, u);
            a[i0] = x0;
            a[i1] = x1;
            a[i2] = x2;
            a[i3] = x3;
        }
        __syncthreads();
    }
}

// Inverse complex FFT (conjugate twiddles), decimation in frequency: natural
// in, bit-reversed out, unnormalised.  Stages L and L/2 taken in pairs as in
// ut_dit; an odd stage count ends with one radix-2 stage (L = 2).
__device__ __forceinline__ void ut_dif_inv(double2* lds, const UtGeom& g, const double2* __restrict__ W) {
    const int glog = 8 - g.llog;
    const int l = threadIdx.x >> glog, t = threadIdx.x & ((1 << glog) - 1);
    double2* a = lds + ((size_t)l << g.mlog);
    int hlog = g.mlog - 1;  // stage span L = 2^(hlog + 1)
    for (; hlog >= 1; hlog -= 2) {
        const int q4 = 1 << (hlog - 1);    // L / 4
        const int sa = g.nlog - hlog - 1;  // twiddle stride N / L
        const int sc = sa + 1;             // 2N / L
#pragma unroll 2
        for (int b = t; b < (g.M >> 2); b += (1 << glog)) {
            const int p = b & (q4 - 1);
            const int i0 = ((b >> (hlog - 1)) << (hlog + 1)) + p, i1 = i0 + q4, i2 = i1 + q4, i3 = i2 + q4;
            double2 x0 = a[i0], x1 = a[i1], x2 = a[i2], x3 = a[i3];
            const double2 wa = conj2(W[p << sa]), wb = conj2(W[(p + q4) << sa]), wc = conj2(W[p << sc]);
            double2 d = csub(x0, x2);
            x0 = cadd(x0, x2);
            x2 = cmul(d, wa);
            d = csub(x1, x3);
            x1 = cadd(x1, x3);
            x3 = cmul(d, wb);
            d = csub(x0, x1);
            x0 = cadd(x0, x1);
            x1 = cmul(d, wc);
            d = csub(x2, x3);
            x2 = cadd(x2, x3);
            x3 = cmul(d, wc);
            a[i0] = x0;
            a[i1] = x1;
            a[i2] = x2;
            a[i3] = x3;
        }
        __syncthreads();
    }
    if (hlog == 0) {
#pragma unroll 4
        for (int b = t; b < (g.M >> 1); b += (1 << glog)) {
            const double2 u = a[2 * b], v = a[2 * b + 1];
            a[2 * b] = cadd(u, v);
            a[2 * b + 1] = csub(u, v);
        }
        __syncthreads();
    }
}

// Copy the twiddle tables of the descriptor into LDS (after the line data):
// W^k (k < N/2) and, for the cosine and sine transforms, e^{-i pi k/2N}
// (k <= N/2).  Returns the LDS copies; the caller synchronises.
__device__ __forceinline__ void ut_tables(const FftDesc& d, const UtGeom& g, double2* lds, double2*& W,
                                          double2*& Q) {
    W = lds + ((size_t)g.lpb << g.mlog);
    Q = W + g.M;
    for (int k = threadIdx.x; k < g.M; k += UT_NT) W[k] = d.twiddle[k];
    if (d.kind != UT_FOURIER)
        for (int k = threadIdx.x; k <= g.M; k += UT_NT) Q[k] = d.qtw[k];
}

template <typename TI, typename TO>
__device__ __forceinline__ void ut_forward(const FftDesc& d, long long blk, double2* lds) {
    const UtGeom g = ut_geom(d, blk);
    double2 *W, *Q;
    ut_tables(d, g, lds, W, Q);
    const int N = g.N, M = g.M, bits = g.mlog, kind = d.kind;
    const TI* in = (const TI*)d.in;
    TO* out = (TO*)d.out;
    double* ldsd = (double*)lds;
    // 1) load into bit-reversed complex slots (v_j -> slot j/2, part j%2);
    //    up to sixteen loads in flight per thread before the LDS stores
    constexpr int UL = 16;
    const int total = g.lpb << g.nlog;
    for (int base = 0; base < total; base += UL * UT_NT) {
        double v[UL];
        int pos[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int idx = base + u * UT_NT + (int)threadIdx.x;
            int l, e;
            ut_item(d, g, g.nlog, idx, l, e);
            pos[u] = -1;
            v[u] = 0.0;
            if (idx < total && ut_valid(d, g, l)) {
                double x = (double)in[ut_off(d, g, l, e)];
                if (kind == UT_DST && (e & 1)) x = -x;
                const int j = ut_vpos(kind, N, e);
                pos[u] = (l << g.nlog) + 2 * bitrev(j >> 1, bits) + (j & 1);
                v[u] = x;
            }
        }
#pragma unroll
        for (int u = 0; u < UL; ++u)
            if (pos[u] >= 0) ldsd[pos[u]] = v[u];
    }
    __syncthreads();
    // 2) complex FFT
    ut_dit(lds, g, W);
    // 3) half spectrum and outputs, from LDS straight to memory; item m = 0
    //    also writes the output of V_M
    const double s = d.scale;
    for (int idx = threadIdx.x; idx < (g.lpb << g.mlog); idx += UT_NT) {
        int l, m;
        ut_item(d, g, g.mlog, idx, l, m);
        if (!ut_valid(d, g, l)) continue;
        const double2* a = lds + ((size_t)l << g.mlog);
        if (kind == UT_FOURIER) {
            const double c0 = s / sqrt((double)N), c1 = s * sqrt(2.0 / N);
            if (m == 0) {
                const double2 z0 = a[0];
                out[ut_off(d, g, l, 0)] = (TO)(c0 * (z0.x + z0.y));      // V_0 = Re Z_0 + Im Z_0
                out[ut_off(d, g, l, N - 1)] = (TO)(c0 * (z0.x - z0.y));  // V_M = Re Z_0 - Im Z_0
            } else {
                const double2 zm = a[m], zc = conj2(a[M - m]);
                const double2 e = cscale(cadd(zm, zc), 0.5);
                const double2 t = cmul(W[m], cscale(csub(zm, zc), 0.5));
                // V_m = e - i t; column 2m-1 takes Re V_m, column 2m takes -Im V_m
                out[ut_off(d, g, l, 2 * m - 1)] = (TO)(c1 * (e.x + t.y));
                out[ut_off(d, g, l, 2 * m)] = (TO)(-c1 * (e.y - t.x));
            }
        } else {
            const double ca = s * sqrt(1.0 / N), cb = s * sqrt(2.0 / N);
            const bool rev = kind == UT_DST;
            if (m == 0) {
                const double2 z0 = a[0];
                out[ut_off(d, g, l, rev ? N - 1 : 0)] = (TO)(ca * (z0.x + z0.y));
                // X_M = cos(pi/4) V_M
                out[ut_off(d, g, l, rev ? N - 1 - M : M)] = (TO)(cb * sqrt(0.5) * (z0.x - z0.y));
            } else {
                const double2 zm = a[m], zc = conj2(a[M - m]);
                const double2 e = cscale(cadd(zm, zc), 0.5);
                const double2 t = cmul(W[m], cscale(csub(zm, zc), 0.5));
                const double2 r = cmul(Q[m], make_double2(e.x + t.y, e.y - t.x));  // e^{-i pi m/2N} V_m
                out[ut_off(d, g, l, rev ? N - 1 - m : m)] = (TO)(cb * r.x);
                out[ut_off(d, g, l, rev ? m - 1 : N - m)] = (TO)(-cb * r.y);
            }
        }
    }
}

template <typename TI, typename TO, int EPI>
__device__ __forceinline__ void ut_inverse(const FftDesc& d, long long blk, double2* lds, double* red) {
    const UtGeom g = ut_geom(d, blk);
    double2 *W, *Q;
    ut_tables(d, g, lds, W, Q);
    __syncthreads();
    const int N = g.N, M = g.M, bits = g.mlog, kind = d.kind;
    const TI* in = (const TI*)d.in;
    const double s = d.scale;  // 1 / sqrt(h)
    // 1) half spectrum F_m, m = 0 .. M-1, in natural order; F_0 and F_M are
    //    real, and F_M rides in the imaginary part of slot 0
    for (int idx = threadIdx.x; idx < (g.lpb << g.mlog); idx += UT_NT) {
        int l, m;
        ut_item(d, g, g.mlog, idx, l, m);
        double2 F = make_double2(0.0, 0.0);
        if (ut_valid(d, g, l)) {
            if (kind == UT_FOURIER) {
                const double cN = s * sqrt((double)N), cH = s * sqrt(0.5 * N);
                if (m == 0)
                    F = make_double2(cN * (double)in[ut_off(d, g, l, 0)], cN * (double)in[ut_off(d, g, l, N - 1)]);
                else
                    F = make_double2(cH * (double)in[ut_off(d, g, l, 2 * m - 1)],
                                     -cH * (double)in[ut_off(d, g, l, 2 * m)]);
            } else {
                // X_k = s c_k phihat_k (DST: phihat read in reverse), X_0 doubled
                const bool rev = kind == UT_DST;
                const double ca = s * sqrt(1.0 / N), cb = s * sqrt(2.0 / N);
                auto X = [&](int k) -> double {
                    return (k == 0 ? 2.0 * ca : cb) * (double)in[ut_off(d, g, l, rev ? N - 1 - k : k)];
                };
                if (m == 0)
                    F = make_double2(X(0), sqrt(2.0) * X(M));  // V_0 = X_0, V_M = sqrt(2) X_M
                else
                    F = cmul(conj2(Q[m]), make_double2(X(m), -X(N - m)));  // e^{i pi m/2N}(X_m - i X_{N-m})
            }
        }
        lds[((size_t)l << g.mlog) + m] = F;
    }
    __syncthreads();
    // 2) fold the pairs (m, M-m) into Z_m = E_m + i O_m in place, with
    //    E_m = (F_m + conj F_{M-m})/2 and O_m = conj(W^m) (F_m - conj F_{M-m})/2;
    //    item 0 folds slot 0 and the self-paired slot M/2
    for (int idx = threadIdx.x; idx < (g.lpb << (g.mlog - 1)); idx += UT_NT) {
        const int l = idx >> (g.mlog - 1), m0 = idx & ((M >> 1) - 1);
        double2* a = lds + ((size_t)l << g.mlog);
        for (int rep = 0; rep < (m0 == 0 ? 2 : 1); ++rep) {
            const int m = rep == 0 ? m0 : (M >> 1);
            if (m == 0) {
                const double f0 = a[0].x, fM = a[0].y;
                a[0] = make_double2(0.5 * (f0 + fM), 0.5 * (f0 - fM));
                continue;
            }
            const int mc = M - m;
            const double2 fm = a[m], fc = a[mc];
            const double2 Em = cscale(cadd(fm, conj2(fc)), 0.5);
            const double2 Om = cmul(conj2(W[m]), cscale(csub(fm, conj2(fc)), 0.5));
            if (mc != m) {
                // E_{M-m} = conj E_m and conj(W^{M-m}) = -W^m
                const double2 Ec = conj2(Em);
                const double2 Oc = cmul(cscale(W[m], -1.0), cscale(csub(fc, conj2(fm)), 0.5));
                a[mc] = make_double2(Ec.x - Oc.y, Ec.y + Oc.x);
            }
            a[m] = make_double2(Em.x - Om.y, Em.y + Om.x);
        }
    }
    __syncthreads();
    // 3) inverse complex FFT, natural in, bit-reversed out
    ut_dif_inv(lds, g, W);
    // 4) unpack and store
    const double* ldsd = (const double*)lds;
    const double post = (kind == UT_FOURIER) ? 1.0 / M : 1.0;
    TO* out = (TO*)d.out;
    double se = 0.0, sx = 0.0;
    for (int idx = threadIdx.x; idx < (g.lpb << g.nlog); idx += UT_NT) {
        int l, e;
        ut_item(d, g, g.nlog, idx, l, e);
        if (!ut_valid(d, g, l)) continue;
        const int j = ut_vpos(kind, N, e);
        double v = ldsd[(l << g.nlog) + 2 * bitrev(j >> 1, bits) + (j & 1)] * post;
        if (kind == UT_DST && (e & 1)) v = -v;
        const long long o = ut_off(d, g, l, e);
        if constexpr (EPI == EPI_ACCUM_F64) {
            const double x = (double)out[o] + v;
            out[o] = (TO)x;
            se += v * v;
            sx += x * x;
        } else {
            out[o] = (TO)v;
        }
    }
    if constexpr (EPI == EPI_ACCUM_F64) {
        block_sum2<UT_NT>(se, sx, red);
        if (threadIdx.x == 0) {
            d.partials[2 * blk] = se;
            d.partials[2 * blk + 1] = sx;
        }
    }
}

template <typename TI, typename TO, int EPI, bool INV>
__device__ __forceinline__ void ut_block(const FftDesc& d, long long blk) {
    extern __shared__ double2 ut_smem[];
    __shared__ double red[2 * (UT_NT / 64)];
    if constexpr (INV) ut_inverse<TI, TO, EPI>(d, blk, ut_smem, red);
    else ut_forward<TI, TO>(d, blk, ut_smem);
}

// Consecutive blocks of strided lines share cache lines: y launches number
// their blocks per XCD (xcd_block).
template <typename TI, typename TO, int EPI, bool INV>
__global__ __launch_bounds__(UT_NT) void ut_kernel(FftDesc d, long long nblocks) {
    const long long b = d.ylines ? xcd_block(blockIdx.x, nblocks) : (long long)blockIdx.x;
    ut_block<TI, TO, EPI, INV>(d, b);
}

template <typename TI, typename TO, int EPI, bool INV>
__global__ __launch_bounds__(UT_NT) void ut_multi_kernel(const FftDesc* __restrict__ work, int nwork,
                                                         long long total) {
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const FftDesc d = work[lo];
        ut_block<TI, TO, EPI, INV>(d, blk - d.block_begin);
        __syncthreads();
    }
}

template <typename TI, typename TO, int EPI, bool INV>
hipError_t launch_ut_t(const FftDesc& d, const FftDesc* d_work, int nwork, long long blocks, hipStream_t s) {
    // line data, then W (N/2 entries) and the quarter-wave table (N/2 + 1)
    const size_t sm = (size_t)ut_lines_per_block(d.n, d.ylines) * d.n * sizeof(double) + (size_t)(d.n + 1) * sizeof(double2);
    if (d_work)
        TPT_KLAUNCH((ut_multi_kernel<TI, TO, EPI, INV>),
                           dim3((unsigned)(blocks < 4 * PERSISTENT_BLOCKS ? blocks : 4 * PERSISTENT_BLOCKS)),
                           dim3(UT_NT), sm, s, d_work, nwork, blocks);
    else
        TPT_KLAUNCH((ut_kernel<TI, TO, EPI, INV>), dim3((unsigned)blocks), dim3(UT_NT), sm, s, d, blocks);
    return hipGetLastError();
}

}  // namespace

bool fft_supported(int n) { return n >= 8 && n <= 2048 && (n & (n - 1)) == 0; }

long long fft_blocks(const FftDesc& d) {
    const int lpb = ut_lines_per_block(d.n, d.ylines);
    return (d.lines + lpb - 1) / lpb;
}

// rep: a representative descriptor (types, direction, epilogue, line length);
// every descriptor of a work list has the same line length n, since the
// block's line count and LDS size depend on it.
hipError_t launch_fft(const FftDesc& rep, const FftDesc* d_work, int nwork, long long blocks, hipStream_t s) {
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL || !fft_supported(rep.n)) return hipErrorInvalidValue;
    if (rep.kind < UT_FOURIER || rep.kind > UT_DST) return hipErrorInvalidValue;
    if (rep.ylines && (rep.inner <= 0 || rep.s_elem <= 0)) return hipErrorInvalidValue;
    if (!rep.inverse) {
        if (rep.epi != EPI_STORE) return hipErrorInvalidValue;
        if (rep.tin == DT_F64 && rep.tout == DT_F64) return launch_ut_t<double, double, EPI_STORE, false>(rep, d_work, nwork, blocks, s);
        if (rep.tin == DT_F64 && rep.tout == DT_F32) return launch_ut_t<double, float, EPI_STORE, false>(rep, d_work, nwork, blocks, s);
        if (rep.tin == DT_F32 && rep.tout == DT_F32) return launch_ut_t<float, float, EPI_STORE, false>(rep, d_work, nwork, blocks, s);
        return hipErrorInvalidValue;
    }
    if (rep.tin == DT_F64 && rep.tout == DT_F64 && rep.epi == EPI_STORE)
        return launch_ut_t<double, double, EPI_STORE, true>(rep, d_work, nwork, blocks, s);
    if (rep.tin == DT_F32 && rep.tout == DT_F64 && rep.epi == EPI_STORE)
        return launch_ut_t<float, double, EPI_STORE, true>(rep, d_work, nwork, blocks, s);
    if (rep.tin == DT_F32 && rep.tout == DT_F64 && rep.epi == EPI_ACCUM_F64)
        return launch_ut_t<float, double, EPI_ACCUM_F64, true>(rep, d_work, nwork, blocks, s);
    if (rep.tin == DT_F32 && rep.tout == DT_F32 && rep.epi == EPI_STORE)
        return launch_ut_t<float, float, EPI_STORE, true>(rep, d_work, nwork, blocks, s);
    return hipErrorInvalidValue;
}

}  // namespace tpt
