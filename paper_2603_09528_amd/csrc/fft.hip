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
// into Z, inverse complex FFT (conjugate twiddles), unpack.  Arithmetic is
// FP64 whatever the storage types.
//
// Complex FFT of M = 2^m points: radix-2 decimation in time grouped into
// passes of up to three stages.  A thread holds the 8 points one pass
// combines in registers (the 2^q points base + k 2^h of a radix-2^q group,
// pre-multiplied by W_{2^(h+q)}^(b bitrev(k)), b = base mod 2^h, then q
// radix-2 stages with constant twiddles); the passes exchange points through
// LDS.  The first pass takes the natural-order input at stride M/2^q, which
// is where the bit-reversed order of the usual in-place algorithm puts a
// group, so no separate reordering is needed and the output comes out in
// natural order.  LDS positions are padded by one complex per sixteen, which
// keeps the power-of-two strides of the passes off a single bank, and lines
// are an odd number of points apart.
//
// Lines are either contiguous (x direction, element stride 1) or strided (y
// direction: the lines of one z slab are its Nx columns, element stride Nx).
// A block holds LPB lines, M/8 threads per line (one thread for M <= 8),
// 256 threads (128 for N = 2048, one line): 2048 complex points, 34 KB of LDS
// plus the twiddle tables (four blocks per CU at N = 256).  Eight points per
// thread rather than sixteen: the register and LDS footprint per thread then
// allows twice the resident waves, which the memory-bound pass needs more
// than the fewer LDS round trips of radix 16.  Loads and stores walk the lines so that
// consecutive lanes touch consecutive addresses: along a line for x (16-byte
// pairs), across lines for y.  The pass is memory-bound: 16 B per unknown in
// FP64.
#include "fft_core.h"

namespace tpt {

namespace {

using namespace fftc;

constexpr int UT_Q = 3;               // radix-2 stages per pass (points per thread = 2^UT_Q)
constexpr int UT_NT = 256;            // block size (fewer for N = 2048)

__host__ __device__ inline int ut_log2(int v) {
    int l = 0;
    while ((2 << l) <= v) ++l;
    return l;
}
// threads per line, lines per block and block size for real length n
__host__ __device__ inline int ut_tpl(int n) { return (n >> 1) > (1 << UT_Q) ? (n >> 1) >> UT_Q : 1; }
__host__ __device__ inline int ut_lines_per_block(int n) { return n >= 2048 ? 1 : UT_NT / ut_tpl(n); }
__host__ __device__ inline int ut_threads(int n) { return ut_lines_per_block(n) * ut_tpl(n); }
// LDS line stride in complex points: M plus one pad slot per sixteen, plus
// three, so that the lanes of strided (y) lines, which run across lines,
// fall in different banks
__host__ __device__ inline int ut_line_stride(int n) { return (n >> 1) + (n >> 5) + 3; }
__host__ __device__ inline size_t ut_lds_bytes(int n) {
    // line data, then W (N/2 entries) and the quarter-wave table (N/2 + 1)
    return ((size_t)ut_lines_per_block(n) * ut_line_stride(n) + (size_t)n + 1) * sizeof(double2);
}

// Complex FFT of the block's lines in LDS (every thread of the block takes
// part).
template <bool INV>
__device__ __forceinline__ void ut_cfft(double2* lds, int ls, int mlog, const double2* W) {
    const int Q = mlog < UT_Q ? mlog : UT_Q;
    const int tlog = mlog - Q;
    const int l = threadIdx.x >> tlog, t = threadIdx.x & ((1 << tlog) - 1);
    ut_cfft_line<UT_Q, INV, SyncBlock>(lds + (size_t)l * ls, t, mlog, W);
}

// Block geometry.  All sizes are powers of two, so work items map to (line,
// index) with shifts and masks.  Strided (y) lines: a thread always serves
// the same line in the load and store phases (lpb divides the block size),
// whose start is computed once.
struct UtGeom {
    int N, M, nlog, mlog, lpb, llog, nt, ls;
    long long line0;
    int ly;          // y lines: this thread's line in the block
    long long ybase; // y lines: offset of element 0 of that line
    bool yvalid;
};

__device__ __forceinline__ UtGeom ut_geom(const FftDesc& d, long long blk) {
    UtGeom g;
    g.N = d.n;
    g.M = d.n >> 1;
    g.nlog = ut_log2(g.N);
    g.mlog = g.nlog - 1;
    g.lpb = ut_lines_per_block(g.N);
    g.llog = ut_log2(g.lpb);
    g.nt = ut_threads(g.N);
    g.ls = ut_line_stride(g.N);
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
// LDS double index of v_j in line l (v_j is part j%2 of complex point j/2)
__device__ __forceinline__ int ut_vslot(const UtGeom& g, int l, int j) {
    return 2 * (l * g.ls + pad16(j >> 1)) + (j & 1);
}

// Copy the twiddle tables of the descriptor into LDS (after the line data):
// W^k (k < N/2) and, for the cosine and sine transforms, e^{-i pi k/2N}
// (k <= N/2).  The caller synchronises.
__device__ __forceinline__ void ut_tables(const FftDesc& d, const UtGeom& g, double2* lds, double2*& W,
                                          double2*& Q) {
    W = lds + (size_t)g.lpb * g.ls;
    Q = W + g.M;
    for (int k = threadIdx.x; k < g.M; k += g.nt) W[k] = d.twiddle[k];
    if (d.kind != UT_FOURIER)
        for (int k = threadIdx.x; k <= g.M; k += g.nt) Q[k] = d.qtw[k];
}

// Sum (a, b) over a block of nt threads (a multiple of 64, at most UT_NT) in a
// fixed order; thread 0 gets the result.
__device__ __forceinline__ void ut_block_sum2(double& a, double& b, double* red, int nt) {
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
        for (int i = 0; i < nt / 64; ++i) {
            sa += red[2 * i];
            sb += red[2 * i + 1];
        }
        a = sa;
        b = sb;
    }
}

// The same for three values (red holds 3 nt / 64 doubles).
__device__ __forceinline__ void ut_block_sum3(double& a, double& b, double& c, double* red, int nt) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) {
        red[3 * w] = a;
        red[3 * w + 1] = b;
        red[3 * w + 2] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0, sc = 0.0;
        for (int i = 0; i < nt / 64; ++i) {
            sa += red[3 * i];
            sb += red[3 * i + 1];
            sc += red[3 * i + 2];
        }
        a = sa;
        b = sb;
        c = sc;
    }
}

template <typename T> struct Pair2;
template <> struct Pair2<double> { typedef double2 type; };
template <> struct Pair2<float> { typedef float2 type; };

template <typename TI, typename TO>
__device__ __forceinline__ void ut_forward_body(const FftDesc& d, long long blk, double2* lds, double* chk) {
    const UtGeom g = ut_geom(d, blk);
    double2 *W, *Q;
    ut_tables(d, g, lds, W, Q);
    const int N = g.N, M = g.M, kind = d.kind;
    const TI* in = (const TI*)d.in;
    TO* out = (TO*)d.out;
    double* ldsd = (double*)lds;
    // 1) load v in natural order (DST: (-1)^e f_e)
    if (!d.ylines && sizeof(TI) == 4 && ((uintptr_t)in % 16) == 0 && !d.cpart) {
        // FP32 contiguous lines: element quads (4q .. 4q+3), 16 bytes per
        // lane, so a wave moves as many bytes per load as in FP64; a block
        // holds 2048 complex points, four quads per thread
        constexpr int UQ = 4;
        const int qlog = g.mlog - 1;
        const int total = g.lpb << qlog;  // quads in the block
        for (int base = 0; base < total; base += UQ * g.nt) {
            float4 v[UQ];
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                const int l = idx >> qlog, q = idx & ((M >> 1) - 1);
                v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (idx < total && g.line0 + l < d.lines)
                    v[u] = *(const float4*)((const float*)in + ((g.line0 + l) << g.nlog) + 4 * q);
            }
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                if (idx >= total) continue;
                const int l = idx >> qlog, q = idx & ((M >> 1) - 1);
                const int c0 = 2 * q, c1 = 2 * q + 1;
                if (kind == UT_FOURIER) {
                    lds[l * g.ls + pad16(c0)] = make_double2((double)v[u].x, (double)v[u].y);
                    lds[l * g.ls + pad16(c1)] = make_double2((double)v[u].z, (double)v[u].w);
                } else {
                    ldsd[ut_vslot(g, l, c0)] = (double)v[u].x;
                    ldsd[ut_vslot(g, l, N - 1 - c0)] = kind == UT_DST ? -(double)v[u].y : (double)v[u].y;
                    ldsd[ut_vslot(g, l, c1)] = (double)v[u].z;
                    ldsd[ut_vslot(g, l, N - 1 - c1)] = kind == UT_DST ? -(double)v[u].w : (double)v[u].w;
                }
            }
        }
    } else if (!d.ylines) {
        // contiguous lines: element pairs (2c, 2c+1), 16 (FP64) or 8 (FP32)
        // bytes per lane when the line data is aligned to it
        constexpr int UL = 1 << UT_Q;
        const int total = g.lpb << g.mlog;  // pairs in the block
        const bool vec = ((uintptr_t)in % sizeof(typename Pair2<TI>::type)) == 0;
        // fused right-hand-side check: volume-weighted sums of the finite
        // values and the count of the others.  Where the block size is a
        // multiple of M (N <= 512) a thread's items share one pair position
        // c, so its x weights are loaded once; the block's lines lie in one
        // rhs, so the (j, k) of line l follow from those of its first line.
        double cs = 0.0, ca = 0.0, cbad = 0.0;
        double cwx0 = 0.0, cwx1 = 0.0, cwx2 = 0.0, cwx3 = 0.0;
        unsigned crr0 = 0;
        const bool cfix = (g.nt & (M - 1)) == 0;
        // M = 2 nt (N = 1024): item u sits at pair position c + (u & 1) nt,
        // so the two weight pairs are loaded once as well
        const bool chalf = !cfix && 2 * g.nt == M;
        if (d.cpart) {
            const int c = (int)threadIdx.x & (M - 1);
            cwx0 = d.cvx[2 * c];
            cwx1 = d.cvx[2 * c + 1];
            if (chalf) {
                cwx2 = d.cvx[2 * (c + g.nt)];
                cwx3 = d.cvx[2 * (c + g.nt) + 1];
            }
            crr0 = (unsigned)g.line0 % d.crows;
        }
        for (int base = 0; base < total; base += UL * g.nt) {
            double2 v[UL];
            double wyz[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                const int l = idx >> g.mlog, c = idx & (M - 1);
                v[u] = make_double2(0.0, 0.0);
                wyz[u] = 0.0;
                if (idx < total && g.line0 + l < d.lines) {
                    if (d.cpart) wyz[u] = d.cvyz[crr0 + (unsigned)l];
                    const long long o = ((g.line0 + l) << g.nlog) + 2 * c;
                    if (vec) {
                        const typename Pair2<TI>::type p = *(const typename Pair2<TI>::type*)(in + o);
                        v[u] = make_double2((double)p.x, (double)p.y);
                    } else {
                        v[u] = make_double2((double)in[o], (double)in[o + 1]);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                if (idx >= total) continue;
                const int l = idx >> g.mlog, c = idx & (M - 1);
                if (d.cpart) {
                    // items past the last line hold zeros (finite, weight 0)
                    const bool odd = (u & 1) != 0;
                    const double wx0 = cfix ? cwx0 : chalf ? (odd ? cwx2 : cwx0) : d.cvx[2 * c];
                    const double wx1 = cfix ? cwx1 : chalf ? (odd ? cwx3 : cwx1) : d.cvx[2 * c + 1];
                    const bool f0 = __builtin_isfinite(v[u].x), f1 = __builtin_isfinite(v[u].y);
                    const double x0 = f0 ? v[u].x : 0.0, x1 = f1 ? v[u].y : 0.0;
                    cs += wyz[u] * (wx0 * x0 + wx1 * x1);
                    ca += wyz[u] * (wx0 * __builtin_fabs(x0) + wx1 * __builtin_fabs(x1));
                    cbad += (f0 ? 0.0 : 1.0) + (f1 ? 0.0 : 1.0);
                }
                if (kind == UT_FOURIER) {
                    lds[l * g.ls + pad16(c)] = v[u];
                } else {
                    // v_c = f_2c, v_{N-1-c} = f_2c+1 (negated for DST)
                    ldsd[ut_vslot(g, l, c)] = v[u].x;
                    ldsd[ut_vslot(g, l, N - 1 - c)] = kind == UT_DST ? -v[u].y : v[u].y;
                }
            }
        }
        chk[0] = cs;
        chk[1] = ca;
        chk[2] = cbad;
    } else {
        constexpr int UL = 16;
        const int total = g.lpb << g.nlog;
        for (int base = 0; base < total; base += UL * g.nt) {
            double v[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                const int e = idx >> g.llog;
                v[u] = 0.0;
                if (idx < total && g.yvalid) v[u] = (double)in[g.ybase + (long long)e * d.s_elem];
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                if (idx >= total) continue;
                const int e = idx >> g.llog;
                const double x = (kind == UT_DST && (e & 1)) ? -v[u] : v[u];
                ldsd[ut_vslot(g, g.ly, ut_vpos(kind, N, e))] = x;
            }
        }
    }
    __syncthreads();
    // 2) complex FFT of z_n = v_2n + i v_2n+1
    ut_cfft<false>(lds, g.ls, g.mlog, W);
    // 3) half spectrum and outputs, from LDS straight to memory
    const double s = d.scale;
    if (kind == UT_FOURIER && !d.ylines && sizeof(TO) == 4 && ((uintptr_t)out % 16) == 0) {
        // FP32 contiguous lines: item q writes the quad (4q .. 4q+3), the
        // output pairs of p = 2q and 2q + 1 (see below), 16 bytes per lane
        const double c0 = s / sqrt((double)N), c1 = s * sqrt(2.0 / N);
        const int qlog = g.mlog - 1;
        for (int idx = threadIdx.x; idx < (g.lpb << qlog); idx += g.nt) {
            const int l = idx >> qlog, q = idx & ((M >> 1) - 1);
            if (g.line0 + l >= d.lines) continue;
            const double2* a = lds + (size_t)l * g.ls;
            auto vm = [&](int m) {  // V_m, 0 < m < M
                const double2 zm = a[pad16(m)], zc = conj2(a[pad16(M - m)]);
                const double2 e = cscale(cadd(zm, zc), 0.5);
                const double2 t = cmul(W[m], cscale(csub(zm, zc), 0.5));
                return make_double2(e.x + t.y, e.y - t.x);
            };
            const double2 z0 = a[0];
            const int p0 = 2 * q, p1 = 2 * q + 1;
            const double lo0 = p0 == 0 ? c0 * (z0.x + z0.y) : -c1 * vm(p0).y;
            const double hi0 = c1 * vm(p0 + 1).x;
            const double lo1 = -c1 * vm(p1).y;
            const double hi1 = p1 == M - 1 ? c0 * (z0.x - z0.y) : c1 * vm(p1 + 1).x;
            *(float4*)((float*)out + ((g.line0 + l) << g.nlog) + 4 * q) =
                make_float4((float)lo0, (float)hi0, (float)lo1, (float)hi1);
        }
        return;
    }
    if (kind == UT_FOURIER && !d.ylines && ((uintptr_t)out % sizeof(typename Pair2<TO>::type)) == 0) {
        // contiguous lines: item p writes the output pair (2p, 2p+1) =
        // (-Im V_p, Re V_{p+1}) scaled, with V_0 and V_M at the two ends
        const double c0 = s / sqrt((double)N), c1 = s * sqrt(2.0 / N);
        for (int idx = threadIdx.x; idx < (g.lpb << g.mlog); idx += g.nt) {
            const int l = idx >> g.mlog, p = idx & (M - 1);
            if (g.line0 + l >= d.lines) continue;
            const double2* a = lds + (size_t)l * g.ls;
            auto vm = [&](int m) {  // V_m, 0 < m < M
                const double2 zm = a[pad16(m)], zc = conj2(a[pad16(M - m)]);
                const double2 e = cscale(cadd(zm, zc), 0.5);
                const double2 t = cmul(W[m], cscale(csub(zm, zc), 0.5));
                return make_double2(e.x + t.y, e.y - t.x);
            };
            const double2 z0 = a[0];
            const double lo = p == 0 ? c0 * (z0.x + z0.y) : -c1 * vm(p).y;
            const double hi = p == M - 1 ? c0 * (z0.x - z0.y) : c1 * vm(p + 1).x;
            typename Pair2<TO>::type o;
            o.x = (TO)lo;
            o.y = (TO)hi;
            *(typename Pair2<TO>::type*)(out + ((g.line0 + l) << g.nlog) + 2 * p) = o;
        }
        return;
    }
    // item m = 0 also writes the output of V_M
    for (int idx = threadIdx.x; idx < (g.lpb << g.mlog); idx += g.nt) {
        int l, m;
        ut_item(d, g, g.mlog, idx, l, m);
        if (!ut_valid(d, g, l)) continue;
        const double2* a = lds + (size_t)l * g.ls;
        if (kind == UT_FOURIER) {
            const double c0 = s / sqrt((double)N), c1 = s * sqrt(2.0 / N);
            if (m == 0) {
                const double2 z0 = a[0];
                out[ut_off(d, g, l, 0)] = (TO)(c0 * (z0.x + z0.y));      // V_0 = Re Z_0 + Im Z_0
                out[ut_off(d, g, l, N - 1)] = (TO)(c0 * (z0.x - z0.y));  // V_M = Re Z_0 - Im Z_0
            } else {
                const double2 zm = a[pad16(m)], zc = conj2(a[pad16(M - m)]);
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
                const double2 zm = a[pad16(m)], zc = conj2(a[pad16(M - m)]);
                const double2 e = cscale(cadd(zm, zc), 0.5);
                const double2 t = cmul(W[m], cscale(csub(zm, zc), 0.5));
                const double2 r = cmul(Q[m], make_double2(e.x + t.y, e.y - t.x));  // e^{-i pi m/2N} V_m
                out[ut_off(d, g, l, rev ? N - 1 - m : m)] = (TO)(cb * r.x);
                out[ut_off(d, g, l, rev ? m - 1 : N - m)] = (TO)(-cb * r.y);
            }
        }
    }
}

// The forward transform; with a fused right-hand-side check (x lines) the
// block's sums are reduced after its stores, where the barriers cost least,
// into one partial record per block.
template <typename TI, typename TO>
__device__ __forceinline__ void ut_forward(const FftDesc& d, long long blk, double2* lds, double* red) {
    double chk[3] = {0.0, 0.0, 0.0};
    ut_forward_body<TI, TO>(d, blk, lds, chk);
    if (d.cpart && !d.ylines) {
        ut_block_sum3(chk[0], chk[1], chk[2], red, ut_threads(d.n));
        if (threadIdx.x == 0) {
            double* q = d.cpart + 4 * blk;
            q[0] = chk[0];
            q[1] = chk[1];
            q[2] = chk[2];
            q[3] = 0.0;
        }
    }
}

template <typename TI, typename TO, int EPI>
__device__ __forceinline__ void ut_inverse(const FftDesc& d, long long blk, double2* lds, double* red) {
    const UtGeom g = ut_geom(d, blk);
    double2 *W, *Q;
    ut_tables(d, g, lds, W, Q);
    __syncthreads();
    const int N = g.N, M = g.M, kind = d.kind;
    const TI* in = (const TI*)d.in;
    const double s = d.scale;  // 1 / sqrt(h)
    // 1) half spectrum F_m, m = 0 .. M-1, in natural order; F_0 and F_M are
    //    real, and F_M rides in the imaginary part of slot 0.  Inputs of up
    //    to eight items are loaded before they are combined.
    constexpr int UL = 1 << UT_Q;
    const int total = g.lpb << g.mlog;
    if (kind == UT_FOURIER && !d.ylines && sizeof(TI) == 4 && ((uintptr_t)in % 16) == 0) {
        // FP32 contiguous lines: item q loads the quad (4q .. 4q+3), the input
        // pairs of p = 2q and 2q + 1 (see below), 16 bytes per lane
        const double cN = s * sqrt((double)N), cH = s * sqrt(0.5 * N);
        double* ldsd = (double*)lds;
        constexpr int UQ = 4;
        const int qlog = g.mlog - 1;
        const int tq = g.lpb << qlog;
        for (int base = 0; base < tq; base += UQ * g.nt) {
            float4 v[UQ];
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                const int l = idx >> qlog, q = idx & ((M >> 1) - 1);
                v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (idx < tq && g.line0 + l < d.lines)
                    v[u] = *(const float4*)((const float*)in + ((g.line0 + l) << g.nlog) + 4 * q);
            }
#pragma unroll
            for (int u = 0; u < UQ; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                if (idx >= tq) continue;
                const int l = idx >> qlog, q = idx & ((M >> 1) - 1);
                const int row = 2 * l * g.ls;
                const int p0 = 2 * q, p1 = 2 * q + 1;
                if (p0 == 0) ldsd[row] = cN * (double)v[u].x;
                else ldsd[row + 2 * pad16(p0) + 1] = -cH * (double)v[u].x;
                ldsd[row + 2 * pad16(p0 + 1)] = cH * (double)v[u].y;
                ldsd[row + 2 * pad16(p1) + 1] = -cH * (double)v[u].z;
                if (p1 == M - 1) ldsd[row + 1] = cN * (double)v[u].w;
                else ldsd[row + 2 * pad16(p1 + 1)] = cH * (double)v[u].w;
            }
        }
    } else if (kind == UT_FOURIER && !d.ylines && ((uintptr_t)in % sizeof(typename Pair2<TI>::type)) == 0) {
        // contiguous lines: item p loads the input pair (2p, 2p+1); 2p is
        // -Im F_p / cH (Re F_0 / cN for p = 0) and 2p+1 is Re F_{p+1} / cH
        // (Im F_0 / cN for p = M-1: F_M rides in slot 0)
        const double cN = s * sqrt((double)N), cH = s * sqrt(0.5 * N);
        double* ldsd = (double*)lds;
        for (int base = 0; base < total; base += UL * g.nt) {
            double2 v[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                const int l = idx >> g.mlog, p = idx & (M - 1);
                v[u] = make_double2(0.0, 0.0);
                if (idx < total && g.line0 + l < d.lines) {
                    const typename Pair2<TI>::type q =
                        *(const typename Pair2<TI>::type*)(in + ((g.line0 + l) << g.nlog) + 2 * p);
                    v[u] = make_double2((double)q.x, (double)q.y);
                }
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int idx = base + u * g.nt + (int)threadIdx.x;
                if (idx >= total) continue;
                const int l = idx >> g.mlog, p = idx & (M - 1);
                const int row = 2 * l * g.ls;
                if (p == 0) ldsd[row] = cN * v[u].x;
                else ldsd[row + 2 * pad16(p) + 1] = -cH * v[u].x;
                if (p == M - 1) ldsd[row + 1] = cN * v[u].y;
                else ldsd[row + 2 * pad16(p + 1)] = cH * v[u].y;
            }
        }
    } else
    for (int base = 0; base < total; base += UL * g.nt) {
        double p0[UL], p1[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int idx = base + u * g.nt + (int)threadIdx.x;
            int l, m;
            ut_item(d, g, g.mlog, idx, l, m);
            p0[u] = 0.0;
            p1[u] = 0.0;
            if (idx < total && ut_valid(d, g, l)) {
                int k0, k1;
                if (kind == UT_FOURIER) {
                    k0 = m == 0 ? 0 : 2 * m - 1;
                    k1 = m == 0 ? N - 1 : 2 * m;
                } else {
                    // X_k at k = m and N - m (m = 0: X_0 and X_M); DST reads reversed
                    k0 = m;
                    k1 = m == 0 ? M : N - m;
                    if (kind == UT_DST) {
                        k0 = N - 1 - k0;
                        k1 = N - 1 - k1;
                    }
                }
                p0[u] = (double)in[ut_off(d, g, l, k0)];
                p1[u] = (double)in[ut_off(d, g, l, k1)];
            }
        }
#pragma unroll
        for (int u = 0; u < UL; ++u) {
            const int idx = base + u * g.nt + (int)threadIdx.x;
            if (idx >= total) continue;
            int l, m;
            ut_item(d, g, g.mlog, idx, l, m);
            double2 F;
            if (kind == UT_FOURIER) {
                const double cN = s * sqrt((double)N), cH = s * sqrt(0.5 * N);
                F = m == 0 ? make_double2(cN * p0[u], cN * p1[u]) : make_double2(cH * p0[u], -cH * p1[u]);
            } else {
                // X_k = s c_k phihat_k, X_0 doubled; V_0 = X_0, V_M = sqrt(2) X_M,
                // V_m = e^{i pi m/2N} (X_m - i X_{N-m})
                const double ca = s * sqrt(1.0 / N), cb = s * sqrt(2.0 / N);
                F = m == 0 ? make_double2(2.0 * ca * p0[u], sqrt(2.0) * cb * p1[u])
                           : cmul(conj2(Q[m]), make_double2(cb * p0[u], -cb * p1[u]));
            }
            lds[(size_t)l * g.ls + pad16(m)] = F;
        }
    }
    __syncthreads();
    // 2) fold into Z and inverse complex FFT, natural order out
    ut_cfft<true>(lds, g.ls, g.mlog, W);
    // 3) unpack and store
    const double* ldsd = (const double*)lds;
    const double post = (kind == UT_FOURIER) ? 1.0 / M : 1.0;
    TO* out = (TO*)d.out;
    double se = 0.0, sx = 0.0;
    if (!d.ylines && ((uintptr_t)out % sizeof(typename Pair2<TO>::type)) == 0) {
        // contiguous lines: item c stores the output pair (2c, 2c+1)
        for (int idx = threadIdx.x; idx < (g.lpb << g.mlog); idx += g.nt) {
            const int l = idx >> g.mlog, c = idx & (M - 1);
            if (g.line0 + l >= d.lines) continue;
            double v0 = ldsd[ut_vslot(g, l, ut_vpos(kind, N, 2 * c))] * post;
            double v1 = ldsd[ut_vslot(g, l, ut_vpos(kind, N, 2 * c + 1))] * post;
            if (kind == UT_DST) v1 = -v1;
            typename Pair2<TO>::type* o = (typename Pair2<TO>::type*)(out + ((g.line0 + l) << g.nlog) + 2 * c);
            if constexpr (EPI == EPI_ACCUM_F64) {
                const typename Pair2<TO>::type prev = *o;
                const double x0 = (double)prev.x + v0, x1 = (double)prev.y + v1;
                typename Pair2<TO>::type r;
                r.x = (TO)x0;
                r.y = (TO)x1;
                *o = r;
                se += v0 * v0 + v1 * v1;
                sx += x0 * x0 + x1 * x1;
            } else {
                typename Pair2<TO>::type r;
                r.x = (TO)v0;
                r.y = (TO)v1;
                *o = r;
            }
        }
    } else
    for (int idx = threadIdx.x; idx < (g.lpb << g.nlog); idx += g.nt) {
        int l, e;
        ut_item(d, g, g.nlog, idx, l, e);
        if (!ut_valid(d, g, l)) continue;
        double v = ldsd[ut_vslot(g, l, ut_vpos(kind, N, e))] * post;
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
        ut_block_sum2(se, sx, red, g.nt);
        if (threadIdx.x == 0) {
            d.partials[2 * blk] = se;
            d.partials[2 * blk + 1] = sx;
        }
    }
}

template <typename TI, typename TO, int EPI, bool INV>
__device__ __forceinline__ void ut_block(const FftDesc& d, long long blk) {
    extern __shared__ double2 ut_smem[];
    __shared__ double red[3 * (UT_NT / 64)];
    if constexpr (INV) ut_inverse<TI, TO, EPI>(d, blk, ut_smem, red);
    else ut_forward<TI, TO>(d, blk, ut_smem, red);
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
    const size_t sm = ut_lds_bytes(d.n);
    const dim3 nt(ut_threads(d.n));
    if (d_work)
        TPT_KLAUNCH((ut_multi_kernel<TI, TO, EPI, INV>),
                           dim3((unsigned)(blocks < 4 * PERSISTENT_BLOCKS ? blocks : 4 * PERSISTENT_BLOCKS)),
                           nt, sm, s, d_work, nwork, blocks);
    else
        TPT_KLAUNCH((ut_kernel<TI, TO, EPI, INV>), dim3((unsigned)blocks), nt, sm, s, d, blocks);
    return hipGetLastError();
}

}  // namespace

bool fft_supported(int n) { return n >= 8 && n <= 2048 && (n & (n - 1)) == 0; }

int fft_lines_per_block(int n) { return ut_lines_per_block(n); }

long long fft_blocks(const FftDesc& d) {
    const int lpb = ut_lines_per_block(d.n);
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
