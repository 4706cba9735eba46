// Uniform periodic x direction: the real-Fourier eigenbasis applied with a
// fast transform instead of a dense GEMM (the "F" option of §3: a uniform
// direction may use FFT-based transforms; the eigenvalues are the analytic
// modified wavenumbers of §2.2.1).
//
// Basis (orthonormal, matching the analytic basis of the plan): column 0 is
// 1/sqrt(N); columns 2m-1, 2m (m = 1 .. N/2-1) are sqrt(2/N) cos(2 pi m i/N)
// and sqrt(2/N) sin(2 pi m i/N); column N-1 is (-1)^i / sqrt(N) (N even).
// Forward  fhat = Q^{-1} f = sqrt(h) Q~^T f ; inverse phi = Q phihat = Q~ phihat / sqrt(h).
//
// A length-N real line is packed as N/2 complex points z_n = f_2n + i f_2n+1,
// transformed by a radix-2 decimation-in-time FFT in LDS (bit-reversed load,
// in-place butterflies), and split into the half spectrum
// F_m = (Z_m + conj Z_{M-m})/2 - i W^m (Z_m - conj Z_{M-m})/2, W = e^{-2 pi i/N};
// the inverse runs the same steps backwards.  Arithmetic is FP64 whatever the
// storage types.  One wave per line, four lines per block; the pass is
// memory-bound (16 B per unknown in FP64).
#include "device_common.h"

namespace tpt {

// Lines (waves) per block: 4 up to N = 512, 2 for N = 1024, 1 for N = 2048,
// so that F (N/2 + 1 points) and Z (N/2 points) of every line fit in 64 KB.
static int fft_lines_per_block(int n) { return n <= 512 ? 4 : (n <= 1024 ? 2 : 1); }

// Sum (a, b) over the waves of the block; thread 0 gets the result.
__device__ __forceinline__ void block_sum2_rt(double& a, double& b, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64, nw = blockDim.x / 64;
    __syncthreads();
    if (l == 0) {
        red[2 * w] = a;
        red[2 * w + 1] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < nw; ++i) {
            sa += red[2 * i];
            sb += red[2 * i + 1];
        }
        a = sa;
        b = sb;
    }
}

__device__ __forceinline__ int bitrev(int v, int bits) { return (int)(__brev((unsigned)v) >> (32 - bits)); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

template <typename T>
__device__ __forceinline__ double ld(const T* p, long long i) {
    return (double)p[i];
}

// In-place radix-2 DIT butterflies over M points held in LDS (bit-reversed
// order on entry, natural order on exit).  W: e^{-2 pi i k/N}, k < N/2.
template <bool INV>
__device__ __forceinline__ void fft_stages(double2* a, int M, int N, const double2* __restrict__ W, int lane) {
    for (int L = 2; L <= M; L <<= 1) {
        const int half = L >> 1;
        const int tstep = N / L;
        for (int b = lane; b < (M >> 1); b += 64) {
            const int g = b / half, pos = b - g * half;
            const int i0 = g * L + pos, i1 = i0 + half;
            double2 w = W[pos * tstep];
            if (INV) w = conj2(w);
            const double2 u = a[i0];
            const double2 v = cmul(a[i1], w);
            a[i0] = make_double2(u.x + v.x, u.y + v.y);
            a[i1] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

template <typename TI, typename TO, int EPI>
__device__ __forceinline__ void fft_fwd_block(const FftDesc& d, long long blk, double2* smem, double* red) {
    const int N = d.n, M = N >> 1, bits = 31 - __clz(M);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64, lpb = blockDim.x / 64;
    const long long line = blk * lpb + w;
    const bool valid = line < d.lines;
    double2* a = smem + w * (2 * M + 1);
    const TI* in = (const TI*)d.in + line * (long long)N;
    if (valid)
        for (int n = lane; n < M; n += 64) a[bitrev(n, bits)] = make_double2(ld(in, 2 * n), ld(in, 2 * n + 1));
    __syncthreads();
    fft_stages<false>(a, M, N, d.twiddle, lane);
    double se = 0.0, sx = 0.0;
    if (valid) {
        TO* out = (TO*)d.out + line * (long long)N;
        const double c0 = d.scale / sqrt((double)N), c1 = d.scale * sqrt(2.0 / N);
        for (int m = lane; m <= M; m += 64) {
            const double2 zm = a[m == M ? 0 : m];
            const double2 zc = conj2(a[m == 0 ? 0 : M - m]);
            if (m == 0) {
                out[0] = (TO)(c0 * (zm.x + zm.y));  // F_0 = Re Z_0 + Im Z_0
            } else if (m == M) {
                out[N - 1] = (TO)(c0 * (zm.x - zm.y));  // F_M = Re Z_0 - Im Z_0
            } else {
                const double2 s = make_double2(0.5 * (zm.x + zc.x), 0.5 * (zm.y + zc.y));
                const double2 df = make_double2(0.5 * (zm.x - zc.x), 0.5 * (zm.y - zc.y));
                const double2 t = cmul(d.twiddle[m], df);  // W^m (Z_m - conj Z_{M-m}) / 2
                // F_m = s - i t
                const double fr = s.x + t.y, fi = s.y - t.x;
                out[2 * m - 1] = (TO)(c1 * fr);
                out[2 * m] = (TO)(-c1 * fi);
            }
        }
    }
    (void)se;
    (void)sx;
    (void)red;
}


template <typename TI, typename TO, int EPI>
__device__ __forceinline__ void fft_inv_block(const FftDesc& d, long long blk, double2* smem, double* red) {
    const int N = d.n, M = N >> 1, bits = 31 - __clz(M);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64, lpb = blockDim.x / 64;
    const long long line = blk * lpb + w;
    const bool valid = line < d.lines;
    double2* F = smem + w * (2 * M + 1);  // half spectrum F_0 .. F_M
    double2* Z = F + (M + 1);             // Z in bit-reversed order
    const TI* in = (const TI*)d.in + line * (long long)N;
    const double s = d.scale;  // 1 / sqrt(h)
    const double cN = s * sqrt((double)N), cH = s * sqrt(0.5 * N);
    if (valid) {
        for (int m = lane; m <= M; m += 64) {
            double2 v;
            if (m == 0) v = make_double2(cN * ld(in, 0), 0.0);
            else if (m == M) v = make_double2(cN * ld(in, N - 1), 0.0);
            else v = make_double2(cH * ld(in, 2 * m - 1), -cH * ld(in, 2 * m));
            F[m] = v;
        }
    }
    __syncthreads();
    // Z_m = E_m + i O_m, E = (F_m + conj F_{M-m})/2, O = conj(W^m) (F_m - conj F_{M-m})/2
    if (valid) {
        for (int m = lane; m < M; m += 64) {
            const double2 fm = F[m], fc = conj2(F[M - m]);
            const double2 e = make_double2(0.5 * (fm.x + fc.x), 0.5 * (fm.y + fc.y));
            const double2 df = make_double2(0.5 * (fm.x - fc.x), 0.5 * (fm.y - fc.y));
            const double2 o = cmul(conj2(d.twiddle[m]), df);
            Z[bitrev(m, bits)] = make_double2(e.x - o.y, e.y + o.x);  // e + i o
        }
    }
    __syncthreads();
    fft_stages<true>(Z, M, N, d.twiddle, lane);
    double se = 0.0, sx = 0.0;
    if (valid) {
        TO* out = (TO*)d.out + line * (long long)N;
        const double inv = 1.0 / M;
        for (int n = lane; n < M; n += 64) {
            const double2 z = Z[n];
            const double v0 = z.x * inv, v1 = z.y * inv;
            if constexpr (EPI == EPI_ACCUM_F64) {
                const double x0 = (double)out[2 * n] + v0, x1 = (double)out[2 * n + 1] + v1;
                out[2 * n] = (TO)x0;
                out[2 * n + 1] = (TO)x1;
                se += v0 * v0 + v1 * v1;
                sx += x0 * x0 + x1 * x1;
            } else {
                out[2 * n] = (TO)v0;
                out[2 * n + 1] = (TO)v1;
            }
        }
    }
    if constexpr (EPI == EPI_ACCUM_F64) {
        block_sum2_rt(se, sx, red);
        if (threadIdx.x == 0) {
            d.partials[2 * blk] = se;
            d.partials[2 * blk + 1] = sx;
        }
    }
}

template <typename TI, typename TO, int EPI, bool INV>
__device__ __forceinline__ void fft_block(const FftDesc& d, long long blk) {
    extern __shared__ double2 fft_smem[];
    __shared__ double red[2 * 4];
    if constexpr (INV) fft_inv_block<TI, TO, EPI>(d, blk, fft_smem, red);
    else fft_fwd_block<TI, TO, EPI>(d, blk, fft_smem, red);
}

template <typename TI, typename TO, int EPI, bool INV>
__global__ __launch_bounds__(256) void fft_kernel(FftDesc d) {
    fft_block<TI, TO, EPI, INV>(d, blockIdx.x);
}

template <typename TI, typename TO, int EPI, bool INV>
__global__ __launch_bounds__(256) void fft_multi_kernel(const FftDesc* __restrict__ work, int nwork,
                                                                   long long total) {
    for (long long blk = blockIdx.x; blk < total; blk += gridDim.x) {
        int lo = 0, hi = nwork - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (work[mid].block_begin <= blk) lo = mid;
            else hi = mid - 1;
        }
        const FftDesc d = work[lo];
        fft_block<TI, TO, EPI, INV>(d, blk - d.block_begin);
        __syncthreads();
    }
}

long long fft_blocks(const FftDesc& d) {
    const int lpb = fft_lines_per_block(d.n);
    return (d.lines + lpb - 1) / lpb;
}

bool fft_supported(int n) { return n >= 8 && n <= 2048 && (n & (n - 1)) == 0; }

template <typename TI, typename TO, int EPI, bool INV>
static hipError_t launch_fft_t(const FftDesc& d, const FftDesc* d_work, int nwork, long long blocks, int n,
                               hipStream_t s) {
    const int lpb = fft_lines_per_block(n);
    const size_t sm = (size_t)lpb * (n + 1) * sizeof(double2);
    if (d_work)
        hipLaunchKernelGGL((fft_multi_kernel<TI, TO, EPI, INV>),
                           dim3((unsigned)(blocks < 4 * PERSISTENT_BLOCKS ? blocks : 4 * PERSISTENT_BLOCKS)),
                           dim3(64 * lpb), sm, s, d_work, nwork, blocks);
    else
        hipLaunchKernelGGL((fft_kernel<TI, TO, EPI, INV>), dim3((unsigned)blocks), dim3(64 * lpb), sm, s, d);
    return hipGetLastError();
}

// rep: a representative descriptor (types, direction, epilogue); every
// descriptor of a work list has the same line length n (the block shape and
// LDS size depend on it).
hipError_t launch_fft(const FftDesc& rep, const FftDesc* d_work, int nwork, long long blocks, hipStream_t s) {
    const int nmax = rep.n;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffffLL || !fft_supported(nmax)) return hipErrorInvalidValue;
    if (!rep.inverse) {
        if (rep.epi != EPI_STORE) return hipErrorInvalidValue;
        if (rep.tin == DT_F64 && rep.tout == DT_F64) return launch_fft_t<double, double, EPI_STORE, false>(rep, d_work, nwork, blocks, nmax, s);
        if (rep.tin == DT_F64 && rep.tout == DT_F32) return launch_fft_t<double, float, EPI_STORE, false>(rep, d_work, nwork, blocks, nmax, s);
        if (rep.tin == DT_F32 && rep.tout == DT_F32) return launch_fft_t<float, float, EPI_STORE, false>(rep, d_work, nwork, blocks, nmax, s);
        return hipErrorInvalidValue;
    }
    if (rep.tin == DT_F64 && rep.tout == DT_F64 && rep.epi == EPI_STORE)
        return launch_fft_t<double, double, EPI_STORE, true>(rep, d_work, nwork, blocks, nmax, s);
    if (rep.tin == DT_F32 && rep.tout == DT_F64 && rep.epi == EPI_STORE)
        return launch_fft_t<float, double, EPI_STORE, true>(rep, d_work, nwork, blocks, nmax, s);
    if (rep.tin == DT_F32 && rep.tout == DT_F64 && rep.epi == EPI_ACCUM_F64)
        return launch_fft_t<float, double, EPI_ACCUM_F64, true>(rep, d_work, nwork, blocks, nmax, s);
    if (rep.tin == DT_F32 && rep.tout == DT_F32 && rep.epi == EPI_STORE)
        return launch_fft_t<float, float, EPI_STORE, true>(rep, d_work, nwork, blocks, nmax, s);
    return hipErrorInvalidValue;
}

}  // namespace tpt
