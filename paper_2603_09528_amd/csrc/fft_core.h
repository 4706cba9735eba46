// Complex FFT core of the fast transforms, shared by the line kernels and
// the fused transform + GEMM kernels: radix-2 decimation in time grouped
// into register passes of up to four stages over LDS (see fft.hip for the
// scheme).  Synchronisation between passes is a policy: a block barrier when
// a block's threads share lines, a wave-level fence when each wave owns its
// lines.
#pragma once
#include "device_common.h"

namespace tpt {
namespace fftc {

struct SyncBlock {
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};
// LDS operations of one wave complete in order; the fences keep the compiler
// from moving LDS accesses across the point.
struct SyncWave {
    static __device__ __forceinline__ void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
};

__device__ __forceinline__ int pad16(int c) { return c + (c >> 4); }
__device__ __forceinline__ int bitrev(int v, int bits) { return bits ? (int)(__brev((unsigned)v) >> (32 - bits)) : 0; }
__host__ __device__ constexpr int brev_c(int v, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
    return r;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// cos and sin of 2 pi e / 16, e = 0 .. 7
__host__ __device__ constexpr double w16c(int e) {
    return e == 0 ? 1.0 : e == 1 ? 0.92387953251128674 : e == 2 ? 0.70710678118654752 : e == 3 ? 0.38268343236508977
         : e == 4 ? 0.0 : e == 5 ? -0.38268343236508977 : e == 6 ? -0.70710678118654752 : -0.92387953251128674;
}
__host__ __device__ constexpr double w16s(int e) {
    return e == 0 ? 0.0 : e == 1 ? 0.38268343236508977 : e == 2 ? 0.70710678118654752 : e == 3 ? 0.92387953251128674
         : e == 4 ? 1.0 : e == 5 ? 0.92387953251128674 : e == 6 ? 0.70710678118654752 : 0.38268343236508977;
}
// a W_16^e (forward, W_16 = e^{-2 pi i/16}) or a conj(W_16^e) (inverse);
// e is a constant after unrolling, so the trivial cases cost nothing
template <bool INV>
__device__ __forceinline__ double2 w16mul(double2 a, int e) {
    if (e == 0) return a;
    if (e == 4) return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
    const double c = w16c(e), s = INV ? w16s(e) : -w16s(e);
    return make_double2(a.x * c - a.y * s, a.x * s + a.y * c);
}

// In-register radix-2 decimation in time over 2^Q points: input in
// bit-reversed order, output natural, unnormalised.
template <int Q, bool INV>
__device__ __forceinline__ void dit_regs(double2* x) {
#pragma unroll
    for (int s = 0; s < Q; ++s) {
        const int half = 1 << s;
#pragma unroll
        for (int b = 0; b < (1 << Q); b += 2 * half) {
#pragma unroll
            for (int p = 0; p < half; ++p) {
                const double2 u = x[b + p], v = w16mul<INV>(x[b + p + half], p << (3 - s));
                x[b + p] = cadd(u, v);
                x[b + p + half] = csub(u, v);
            }
        }
    }
}

// Inverse input fold: Z_n = E_n + i O_n from the half spectrum F (natural
// order, F_M in the imaginary part of slot 0), E_n = (F_n + conj F_{M-n})/2,
// O_n = conj(W^n) (F_n - conj F_{M-n})/2.
__device__ __forceinline__ double2 ut_fold(const double2* a, int n, int M, const double2* W) {
    if (n == 0) {
        const double2 f = a[0];
        return make_double2(0.5 * (f.x + f.y), 0.5 * (f.x - f.y));
    }
    const double2 fm = a[pad16(n)], fc = conj2(a[pad16(M - n)]);
    const double2 E = cscale(cadd(fm, fc), 0.5);
    const double2 O = cmul(conj2(W[n]), cscale(csub(fm, fc), 0.5));
    return make_double2(E.x - O.y, E.y + O.x);
}

// First pass: Q0 stages, 2^(Q-Q0) groups per thread.  Group g reads the
// natural-order points g + j M/2^Q0 and, after a synchronisation (the writes
// land where other groups read), writes its outputs to base + j, base =
// bitrev(g) 2^Q0.
template <int Q, int Q0, bool INV, class SY>
__device__ __forceinline__ void ut_pass0(double2* a, int t, int T, int mlog, const double2* W) {
    constexpr int R0 = 1 << (Q - Q0), P0 = 1 << Q0;
    const int M = 1 << mlog, G0 = M >> Q0;
    double2 x[1 << Q];
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        const int g = t + r * T;
#pragma unroll
        for (int j = 0; j < P0; ++j) {
            const int n = g + j * G0;
            x[r * P0 + brev_c(j, Q0)] = INV ? ut_fold(a, n, M, W) : a[pad16(n)];
        }
    }
    SY::sync();
#pragma unroll
    for (int r = 0; r < R0; ++r) {
        dit_regs<Q0, INV>(x + r * P0);
        const int base = bitrev(t + r * T, mlog - Q0) << Q0;
#pragma unroll
        for (int j = 0; j < P0; ++j) a[pad16(base + j)] = x[r * P0 + j];
    }
    SY::sync();
}

// Later passes (Q stages from span 2^h): one group per thread, read and
// written in place.
template <int Q, bool INV, class SY>
__device__ __forceinline__ void ut_passk(double2* a, int t, int mlog, int h, const double2* W) {
    constexpr int P = 1 << Q;
    const int blo = t & ((1 << h) - 1);
    const int base = blo | ((t >> h) << (h + Q));
    const int idx1 = blo << (mlog + 1 - h - Q);  // W_{2^(h+Q)}^blo = W_N^idx1
    double2 tw[P];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double2 w = W[idx1 << i];  // idx1 << (Q-1) < M
        tw[1 << i] = INV ? conj2(w) : w;
    }
#pragma unroll
    for (int k = 3; k < P; ++k)
        if (k & (k - 1)) {
            const int hb = 1 << (31 - __builtin_clz(k));
            tw[k] = cmul(tw[hb], tw[k - hb]);
        }
    double2 x[P];
#pragma unroll
    for (int k = 0; k < P; ++k) x[k] = a[pad16(base + (k << h))];
#pragma unroll
    for (int k = 1; k < P; ++k) x[k] = cmul(x[k], tw[brev_c(k, Q)]);
    dit_regs<Q, INV>(x);
#pragma unroll
    for (int j = 0; j < P; ++j) a[pad16(base + (j << h))] = x[j];
    SY::sync();
}

// Complex FFT of one line of M = 2^mlog points at a (padded positions),
// natural order in and out, by the threads t = 0 .. M/2^QM - 1 of the line
// (one thread for M <= 2^QM), each holding up to 2^QM points per pass.  Every
// thread of the synchronisation group SY takes part (the passes hold its
// barriers); INV folds the half spectrum on the first read and uses
// conjugate twiddles.
template <int QM, bool INV, class SY>
__device__ __forceinline__ void ut_cfft_line(double2* a, int t, int mlog, const double2* W) {
    const int Q = mlog < QM ? mlog : QM;
    const int T = 1 << (mlog - Q);
    const int npass = (mlog + Q - 1) / Q, q0 = mlog - (npass - 1) * Q;
    if (Q < QM) {  // short lines: one pass of mlog = Q stages
        if (Q == 2) ut_pass0<2, 2, INV, SY>(a, t, T, mlog, W);
        else if constexpr (QM > 3) ut_pass0<3, 3, INV, SY>(a, t, T, mlog, W);
    } else if (q0 == 1) ut_pass0<QM, 1, INV, SY>(a, t, T, mlog, W);
    else if constexpr (QM == 2) ut_pass0<QM, 2, INV, SY>(a, t, T, mlog, W);
    else if (q0 == 2) ut_pass0<QM, 2, INV, SY>(a, t, T, mlog, W);
    else if constexpr (QM == 3) ut_pass0<QM, 3, INV, SY>(a, t, T, mlog, W);
    else if (q0 == 3) ut_pass0<QM, 3, INV, SY>(a, t, T, mlog, W);
    else ut_pass0<QM, 4, INV, SY>(a, t, T, mlog, W);
    for (int h = q0; h < mlog; h += QM) ut_passk<QM, INV, SY>(a, t, mlog, h, W);
}

}  // namespace fftc
}  // namespace tpt
