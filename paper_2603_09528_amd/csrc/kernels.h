// Device kernels of the tensor-product–Thomas solve and their launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace tpt {

// Kernel timing: while a timed scope is open on this thread, the next kernel
// launch records these events at the kernel's own start and end
// (hipExtLaunchKernel), so a timed duration is the kernel's execution time.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
    bool used = false;
};
LaunchEvents& launch_events();  // thread-local

// Element types of GEMM operands/results in global memory.
enum DType { DT_F64 = 0, DT_F32 = 1 };
// MFMA arithmetic of a GEMM.
enum GemmPrec { GP_F64 = 0, GP_F32 = 1, GP_BF16X3 = 2 };
// What the epilogue does with the accumulated tile.
enum Epilogue {
    EPI_STORE = 0,      // C = acc (converted to C's type)
    EPI_ACCUM_F64 = 1   // C (double) += acc; per-block partial sums of acc^2 and C^2
};

// Tile shapes (BM x BN) compiled for every precision; the autotuner picks.
// TV_128x128_K32: 128 x 128 with a deep K tile in a single LDS buffer (32
// deep for FP64 and FP32, 64 deep for BF16X3).
// TV_128x128_P: the 128 x 128 tile in a persistent grid that loads the next
// tile's first K tile during the current one (FP64 / FP32; edge tiles and a
// ragged K through range-limited buffer resources and masks).
// TV_128x128_P8: the same with eight waves of 64 x 32 instead of four of
// 64 x 64 (half the accumulator registers per wave, twice the waves).
// TV_128x128_W8: the plain 128 x 128 tile over eight waves of 64 x 32 (FP64 /
// FP32; any shape).
enum TileVariant {
    TV_128x128 = 0, TV_64x128 = 1, TV_128x64 = 2, TV_64x64 = 3, TV_32x64 = 4, TV_128x128_K32 = 5,
    TV_128x128_P = 6, TV_128x128_P8 = 7, TV_128x128_W8 = 8, TV_COUNT = 9
};
// the persistent tiles (FP64 / FP32)
inline bool tv_persistent(int v) { return v == TV_128x128_P || v == TV_128x128_P8; }
// Grid of the persistent GEMM: two blocks per CU (a multiple of 8, so that a
// block keeps its XCD), at most the tile count.
long long persistent_gemm_grid(long long tiles);
const char* tile_variant_name(int v);
void tile_variant_shape(int v, int* bm, int* bn);

// One strided-batched GEMM C_b = A_b op(B_b), A row-major M x K (lda),
// C row-major M x N (ldc).  b_nk = 0: B stored K x N row-major (ldb);
// b_nk = 1: B stored N x K row-major (ldb), i.e. C = A B^T.
// For GP_BF16X3 the basis operand (A when basis_is_A, else B) is given as
// pre-split bf16 planes basis_hi / basis_lo in the same layout; the other
// operand is split on the fly.
struct GemmDesc {
    const void* A;
    const void* B;
    void* C;
    int M, N, K;
    int lda, ldb, ldc;
    long long sA, sB, sC;   // batch strides in elements (0 = shared)
    int batch;
    int b_nk;
    int tA, tB, tC;         // DType of A, B, C in global memory (basis planes ignore tA/tB)
    const uint16_t* basis_hi;
    const uint16_t* basis_lo;
    int ldp;                // row stride of basis_hi / basis_lo (0: lda or ldb, as the basis operand)
    int basis_is_A;
    int epi;                // Epilogue
    double* partials;       // EPI_ACCUM_F64: 2 doubles per block
    // filled by the launcher / work-list builder
    int tiles_m, tiles_n;
    long long block_begin;
};

long long gemm_blocks(const GemmDesc& g, int variant);
// One launch for one descriptor.
hipError_t launch_gemm(GemmDesc g, int prec, int variant, hipStream_t s);
// One launch over a device array of descriptors (block_begin, tiles_m/n set
// by the caller, sorted by block_begin, all sharing prec, variant, b_nk, the
// operand types and the epilogue of `rep`).
hipError_t launch_gemm_multi(const GemmDesc& rep, const GemmDesc* d_work, int nwork, long long total_blocks,
                             int prec, int variant, hipStream_t s);
// Work-list GEMM (FP64 / FP32, persistent, next tile prefetched): x pass
// (b_nk = 1) in 128 x 64 tiles, y pass (b_nk = 0) in 64 x 128 tiles over
// N' = batch N slab-folded columns.  worklist_tiles gives a descriptor's tile
// count (tiles_m, tiles_n are set by worklist_shape); worklist_ok whether its
// extents fit the kernel's 32-bit offsets.
void worklist_shape(GemmDesc& g);
long long worklist_tiles(const GemmDesc& g);
bool worklist_ok(const GemmDesc& g, int prec);
hipError_t launch_gemm_worklist(const GemmDesc& rep, const GemmDesc* d_work, int nwork, long long tiles, int prec,
                                hipStream_t s);
hipError_t launch_gemm_worklist_f64(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long tiles,
                                    hipStream_t s);
hipError_t launch_gemm_worklist_f32(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long tiles,
                                    hipStream_t s);
// Per-precision launchers (gemm_f64.hip, gemm_f32.hip, gemm_bf16.hip).
hipError_t launch_gemm_f64(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks, int variant,
                           hipStream_t s);
hipError_t launch_gemm_f32(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks, int variant,
                           hipStream_t s);
hipError_t launch_gemm_bf16(const GemmDesc& g, const GemmDesc* d_work, int nwork, long long blocks, int variant,
                            hipStream_t s);

// Fast transforms of the lines of a uniform direction (analytic bases:
// real Fourier for periodic, DCT-II for Neumann-Neumann, DST-II for
// Dirichlet-Dirichlet, cell-centred): forward fhat = sqrt(h) Q~^T f or inverse
// phi = Q~ phihat / sqrt(h) for `lines` lines of length n (a power of two,
// 8..2048), either contiguous (x lines) or strided (y lines: column `col` of
// slab `slab` starts at slab * s_outer + col, element stride s_elem).
enum XformKind { UT_FOURIER = 0, UT_DCT = 1, UT_DST = 2 };
struct FftDesc {
    int n;
    int kind;               // XformKind
    int inverse;
    int ylines;             // 0: line l starts at l * n; 1: strided as above
    long long lines;
    long long inner;        // ylines: lines per slab (Nx)
    long long s_elem;       // ylines: element stride (Nx)
    long long s_outer;      // ylines: slab stride (Nx Ny)
    const void* in;
    void* out;
    int tin, tout;          // DType of in / out
    int epi;                // EPI_STORE, or EPI_ACCUM_F64 (inverse only, FP64 out)
    double scale;           // sqrt(h) forward, 1/sqrt(h) inverse
    const double2* twiddle; // e^{-2 pi i k / n}, k < n/2
    const double2* qtw;     // e^{-i pi k / 2n}, k <= n/2 (DCT, DST)
    double* partials;       // EPI_ACCUM_F64: 2 doubles per block
    long long block_begin;  // multi-problem
    // forward x lines only: the right-hand-side check fused into the loads
    // (cpart non-null): per block the partials of CheckDesc (4 doubles at
    // cpart + 4 blk) over its lines, line = row of rhs
    // line / crows, crows = Ny Nz a multiple of the lines per block; weights
    // vx_i cvyz[row] (cvyz[j + Ny k] = vy_j vz_k)
    const double* cvx;
    const double* cvyz;
    double* cpart;
    unsigned crows;
};
bool fft_supported(int n);
long long fft_blocks(const FftDesc& d);
int fft_lines_per_block(int n);
hipError_t launch_fft(const FftDesc& rep, const FftDesc* d_work, int nwork, long long blocks, hipStream_t s);

// y GEMM of one problem (descriptor of the y pass) whose B rows are first
// transformed along x (descriptor of the x pass: kind, direction, scale,
// tables); FP64, N = n_x = 128 or 256, M a multiple of 128, K of 16.
bool xgemm_supported(const GemmDesc& g, const FftDesc& xf);
hipError_t launch_xgemm(const GemmDesc& g, const FftDesc& xf, hipStream_t s);

// Thomas solve along z (§2.2.2 step 2.3) for nsys systems of nx*ny lines.
struct ThomasDesc {
    int nx, ny, nz, nsys;
    const double* lamx;
    const double* lamy;
    const double* az;
    const double* bz;
    const double* cz;
    double sigma, tau;
    int pin_line;
    int periodic;          // cyclic z lines (corners az[0], cz[nz-1])
    const void* f;
    void* x;
    double* scratch;       // thomas_scratch_doubles() doubles
    int tf, tx;            // DType of f and x
    long long block_begin; // multi-problem: first block of this problem
    int variant;           // THOMAS_AUTO, THOMAS_SEQ or THOMAS_PART + configuration
};
// Thomas kernels: sequential (one lane per line, checkpointed chunks; the
// only one for periodic lines and mixed storage types) or partitioned (P
// segments of L planes per line, one lane per segment, LB lines per block)
// in one of THOMAS_NPART configurations.
enum { THOMAS_AUTO = 0, THOMAS_SEQ = 1, THOMAS_PART = 2, THOMAS_NPART = 17 };
// the variant launch_thomas runs for t (-1: t.variant does not fit t)
int thomas_variant(const ThomasDesc& t);
void thomas_part_shape(int v, int* lb, int* p, int* l);
long long thomas_part_blocks(const ThomasDesc& t, int v);
hipError_t launch_thomas_part(const ThomasDesc& t, int v, hipStream_t s);
// every problem of the list in configuration v with storage type dtype (f
// and x alike); block_begin counts blocks of that configuration's LB lines
hipError_t launch_thomas_part_multi(const ThomasDesc* d_work, int nwork, long long total_blocks, int v, int dtype,
                                    hipStream_t s);
hipError_t launch_thomas(const ThomasDesc& t, hipStream_t s);
long long thomas_blocks(const ThomasDesc& t);
// Scratch the Thomas kernel needs: (c', d') checkpoints, one per line every
// 32 planes, and for cyclic lines also the d' of the second right-hand side.
long long thomas_scratch_doubles(int nx, int ny, int nz, int nsys, int periodic);
// nz_max: the largest nz of the work list (LDS for its coefficients)
hipError_t launch_thomas_multi(const ThomasDesc* d_work, int nwork, long long total_blocks, int nz_max,
                               hipStream_t s);

// Residual r = f - A x of the 7-point operator in FP64, r stored as float,
// with per-block partial sums (r^2, f^2).
struct StencilDesc {
    int nx, ny, nz;
    const double* ax; const double* bx; const double* cx;
    const double* ay; const double* by; const double* cy;
    const double* az; const double* bz; const double* cz;
    int perx, pery, perz;
    int helmholtz;
    double alpha;
    const double* x;
    const double* f;
    float* r;
    double* partials;  // 2 doubles per block (sums of r^2 and f^2), or null
    // singular problems: f on the last z plane is read as f - S * wscale, with
    // S = *wsum = sum dV f (the right-hand-side check) and wscale = 1 / (the
    // area sum dV of that plane), so that sum dV r = 0 (null = no change)
    const double* wsum;
    double wscale;
    long long block_begin;  // multi-problem
    // two columns per thread (set from residual_pairs_ok; 0 gives the
    // larger block count, which sizes the partial sums)
    int pair;
};
bool residual_pairs_ok(const StencilDesc& st);
int residual_blocks(const StencilDesc& st);
hipError_t launch_residual(const StencilDesc& st, hipStream_t s);
hipError_t launch_residual_multi(const StencilDesc* d_work, int nwork, long long total_blocks, hipStream_t s);

// Deterministic sum of n (a, b) pairs into out[0], out[1].
hipError_t launch_reduce_pairs(const double* partials, int n, double* out, hipStream_t s);
struct ReduceDesc {
    const double* partials;
    int n;
    double* out;
};
hipError_t launch_reduce_pairs_multi(const ReduceDesc* d_work, int nwork, hipStream_t s);

// Right-hand-side check of one solve (tpt_info compat_defect and nonfinite):
// per field, the weighted sums S = sum w f and A = sum w |f| over the finite
// values, w = vx_i vy_j vz_k (the control volumes: the left null vector of a
// singular operator), and the count of NaN / Inf values.  Blocks write
// partials (4 doubles each); one block per field then folds them in a fixed
// order into out + sys * out_stride: [S, A, count].
struct CheckDesc {
    int nx, ny, nz;
    int nsys;               // fields back to back at f
    const double* f;
    const double* vx;
    const double* vy;
    const double* vz;
    const double* vyz;      // vy_j vz_k at j + Ny k
    double* partials;       // 4 doubles per block, nsys * check_blocks(c) blocks
    double* out;
    int out_stride;
    long long block_begin;  // multi-problem: first block of this problem
    long long nblk;         // partials per field when written by another kernel
                            // (the fused x-forward check), else 0
};
long long check_blocks(const CheckDesc& c);  // blocks per field
hipError_t launch_check(const CheckDesc& c, hipStream_t s);
// only the folding of partials written elsewhere (nb blocks per field)
hipError_t launch_check_reduce(const CheckDesc& c, long long nb, hipStream_t s);
// the same for a list (one field each, c.nblk partials each)
hipError_t launch_check_reduce_multi(const CheckDesc* d_work, int nwork, hipStream_t s);
// every problem of the list (one field each); then one reduction block each
hipError_t launch_check_multi(const CheckDesc* d_work, int nwork, long long total_blocks, hipStream_t s);

// Split float -> bf16 hi/lo planes (round to nearest even), n elements.
hipError_t launch_split_bf16(const float* x, uint16_t* hi, uint16_t* lo, long long n, hipStream_t s);
hipError_t launch_convert_f64_f32(const double* x, float* y, long long n, hipStream_t s);

}  // namespace tpt
