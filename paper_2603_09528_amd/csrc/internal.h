// Internal types of the tpt library (plans, eigenbasis cache, workspace
// layout, error reporting, kernel timing).
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tpt.h"
#include "host_ops.h"
#include "kernels.h"

namespace tpt {

// ---- errors ---------------------------------------------------------------
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
const char* last_error_cstr();
#define TPT_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::tpt::fail(TPT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---- device eigenbasis of one direction (shared through the cache) --------
// Orientation: Qinv[p][i] = Q~[i][p] s_i (forward, Q^{-1} = Q~^T D^{1/2}) and
// Q[i][p] = Q~[i][p] / s_i (inverse, Q = D^{-1/2} Q~), both row-major
// [out][in] (Eq. q-from-tildeq).
struct DirBasis {
    int device = 0;
    int n = 0;
    Eig1D eig;                       // host eigen data
    double* d_lam = nullptr;         // device eigenvalues
    double* d_qinv = nullptr;        // FP64
    double* d_q = nullptr;
    float* s_qinv = nullptr;         // FP32 copies
    float* s_q = nullptr;
    uint16_t* h_qinv = nullptr;      // bf16 hi / lo planes, rows of ldp elements
    uint16_t* l_qinv = nullptr;      // (n rounded up to 8: 16-byte rows, zero padded)
    uint16_t* h_q = nullptr;
    uint16_t* l_q = nullptr;
    int ldp = 0;
    int fast_kind = -1;              // XformKind of the fast transform, -1 = none
    double2* d_twiddle = nullptr;    // e^{-2 pi i k/n}, k < n/2 (fast transform)
    double2* d_qtw = nullptr;        // e^{-i pi k/2n}, k <= n/2 (DCT, DST)
    double h = 0.0;                  // uniform spacing (analytic bases)
    void* block = nullptr;           // single allocation holding all of the above
    size_t bytes = 0;
    ~DirBasis();
};

// Device-resident cache of eigenbases keyed by (device, faces, BC, location).
std::shared_ptr<DirBasis> basis_cache_get(int ncells, const double* faces, int bc_lo, int bc_hi, int loc,
                                          bool host_only, std::string& err);
size_t basis_cache_bytes();   // device bytes held by live cached bases

// ---- plans ------------------------------------------------------------------
struct PlanBuffers {  // per-plan small device arrays
    double* ax = nullptr; double* bx = nullptr; double* cx = nullptr;
    double* ay = nullptr; double* by = nullptr; double* cy = nullptr;
    double* az = nullptr; double* bz = nullptr; double* cz = nullptr;
    double* vx = nullptr; double* vy = nullptr; double* vz = nullptr;  // control volumes
    double* vyz = nullptr;       // vy_j vz_k at j + Ny k
    double* zeros = nullptr;     // max(Nx, Ny) zeros: the shift of an explicit direction
    // distance between the centres of cells m and m+1 (the last one wrapped
    // for a periodic direction), N per direction: the face spacing of the
    // projection's gradient
    double* dcx = nullptr; double* dcy = nullptr; double* dcz = nullptr;
    double* norms = nullptr;     // device sums, TPT_STATS doubles per rhs (StatSlot)
    void* block = nullptr;
};

// Reduced sums of one right-hand side, TPT_STATS doubles: refinement norms
// (||r||^2, ||f||^2 of the last residual; ||e||^2, ||x||^2 of the last
// correction and iterate) and the right-hand-side check (sum dV f,
// sum dV |f|, non-finite count).
enum StatSlot { SS_R2 = 0, SS_F2 = 1, SS_E2 = 2, SS_X2 = 3, SS_WF = 4, SS_WABS = 5, SS_BAD = 6 };
constexpr int TPT_STATS = 8;

}  // namespace tpt

struct tpt_plan_s {
    tpt_plan_desc desc{};
    std::vector<double> faces[3];
    tpt::Op1D op[3];
    std::shared_ptr<tpt::DirBasis> bx, by;
    int N[3] = {0, 0, 0};            // unknowns x, y, z
    long long dof = 0;               // per right-hand side
    double sigma = 0.0, tau = 1.0;   // line operator sigma + tau (lambda + T_z)
    int null_line = -1;
    bool host_only = false;
    int device = 0;
    tpt::PlanBuffers buf;
    void* own_ws = nullptr;
    size_t own_ws_bytes = 0;
    double* h_norms = nullptr;       // pinned host copy of norms (adaptive mode)
    tpt_info info{};
    bool info_on_device = false;     // info fields still to be read from buf.norms
    bool check = true;               // right-hand-side check reported in tpt_info
    bool run_check = true;           // check kernel runs (also for mixed singular plans,
                                     // whose residuals use its weighted sum)
    double last_area_inv = 0.0;      // 1 / sum dV over the last z plane
    int gemm_variant[4] = {-1, -1, -1, -1};  // per stage (x fwd, y fwd, y inv, x inv); -1 = table
    int fast[2] = {-1, -1};          // x, y: XformKind of the fast transform, -1 = GEMM
    bool fuse_xy = false;            // FP64: x transform fused into the y GEMM's loads
    bool seq_thomas = false;         // z lines by the sequential Thomas kernel
    bool tx = true, ty = true;       // x / y transformed (implicit in the operator)
    ~tpt_plan_s();
};

namespace tpt {

// Workspace layout of one solve (bytes per unknown * dof * nrhs).
size_t plan_workspace_bytes(const tpt_plan_s* p);

// GEMM descriptors for the four transform stages of a plan.
enum Stage { ST_XF = 0, ST_YF = 1, ST_YI = 2, ST_XI = 3 };
GemmDesc stage_gemm(const tpt_plan_s* p, int stage, int prec, const void* in, int tin, void* out, int tout,
                    int epi, double* partials, int nrhs);
// Stages of a direction with a fast transform: all lines of that direction.
bool stage_is_fast(const tpt_plan_s* p, int stage);
FftDesc stage_fft(const tpt_plan_s* p, int stage, const void* in, int tin, void* out, int tout, int epi,
                  double* partials, int nrhs);
ThomasDesc plan_thomas(const tpt_plan_s* p, const void* f, int tf, void* x, int tx, double* scratch, int nrhs);
// stats: the rhs's TPT_STATS sums (after the right-hand-side check), or NULL
StencilDesc plan_stencil(const tpt_plan_s* p, const double* x, const double* f, float* r, double* partials,
                         const double* stats);
int plan_gemm_prec(const tpt_plan_s* p);

// Tile selection: autotuned table lookup (falls back to a size heuristic).
int choose_variant(int prec, int stage_kind, int M, int N, int K);
void autotune_record(int prec, int stage_kind, int M, int N, int K, int variant);
// tuning-table kind of the Thomas kernel entries: (prec, TUNE_THOMAS, lines,
// nz, 0) -> THOMAS_SEQ or THOMAS_PART + configuration
constexpr int TUNE_THOMAS = 2;
// the recorded Thomas variant for that key, or THOMAS_AUTO
int tuned_thomas(int prec, long long lines, int nz);
// stage_kind: 0 = x pass (B = basis), 1 = y pass (A = basis)

// ---- kernel timing ------------------------------------------------------------
bool timing_enabled();
// Scope around one kernel launch on stream s: when timing is on (and s is
// not capturing a graph) the launch records a pair of events at the kernel's
// own start and end, collected by tpt_timing_collect under `name`.
struct TimedScope {
    TimedScope(const char* name, hipStream_t s);
    ~TimedScope();
    const char* name;
    hipStream_t s;
    hipEvent_t e0 = nullptr;
    hipEvent_t e1 = nullptr;
    bool on = false;
};

int solve_one(tpt_plan_s* p, const double* rhs, double* out, void* ws, size_t ws_bytes, hipStream_t s);
// Right-hand-side check of a solve: its descriptor (stats into the plan's
// buffer), whether it rides in the x forward fast transform's loads (x lines
// by FFT, whole blocks of lines per rhs), the partials per rhs it then
// writes, and the descriptor fields of that transform.
CheckDesc check_desc(const tpt_plan_s* p, const double* rhs, double* partials);
bool check_fused(const tpt_plan_s* p);
long long check_fused_blocks(const tpt_plan_s* p);
void attach_check(const tpt_plan_s* p, const CheckDesc& c, FftDesc& f);
// tpt_info fields of plan p from its reduced per-rhs sums h (TPT_STATS
// doubles per rhs): the refinement norms when `norms`, the check fields when
// the plan checks its right-hand sides; other fields are left as they are.
void stats_to_info(const tpt_plan_s* p, const double* h, bool norms, tpt_info* info);

// Workspace carve-up of one plan's solve (see plan_workspace_bytes).
struct Ws {
    char* base;
    size_t n;  // unknowns over all rhs
    void* w1;
    void* w2;
    float* r;
    double* scratch;
    double* partials;
};
Ws carve(const tpt_plan_s* p, void* ws);
int stage_variant(const tpt_plan_s* p, int stage, const GemmDesc& g, int prec);
const char* stage_name(int stage, int prec);
long long plan_residual_blocks(const tpt_plan_s* p);

}  // namespace tpt
