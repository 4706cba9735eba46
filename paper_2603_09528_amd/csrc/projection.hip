// Projection step on the staggered grid (§2.1): the finite-volume divergence
// of a face-located velocity at the cell centres, and the update
// u = u* - G phi of the velocity by the gradient of a cell-centred field on
// the faces.  With phi the solution of L phi = D u* (L the pressure operator
// of Eq. poisson-fd2, whose rows are D G), the updated field has D u = 0 up
// to rounding (§4.1 checks this on a white-noise velocity).
//
// Layout (x fastest): pressure-like fields (Nz, Ny, Nx); u (Nz, Ny, Nux),
// v (Nz, Nvy, Nx), w (Nwz, Ny, Nx) where a direction has N face unknowns if
// periodic (face m between cells m and m+1, the last wrapping to cell 0) or
// N - 1 between walls (interior faces; the wall faces carry no flux).
//
// Both kernels give a thread one (i, j) column and march it up RES_RZ-plane
// chunks of z, carrying the z neighbour in registers; x and y neighbours are
// cache hits of the neighbouring lanes' loads.  Memory-bound: the divergence
// moves 32 B per cell (u, v, w read, div written), the update 56 B (phi
// read, u, v, w read and written).
#include "device_common.h"

#include "internal.h"
#include "projection.h"

namespace tpt {

namespace {

constexpr int PJ_NT = 256;
constexpr int PJ_RZ = 32;

inline long long proj_blocks(const ProjDesc& d) {
    const long long ncb = ((long long)d.nx * d.ny + PJ_NT - 1) / PJ_NT;
    return ncb * ((d.nz + PJ_RZ - 1) / PJ_RZ);
}

__global__ __launch_bounds__(PJ_NT) void divergence_kernel(ProjDesc d) {
    const long long sxy = (long long)d.nx * d.ny;
    const long long ncb = (sxy + PJ_NT - 1) / PJ_NT;
    // neighbouring rows on one XCD (they read each other's y neighbours)
    const long long lb = xcd_block(blockIdx.x, gridDim.x);
    const long long zc = lb / ncb;
    const long long c = (lb - zc * ncb) * PJ_NT + threadIdx.x;
    if (c >= sxy) return;
    const int j = (int)(c / d.nx), i = (int)(c - (long long)j * d.nx);
    const int k0 = (int)zc * PJ_RZ, k1 = min(d.nz, k0 + PJ_RZ);
    // x faces on both sides of cell i: upper face i (absent at a wall for
    // i = nx - 1), lower face i - 1 (wrapped or absent for i = 0)
    const bool xhi = i < d.nux;
    const int ilo = i > 0 ? i - 1 : (d.perx ? d.nx - 1 : -1);
    const bool yhi = j < d.nvy;
    const int jlo = j > 0 ? j - 1 : (d.pery ? d.ny - 1 : -1);
    const double rwx = 1.0 / d.wx[i], rwy = 1.0 / d.wy[j];
    // z faces below k0
    const int klo0 = k0 > 0 ? k0 - 1 : (d.perz ? d.nz - 1 : -1);
    double wlo = klo0 >= 0 ? d.w[(long long)klo0 * sxy + c] : 0.0;
    for (int k = k0; k < k1; ++k) {
        const long long urow = ((long long)k * d.ny + j) * d.nux;
        const double uh = xhi ? d.u[urow + i] : 0.0;
        const double ul = ilo >= 0 ? d.u[urow + ilo] : 0.0;
        const long long vbase = (long long)k * d.nvy * d.nx + i;
        const double vh = yhi ? d.v[vbase + (long long)j * d.nx] : 0.0;
        const double vl = jlo >= 0 ? d.v[vbase + (long long)jlo * d.nx] : 0.0;
        const double wh = k < d.nwz ? d.w[(long long)k * sxy + c] : 0.0;
        d.div[(long long)k * sxy + c] = ((uh - ul) * rwx + (vh - vl) * rwy + (wh - wlo) / d.wz[k]) * d.scale;
        wlo = wh;
    }
}

__global__ __launch_bounds__(PJ_NT) void gradient_update_kernel(ProjDesc d) {
    const long long sxy = (long long)d.nx * d.ny;
    const long long ncb = (sxy + PJ_NT - 1) / PJ_NT;
    // neighbouring rows on one XCD (they read each other's y neighbours)
    const long long lb = xcd_block(blockIdx.x, gridDim.x);
    const long long zc = lb / ncb;
    const long long c = (lb - zc * ncb) * PJ_NT + threadIdx.x;
    if (c >= sxy) return;
    const int j = (int)(c / d.nx), i = (int)(c - (long long)j * d.nx);
    const int k0 = (int)zc * PJ_RZ, k1 = min(d.nz, k0 + PJ_RZ);
    // the face above cell i (and above j, k) joins it to cell i + 1, wrapped
    const bool xf = i < d.nux, yf = j < d.nvy;
    const long long ox = i + 1 < d.nx ? 1 : -(long long)(d.nx - 1);
    const long long oy = j + 1 < d.ny ? (long long)d.nx : -(long long)(d.ny - 1) * d.nx;
    const double rdx = xf ? d.gscale / d.dx[i] : 0.0, rdy = yf ? d.gscale / d.dy[j] : 0.0;
    double pc = d.phi[(long long)k0 * sxy + c];
    // pressure update: phi below plane k (zero below a wall, where the
    // Neumann row has no coupling) and the lower x / y neighbours (wrapped;
    // at a wall their coefficient is zero)
    const bool pup = d.P != nullptr;
    double pm = 0.0;
    if (pup && (k0 > 0 || d.perz)) pm = d.phi[(long long)(k0 > 0 ? k0 - 1 : d.nz - 1) * sxy + c];
    const long long oxm = i > 0 ? -1 : (long long)(d.nx - 1);
    const long long oym = j > 0 ? -(long long)d.nx : (long long)(d.ny - 1) * d.nx;
    for (int k = k0; k < k1; ++k) {
        const long long idx = (long long)k * sxy + c;
        if (xf) {
            const long long o = ((long long)k * d.ny + j) * d.nux + i;
            d.uo[o] = d.u[o] - (d.phi[idx + ox] - pc) * rdx;
        }
        if (yf) {
            const long long o = ((long long)k * d.nvy + j) * d.nx + i;
            d.vo[o] = d.v[o] - (d.phi[idx + oy] - pc) * rdy;
        }
        const int kp = k + 1 < d.nz ? k + 1 : 0;
        const double pn = (k + 1 < d.nz || d.perz) ? d.phi[(long long)kp * sxy + c] : 0.0;
        if (k < d.nwz) d.wo[idx] = d.w[idx] - (pn - pc) * d.gscale / d.dz[k];
        if (pup) {
            double li = 0.0;
            if (d.pimpl[0]) li += d.pcb[0][i] * pc + d.pca[0][i] * (i > 0 || d.perx ? d.phi[idx + oxm] : 0.0)
                                  + d.pcc[0][i] * (i + 1 < d.nx || d.perx ? d.phi[idx + ox] : 0.0);
            if (d.pimpl[1]) li += d.pcb[1][j] * pc + d.pca[1][j] * (j > 0 || d.pery ? d.phi[idx + oym] : 0.0)
                                  + d.pcc[1][j] * (j + 1 < d.ny || d.pery ? d.phi[idx + oy] : 0.0);
            if (d.pimpl[2]) li += d.pcb[2][k] * pc + d.pca[2][k] * pm + d.pcc[2][k] * pn;
            d.P[idx] = d.P[idx] + pc - d.pcn * li;
        }
        pm = pc;
        pc = pn;
    }
}

}  // namespace

// Descriptor of the plan's grid; TPT_OK or an error for a plan that is not
// a cell-centred pressure problem with periodic / Neumann (wall) boundaries.
int proj_desc(const tpt_plan_s* p, ProjDesc& d) {
    if (p->host_only) return fail(TPT_ERR_INVALID, "host-only plan");
    if (p->desc.kind != TPT_POISSON || p->desc.nrhs != 1)
        return fail(TPT_ERR_INVALID, "the projection needs a Poisson plan with nrhs = 1");
    for (int k = 0; k < 3; ++k) {
        if (p->desc.loc[k] != TPT_LOC_CENTER) return fail(TPT_ERR_INVALID, "the pressure is cell-centred");
        const int lo = p->desc.bc[k][0], hi = p->desc.bc[k][1];
        if (lo != hi || (lo != TPT_BC_PERIODIC && lo != TPT_BC_NEUMANN))
            return fail(TPT_ERR_INVALID, "pressure boundaries must be periodic or Neumann (walls)");
    }
    d = ProjDesc{};
    d.nx = p->N[0];
    d.ny = p->N[1];
    d.nz = p->N[2];
    d.perx = p->op[0].periodic ? 1 : 0;
    d.pery = p->op[1].periodic ? 1 : 0;
    d.perz = p->op[2].periodic ? 1 : 0;
    d.nux = d.perx ? d.nx : d.nx - 1;
    d.nvy = d.pery ? d.ny : d.ny - 1;
    d.nwz = d.perz ? d.nz : d.nz - 1;
    d.wx = p->buf.vx;
    d.wy = p->buf.vy;
    d.wz = p->buf.vz;
    d.dx = p->buf.dcx;
    d.dy = p->buf.dcy;
    d.dz = p->buf.dcz;
    d.scale = 1.0;
    d.gscale = 1.0;
    d.P = nullptr;
    return TPT_OK;
}

hipError_t launch_divergence(const ProjDesc& d, hipStream_t s) {
    const long long nb = proj_blocks(d);
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    TPT_KLAUNCH(divergence_kernel, dim3((unsigned)nb), dim3(PJ_NT), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_gradient_update(const ProjDesc& d, hipStream_t s) {
    const long long nb = proj_blocks(d);
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    TPT_KLAUNCH(gradient_update_kernel, dim3((unsigned)nb), dim3(PJ_NT), 0, s, d);
    return hipGetLastError();
}

}  // namespace tpt

using namespace tpt;

extern "C" {

int tpt_divergence(tpt_plan plan, const double* u, const double* v, const double* w, double* div, void* stream) {
    if (!plan || !u || !v || !w || !div) return fail(TPT_ERR_INVALID, "NULL argument");
    ProjDesc d;
    int rc = proj_desc(plan, d);
    if (rc) return rc;
    d.u = u;
    d.v = v;
    d.w = w;
    d.div = div;
    TimedScope ts("divergence", (hipStream_t)stream);
    hipError_t e = launch_divergence(d, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("divergence launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

int tpt_gradient_update(tpt_plan plan, const double* phi, double* u, double* v, double* w, void* stream) {
    if (!plan || !phi || !u || !v || !w) return fail(TPT_ERR_INVALID, "NULL argument");
    ProjDesc d;
    int rc = proj_desc(plan, d);
    if (rc) return rc;
    d.u = u;
    d.v = v;
    d.w = w;
    d.uo = u;
    d.vo = v;
    d.wo = w;
    d.phi = phi;
    TimedScope ts("gradient_update", (hipStream_t)stream);
    hipError_t e = launch_gradient_update(d, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("gradient update launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

int tpt_project_workspace_bytes(tpt_plan plan, size_t* bytes) {
    if (!plan || !bytes) return fail(TPT_ERR_INVALID, "NULL argument");
    *bytes = (((size_t)plan->dof * 8 + 255) & ~(size_t)255) + plan_workspace_bytes(plan);
    return TPT_OK;
}

int tpt_project(tpt_plan plan, double* u, double* v, double* w, double* phi, void* workspace,
                size_t workspace_bytes, void* stream) {
    if (!plan || !u || !v || !w || !phi || !workspace) return fail(TPT_ERR_INVALID, "NULL argument");
    ProjDesc d;
    int rc = proj_desc(plan, d);
    if (rc) return rc;
    size_t need = 0;
    tpt_project_workspace_bytes(plan, &need);
    if (workspace_bytes < need) return fail(TPT_ERR_WORKSPACE, "projection workspace too small: need " + std::to_string(need));
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) TPT_HIP(hipSetDevice(plan->device));
    hipStream_t s = (hipStream_t)stream;
    double* div = (double*)workspace;
    const size_t off = ((size_t)plan->dof * 8 + 255) & ~(size_t)255;
    d.u = u;
    d.v = v;
    d.w = w;
    d.uo = u;
    d.vo = v;
    d.wo = w;
    d.div = div;
    d.phi = phi;
    {
        TimedScope ts("divergence", s);
        hipError_t e = launch_divergence(d, s);
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("divergence launch: ") + hipGetErrorString(e));
    }
    if ((rc = solve_one(plan, div, phi, (char*)workspace + off, workspace_bytes - off, s))) return rc;
    TimedScope ts("gradient_update", s);
    hipError_t e = launch_gradient_update(d, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("gradient update launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

}  // extern "C"
