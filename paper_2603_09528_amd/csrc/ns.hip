// One Runge–Kutta substep of the incompressible Navier–Stokes solver on the
// staggered grid (§2.1, Eq. rk3): the explicit terms and the predictor, the
// Helmholtz solve of each velocity component, the pressure Poisson solve,
// the correction of the velocity and the update of the pressure.
//
// Per substep k (alpha_k, beta_k, gamma_k; c = gamma_k nu dt / 2):
//   E^k   = A u^k + nu L_E u^k                         (kept for substep k+1)
//   rhs   = u^k + dt (alpha_k E^k + beta_k E^{k-1} - gamma_k G P) + c L_I u^k
//   (I - c L_I) u* = rhs                               (u* = rhs if L_I = 0)
//   L Phi = D u* / (gamma_k dt),   u^{k+1} = u* - gamma_k dt G Phi
//   P    += Phi - c L_I Phi
// (the right-hand side folds the predictor u** and the -c L_I u^k of the
// Helmholtz equation into one expression).
//
// Advection A u = -div(u (x) u) in the symmetry-preserving finite-volume
// form (the paper states second order and semi-discrete kinetic-energy
// conservation): the control volume of a face unknown is the half cells on
// both sides of the face; through its faces the mass flux is the mean of
// the two normal velocities along the component's own direction and the
// cell-width weighted mean of the two transverse velocities elsewhere (the
// fluxes for which the volume's discrete continuity is the half-sum of its
// two cells'), and the transported velocity is the plain mean of the two
// neighbouring unknowns.  The operator is then skew-symmetric for a
// discretely divergence-free field.
//
// Velocity walls: no penetration (wall faces carry no normal velocity and
// are not stored) and no slip (tangential components vanish on the wall:
// the Dirichlet rows of the 1-D operators, face-located along the
// component's own direction).
//
// Memory-bound kernels.  The explicit kernel of a component reads the
// component, the two transverse components, P and E^{k-1} and writes E^k
// and rhs: 56 B per unknown (48 B for k = 1).  A thread marches one (i, j)
// column through a chunk of z planes with the z neighbours in registers;
// in-plane neighbours are cache hits of the adjacent lanes and rows.  The
// pressure update rides in the gradient update's pass (which reads Phi
// anyway): 16 B per cell more there, P read and written.
#include <algorithm>
#include <cmath>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "device_common.h"

#include "host_ops.h"
#include "internal.h"
#include "projection.h"

namespace tpt {

struct NsDesc {
    int N[3];                   // cells per direction
    int nf[3];                  // face unknowns per direction (N periodic, N - 1 walls)
    int per[3];
    int impl[3];                // direction in L_I
    const double* w[3];         // cell widths
    const double* h[3];         // face spacings: distance of the centres of cells m, m+1
    const double* ca[3];        // 1-D operator of this component, per direction
    const double* cb[3];
    const double* cc[3];
    const double* q[3];         // u, v, w (u^k)
    const double* P;            // P^{k-1/2}
    double* e;                  // E^{k-1} in (if use_prev), E^k out
    double* rhs;                // Helmholtz right-hand side (u* for L_I = 0)
    double dt, nu, alpha, beta, gamma, cn;
    int use_prev;
};

namespace {

constexpr int NS_NT = 256;
constexpr int NS_RZ = 32;   // z planes one thread marches through

// Column blocks of a plane of ncol columns times chunks of NS_RZ planes.
inline long long ns_blocks(long long ncol, int nplanes) {
    return ((ncol + NS_NT - 1) / NS_NT) * ((nplanes + NS_RZ - 1) / NS_RZ);
}

// Offsets of the two neighbours along an in-plane direction (wrapped if
// periodic); hm / hp are false where the neighbour is a wall.
struct Nb {
    long long m, p;
    bool hm, hp;
};
__device__ __forceinline__ Nb ns_nb(int pos, int n, long long stride, int periodic) {
    Nb b;
    b.hm = pos > 0 || periodic;
    b.hp = pos < n - 1 || periodic;
    b.m = pos > 0 ? -stride : (long long)(n - 1) * stride;
    b.p = pos < n - 1 ? stride : -(long long)(n - 1) * stride;
    return b;
}

// Explicit terms and right-hand side of u (C = 0) or v (C = 1).  A thread
// owns one (i, j) column of the component and marches it up NS_RZ planes,
// carrying the z neighbours of the component and the z-face mass flux below
// the current plane in registers; in-plane neighbours are cache hits of the
// adjacent lanes and rows (neighbouring rows run on one XCD).
template <int C>
__global__ __launch_bounds__(NS_NT) void ns_explicit_xy_kernel(NsDesc d) {
    constexpr int T = 1 - C;                        // the other in-plane direction
    const int ext[2] = {C == 0 ? d.nf[0] : d.N[0], C == 1 ? d.nf[1] : d.N[1]};
    const int nz = d.N[2];
    const long long sxy = (long long)ext[0] * ext[1];
    const long long ncb = (sxy + NS_NT - 1) / NS_NT;
    const long long lb = xcd_block(blockIdx.x, gridDim.x);
    const long long zc = lb / ncb;
    const long long col = (lb - zc * ncb) * NS_NT + threadIdx.x;
    if (col >= sxy) return;
    const int j = (int)(col / ext[0]), i = (int)(col - (long long)j * ext[0]);
    const int idx[2] = {i, j};
    const int k0 = (int)zc * NS_RZ, k1 = min(nz, k0 + NS_RZ);
    const Nb nb[2] = {ns_nb(i, ext[0], 1, d.per[0]), ns_nb(j, ext[1], ext[0], d.per[1])};
    const double ax = d.ca[0][i], bx = d.cb[0][i], cx = d.cc[0][i];
    const double ay = d.ca[1][j], by = d.cb[1][j], cy = d.cc[1][j];
    const int m = idx[C];
    const int m1 = m + 1 < d.N[C] ? m + 1 : 0;
    const double hC = d.h[C][m], w0 = d.w[C][m], w1 = d.w[C][m1];
    const double wT = d.w[T][idx[T]];
    // component T: cells along C, faces along T (plane tx0 x tx1)
    const int tx0 = T == 0 ? d.nf[0] : d.N[0];
    const long long tsxy = (long long)tx0 * (T == 1 ? d.nf[1] : d.N[1]);
    const long long tst[2] = {1, tx0};
    const int jT = idx[T];
    const bool tt = jT < d.nf[T];
    const int jb = jT > 0 ? jT - 1 : (d.per[T] ? d.nf[T] - 1 : -1);
    const long long to0 = (long long)m * tst[C], to1 = (long long)m1 * tst[C];
    const long long tjt = (long long)jT * tst[T], tjb = (long long)(jb > 0 ? jb : 0) * tst[T];
    // w and P: planes of N0 x N1 cells
    const long long psxy = (long long)d.N[0] * d.N[1];
    const long long pst[2] = {1, d.N[0]};
    const long long po0 = (long long)m * pst[C] + (long long)idx[T] * pst[T];
    const long long po1 = (long long)m1 * pst[C] + (long long)idx[T] * pst[T];
    const double* Q = d.q[C];
    const double* Qt = d.q[T];
    const double* Qw = d.q[2];
    double q0 = Q[(long long)k0 * sxy + col];
    double qzm = k0 > 0 ? Q[(long long)(k0 - 1) * sxy + col] : (d.per[2] ? Q[(long long)(nz - 1) * sxy + col] : 0.0);
    const int kb = k0 > 0 ? k0 - 1 : (d.per[2] ? d.nf[2] - 1 : -1);
    double fzb = kb >= 0 ? 0.5 * (w0 * Qw[(long long)kb * psxy + po0] + w1 * Qw[(long long)kb * psxy + po1]) : 0.0;
    for (int k = k0; k < k1; ++k) {
        const long long o = (long long)k * sxy + col;
        const double qzp = k + 1 < nz ? Q[o + sxy] : (d.per[2] ? Q[col] : 0.0);
        const double qxm = nb[0].hm ? Q[o + nb[0].m] : 0.0, qxp = nb[0].hp ? Q[o + nb[0].p] : 0.0;
        const double qym = nb[1].hm ? Q[o + nb[1].m] : 0.0, qyp = nb[1].hp ? Q[o + nb[1].p] : 0.0;
        const double lx = bx * q0 + ax * qxm + cx * qxp;
        const double ly = by * q0 + ay * qym + cy * qyp;
        const double lz = d.cb[2][k] * q0 + d.ca[2][k] * qzm + d.cc[2][k] * qzp;
        const double li = (d.impl[0] ? lx : 0.0) + (d.impl[1] ? ly : 0.0) + (d.impl[2] ? lz : 0.0);
        const double le = (d.impl[0] ? 0.0 : lx) + (d.impl[1] ? 0.0 : ly) + (d.impl[2] ? 0.0 : lz);
        const double qcm = C == 0 ? qxm : qym, qcp = C == 0 ? qxp : qyp;
        const double qtm = C == 0 ? qym : qxm, qtp = C == 0 ? qyp : qxp;
        // along C: fluxes through the cell centres on both sides of face m
        const double ul = 0.5 * (qcm + q0), uh = 0.5 * (q0 + qcp);
        double adv = -(uh * uh - ul * ul) / hC;
        // across T: component T's face velocities, width-weighted over cells m, m1
        const long long tk = (long long)k * tsxy;
        const double ft = tt ? 0.5 * (w0 * Qt[tk + to0 + tjt] + w1 * Qt[tk + to1 + tjt]) : 0.0;
        const double fb = jb >= 0 ? 0.5 * (w0 * Qt[tk + to0 + tjb] + w1 * Qt[tk + to1 + tjb]) : 0.0;
        adv -= (ft * (0.5 * (q0 + qtp)) - fb * (0.5 * (q0 + qtm))) / (hC * wT);
        // across z: w on the face above plane k (the one below is carried)
        const long long pk = (long long)k * psxy;
        const double fzt = k < d.nf[2] ? 0.5 * (w0 * Qw[pk + po0] + w1 * Qw[pk + po1]) : 0.0;
        adv -= (fzt * (0.5 * (q0 + qzp)) - fzb * (0.5 * (q0 + qzm))) / (hC * d.w[2][k]);
        const double gp = (d.P[pk + po1] - d.P[pk + po0]) / hC;
        const double ek = adv + d.nu * le;
        double r = q0 + d.dt * (d.alpha * ek - d.gamma * gp) + d.cn * li;
        if (d.use_prev) r += d.dt * d.beta * d.e[o];
        d.e[o] = ek;
        d.rhs[o] = r;
        fzb = fzt;
        qzm = q0;
        q0 = qzp;
    }
}

// Explicit terms and right-hand side of w (faces along z): a thread owns an
// (i, j) column of cells and marches the z faces; the transverse velocities
// and the pressure of the cell above face k are carried to face k + 1.
__global__ __launch_bounds__(NS_NT) void ns_explicit_z_kernel(NsDesc d) {
    const int nx = d.N[0], ny = d.N[1], nz = d.N[2], nzf = d.nf[2];
    const long long sxy = (long long)nx * ny;
    const long long ncb = (sxy + NS_NT - 1) / NS_NT;
    const long long lb = xcd_block(blockIdx.x, gridDim.x);
    const long long zc = lb / ncb;
    const long long col = (lb - zc * ncb) * NS_NT + threadIdx.x;
    if (col >= sxy) return;
    const int j = (int)(col / nx), i = (int)(col - (long long)j * nx);
    const int k0 = (int)zc * NS_RZ, k1 = min(nzf, k0 + NS_RZ);
    const Nb nbx = ns_nb(i, nx, 1, d.per[0]), nby = ns_nb(j, ny, nx, d.per[1]);
    const double ax = d.ca[0][i], bx = d.cb[0][i], cx = d.cc[0][i];
    const double ay = d.ca[1][j], by = d.cb[1][j], cy = d.cc[1][j];
    const double wx = d.w[0][i], wy = d.w[1][j];
    // u: planes of nf0 x ny, x faces i (above) and i - 1 (below)
    const long long usxy = (long long)d.nf[0] * ny;
    const bool ut = i < d.nf[0];
    const int ib = i > 0 ? i - 1 : (d.per[0] ? d.nf[0] - 1 : -1);
    const long long uot = (long long)j * d.nf[0] + i, uob = (long long)j * d.nf[0] + (ib > 0 ? ib : 0);
    // v: planes of nx x nf1, y faces j and j - 1
    const long long vsxy = (long long)nx * d.nf[1];
    const bool vt = j < d.nf[1];
    const int jbv = j > 0 ? j - 1 : (d.per[1] ? d.nf[1] - 1 : -1);
    const long long vot = (long long)j * nx + i, vob = (long long)(jbv > 0 ? jbv : 0) * nx + i;
    const double* Q = d.q[2];
    const double* U = d.q[0];
    const double* V = d.q[1];
    auto cell = [&](int m, double& ut_, double& ub_, double& vt_, double& vb_, double& p_) {
        ut_ = ut ? U[(long long)m * usxy + uot] : 0.0;
        ub_ = ib >= 0 ? U[(long long)m * usxy + uob] : 0.0;
        vt_ = vt ? V[(long long)m * vsxy + vot] : 0.0;
        vb_ = jbv >= 0 ? V[(long long)m * vsxy + vob] : 0.0;
        p_ = d.P[(long long)m * sxy + col];
    };
    double ut0, ub0, vt0, vb0, p0;
    cell(k0, ut0, ub0, vt0, vb0, p0);
    double q0 = Q[(long long)k0 * sxy + col];
    double qzm = k0 > 0 ? Q[(long long)(k0 - 1) * sxy + col] : (d.per[2] ? Q[(long long)(nzf - 1) * sxy + col] : 0.0);
    for (int k = k0; k < k1; ++k) {
        const long long o = (long long)k * sxy + col;
        const int m1 = k + 1 < nz ? k + 1 : 0;
        double ut1, ub1, vt1, vb1, p1;
        cell(m1, ut1, ub1, vt1, vb1, p1);
        const double qzp = k + 1 < nzf ? Q[o + sxy] : (d.per[2] ? Q[col] : 0.0);
        const double qxm = nbx.hm ? Q[o + nbx.m] : 0.0, qxp = nbx.hp ? Q[o + nbx.p] : 0.0;
        const double qym = nby.hm ? Q[o + nby.m] : 0.0, qyp = nby.hp ? Q[o + nby.p] : 0.0;
        const double lx = bx * q0 + ax * qxm + cx * qxp;
        const double ly = by * q0 + ay * qym + cy * qyp;
        const double lz = d.cb[2][k] * q0 + d.ca[2][k] * qzm + d.cc[2][k] * qzp;
        const double li = (d.impl[0] ? lx : 0.0) + (d.impl[1] ? ly : 0.0) + (d.impl[2] ? lz : 0.0);
        const double le = (d.impl[0] ? 0.0 : lx) + (d.impl[1] ? 0.0 : ly) + (d.impl[2] ? 0.0 : lz);
        const double hz = d.h[2][k], w0 = d.w[2][k], w1 = d.w[2][m1];
        const double ul = 0.5 * (qzm + q0), uh = 0.5 * (q0 + qzp);
        double adv = -(uh * uh - ul * ul) / hz;
        const double fxt = 0.5 * (w0 * ut0 + w1 * ut1), fxb = 0.5 * (w0 * ub0 + w1 * ub1);
        adv -= (fxt * (0.5 * (q0 + qxp)) - fxb * (0.5 * (q0 + qxm))) / (hz * wx);
        const double fyt = 0.5 * (w0 * vt0 + w1 * vt1), fyb = 0.5 * (w0 * vb0 + w1 * vb1);
        adv -= (fyt * (0.5 * (q0 + qyp)) - fyb * (0.5 * (q0 + qym))) / (hz * wy);
        const double gp = (p1 - p0) / hz;
        const double ek = adv + d.nu * le;
        double r = q0 + d.dt * (d.alpha * ek - d.gamma * gp) + d.cn * li;
        if (d.use_prev) r += d.dt * d.beta * d.e[o];
        d.e[o] = ek;
        d.rhs[o] = r;
        ut0 = ut1; ub0 = ub1; vt0 = vt1; vb0 = vb1; p0 = p1;
        qzm = q0;
        q0 = qzp;
    }
}

constexpr double kAlpha[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double kBeta[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

hipError_t launch_ns_explicit(int comp, const NsDesc& d, hipStream_t s) {
    const long long ncol = comp == 0 ? (long long)d.nf[0] * d.N[1]
                         : comp == 1 ? (long long)d.N[0] * d.nf[1] : (long long)d.N[0] * d.N[1];
    const int planes = comp == 2 ? d.nf[2] : d.N[2];
    const long long nb = ns_blocks(ncol, planes);
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (comp == 0) TPT_KLAUNCH(ns_explicit_xy_kernel<0>, dim3((unsigned)nb), dim3(NS_NT), 0, s, d);
    else if (comp == 1) TPT_KLAUNCH(ns_explicit_xy_kernel<1>, dim3((unsigned)nb), dim3(NS_NT), 0, s, d);
    else TPT_KLAUNCH(ns_explicit_z_kernel, dim3((unsigned)nb), dim3(NS_NT), 0, s, d);
    return hipGetLastError();
}

}  // namespace tpt

using namespace tpt;

struct tpt_ns_s {
    tpt_plan pressure = nullptr;
    double nu = 0.0, dt = 0.0;
    int implicit = TPT_IMPLICIT_NONE;
    int impl[3] = {0, 0, 0};
    int device = 0;
    int N[3] = {0, 0, 0}, nf[3] = {0, 0, 0}, per[3] = {0, 0, 0};
    long long count[3] = {0, 0, 0};    // unknowns of u, v, w
    tpt_plan helm[3][3] = {};          // [substep][component], implicit diffusion only
    double* coef = nullptr;            // a, b, c of each component's 1-D operators
    const double* ca[3][3] = {};       // [component][direction]
    const double* cb[3][3] = {};
    const double* cc[3][3] = {};
    ~tpt_ns_s() {
        for (auto& row : helm)
            for (auto& p : row)
                if (p) tpt_plan_destroy(p);
        if (coef) (void)hipFree(coef);
    }
};

namespace {

size_t ns_solve_ws(const tpt_ns_s* ns) {
    size_t b = plan_workspace_bytes(ns->pressure);
    for (auto& row : ns->helm)
        for (auto* p : row)
            if (p) b = std::max(b, plan_workspace_bytes(p));
    return b;
}

size_t ns_ws_bytes(const tpt_ns_s* ns) {
    size_t b = 0;
    for (int c = 0; c < 3; ++c) b += align256((size_t)ns->count[c] * 8);
    return b + align256((size_t)ns->pressure->dof * 8) + ns_solve_ws(ns);
}

}  // namespace

extern "C" {

int tpt_ns_create(tpt_plan pressure, double nu, double dt, int implicit, tpt_ns* out) {
    if (!pressure || !out) return fail(TPT_ERR_INVALID, "NULL argument");
    *out = nullptr;
    ProjDesc pd;
    int rc = proj_desc(pressure, pd);
    if (rc) return rc;
    if (!(std::isfinite(nu) && nu >= 0.0)) return fail(TPT_ERR_INVALID, "nu must be finite and >= 0");
    if (!(std::isfinite(dt) && dt > 0.0)) return fail(TPT_ERR_INVALID, "dt must be finite and > 0");
    if (implicit < TPT_IMPLICIT_XYZ || implicit > TPT_IMPLICIT_NONE)
        return fail(TPT_ERR_INVALID, "unknown implicit directions");
    if (implicit != TPT_IMPLICIT_NONE && !(nu > 0.0))
        return fail(TPT_ERR_INVALID, "implicit diffusion needs nu > 0");
    std::unique_ptr<tpt_ns_s> ns(new (std::nothrow) tpt_ns_s);
    if (!ns) return fail(TPT_ERR_OOM, "host allocation");
    ns->pressure = pressure;
    ns->nu = nu;
    ns->dt = dt;
    ns->implicit = implicit;
    ns->device = pressure->device;
    ns->impl[2] = implicit != TPT_IMPLICIT_NONE;
    ns->impl[1] = implicit == TPT_IMPLICIT_YZ || implicit == TPT_IMPLICIT_XYZ;
    ns->impl[0] = implicit == TPT_IMPLICIT_XYZ;
    for (int d = 0; d < 3; ++d) {
        ns->N[d] = pressure->N[d];
        ns->per[d] = pressure->op[d].periodic ? 1 : 0;
        ns->nf[d] = ns->per[d] ? ns->N[d] : ns->N[d] - 1;
    }
    for (int c = 0; c < 3; ++c) {
        long long n = 1;
        for (int d = 0; d < 3; ++d) n *= d == c ? ns->nf[d] : ns->N[d];
        ns->count[c] = n;
        if (n >= (1LL << 31)) return fail(TPT_ERR_UNSUPPORTED, "velocity component of 2^31 or more unknowns");
    }
    if (pressure->dof >= (1LL << 31)) return fail(TPT_ERR_UNSUPPORTED, "pressure grid of 2^31 or more cells");
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != ns->device) TPT_HIP(hipSetDevice(ns->device));
    // 1-D operators of the velocity components: face-located along their own
    // direction, Dirichlet (no slip / no penetration) at walls
    Op1D ops[3][3];
    size_t total = 0;
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
            const int bc = ns->per[d] ? BC_P : BC_D;
            std::string err = build_op1d(ns->N[d], pressure->faces[d].data(), bc, bc, d == c ? LOC_F : LOC_C,
                                         ops[c][d]);
            if (!err.empty()) return fail(TPT_ERR_INVALID, "velocity operator: " + err);
            total += 3 * (size_t)ops[c][d].n;
        }
    std::vector<double> h(total);
    size_t off = 0;
    size_t offs[3][3];
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
            const Op1D& op = ops[c][d];
            offs[c][d] = off;
            std::copy(op.a.begin(), op.a.end(), h.begin() + off);
            std::copy(op.b.begin(), op.b.end(), h.begin() + off + op.n);
            std::copy(op.c.begin(), op.c.end(), h.begin() + off + 2 * op.n);
            off += 3 * (size_t)op.n;
        }
    if (hipMalloc(&ns->coef, total * sizeof(double)) != hipSuccess) {
        ns->coef = nullptr;
        return fail(TPT_ERR_OOM, "NS coefficients");
    }
    TPT_HIP(hipMemcpy(ns->coef, h.data(), total * sizeof(double), hipMemcpyHostToDevice));
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
            const int n = ops[c][d].n;
            ns->ca[c][d] = ns->coef + offs[c][d];
            ns->cb[c][d] = ns->coef + offs[c][d] + n;
            ns->cc[c][d] = ns->coef + offs[c][d] + 2 * n;
        }
    // the Helmholtz problems of the velocity components, one per substep
    // coefficient gamma_k nu dt / 2 (eigenbases shared through the cache)
    if (implicit != TPT_IMPLICIT_NONE) {
        for (int k = 0; k < 3; ++k)
            for (int c = 0; c < 3; ++c) {
                tpt_plan_desc hd;
                tpt_plan_desc_init(&hd);
                for (int d = 0; d < 3; ++d) {
                    hd.n[d] = ns->N[d];
                    hd.faces[d] = pressure->faces[d].data();
                    const int bc = ns->per[d] ? TPT_BC_PERIODIC : TPT_BC_DIRICHLET;
                    hd.bc[d][0] = hd.bc[d][1] = bc;
                    hd.loc[d] = d == c ? TPT_LOC_FACE : TPT_LOC_CENTER;
                }
                hd.kind = TPT_HELMHOLTZ;
                hd.alpha = (kAlpha[k] + kBeta[k]) * nu * dt / 2.0;
                hd.precision = TPT_FP64;
                hd.nrhs = 1;
                hd.flags = TPT_FLAG_NO_CHECK;
                hd.implicit = implicit;
                if ((rc = tpt_plan_create(&hd, &ns->helm[k][c]))) return rc;
            }
    }
    *out = ns.release();
    return TPT_OK;
}

int tpt_ns_destroy(tpt_ns ns) {
    delete ns;
    return TPT_OK;
}

int tpt_ns_workspace_bytes(tpt_ns ns, size_t* bytes) {
    if (!ns || !bytes) return fail(TPT_ERR_INVALID, "NULL argument");
    *bytes = ns_ws_bytes(ns);
    return TPT_OK;
}

int tpt_ns_substep(tpt_ns ns, int k, double* u, double* v, double* w, double* eu, double* ev, double* ew,
                   double* p, double* phi, void* workspace, size_t workspace_bytes, void* stream) {
    if (!ns || !u || !v || !w || !eu || !ev || !ew || !p || !phi || !workspace)
        return fail(TPT_ERR_INVALID, "NULL argument");
    if (k < 1 || k > 3) return fail(TPT_ERR_INVALID, "substep k must be 1, 2 or 3");
    const size_t need = ns_ws_bytes(ns);
    if (workspace_bytes < need) return fail(TPT_ERR_WORKSPACE, "NS workspace too small: need " + std::to_string(need));
    int cur = 0;
    if (hipGetDevice(&cur) == hipSuccess && cur != ns->device) TPT_HIP(hipSetDevice(ns->device));
    hipStream_t s = (hipStream_t)stream;
    const double alpha = kAlpha[k - 1], beta = kBeta[k - 1], gamma = alpha + beta;
    const double cn = ns->implicit == TPT_IMPLICIT_NONE ? 0.0 : gamma * ns->nu * ns->dt / 2.0;
    double* vel[3] = {u, v, w};
    double* ex[3] = {eu, ev, ew};
    char* base = (char*)workspace;
    double* rhs[3];
    for (int c = 0; c < 3; ++c) {
        rhs[c] = (double*)base;
        base += align256((size_t)ns->count[c] * 8);
    }
    double* div = (double*)base;
    base += align256((size_t)ns->pressure->dof * 8);
    void* sws = base;
    const size_t sws_bytes = workspace_bytes - (size_t)(base - (char*)workspace);
    // explicit terms and the right-hand sides of the three components (all
    // read u^k, so the velocity is overwritten only after the last one)
    const tpt_plan_s* pp = ns->pressure;
    static const char* names[3] = {"ns_explicit_u", "ns_explicit_v", "ns_explicit_w"};
    for (int c = 0; c < 3; ++c) {
        NsDesc d{};
        for (int e = 0; e < 3; ++e) {
            d.N[e] = ns->N[e];
            d.nf[e] = ns->nf[e];
            d.per[e] = ns->per[e];
            d.impl[e] = ns->impl[e];
            d.ca[e] = ns->ca[c][e];
            d.cb[e] = ns->cb[c][e];
            d.cc[e] = ns->cc[c][e];
            d.q[e] = vel[e];
        }
        d.w[0] = pp->buf.vx; d.w[1] = pp->buf.vy; d.w[2] = pp->buf.vz;
        d.h[0] = pp->buf.dcx; d.h[1] = pp->buf.dcy; d.h[2] = pp->buf.dcz;
        d.P = p;
        d.e = ex[c];
        d.rhs = rhs[c];
        d.dt = ns->dt;
        d.nu = ns->nu;
        d.alpha = alpha;
        d.beta = beta;
        d.gamma = gamma;
        d.cn = cn;
        d.use_prev = k > 1 ? 1 : 0;
        TimedScope ts(names[c], s);
        hipError_t e = launch_ns_explicit(c, d, s);
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("NS explicit launch: ") + hipGetErrorString(e));
    }
    // implicit diffusion: (I - c L_I) u* = rhs, u* into the velocity arrays
    double* ustar[3] = {rhs[0], rhs[1], rhs[2]};
    int rc;
    if (ns->implicit != TPT_IMPLICIT_NONE) {
        for (int c = 0; c < 3; ++c)
            if ((rc = solve_one(ns->helm[k - 1][c], rhs[c], vel[c], sws, sws_bytes, s))) return rc;
        for (int c = 0; c < 3; ++c) ustar[c] = vel[c];
    }
    // projection: L Phi = D u* / (gamma dt), u = u* - gamma dt G Phi
    ProjDesc pd;
    if ((rc = proj_desc(pp, pd))) return rc;
    pd.u = ustar[0];
    pd.v = ustar[1];
    pd.w = ustar[2];
    pd.uo = u;
    pd.vo = v;
    pd.wo = w;
    pd.div = div;
    pd.phi = phi;
    pd.scale = 1.0 / (gamma * ns->dt);
    pd.gscale = gamma * ns->dt;
    {
        TimedScope ts("divergence", s);
        hipError_t e = launch_divergence(pd, s);
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("divergence launch: ") + hipGetErrorString(e));
    }
    if ((rc = solve_one(ns->pressure, div, phi, sws, sws_bytes, s))) return rc;
    // u = u* - gamma dt G Phi and, in the same pass,
    // P^{k+1/2} = P^{k-1/2} + Phi - c L_I Phi
    pd.P = p;
    pd.pcn = cn;
    const double* pa[3] = {pp->buf.ax, pp->buf.ay, pp->buf.az};
    const double* pb[3] = {pp->buf.bx, pp->buf.by, pp->buf.bz};
    const double* pc[3] = {pp->buf.cx, pp->buf.cy, pp->buf.cz};
    for (int e = 0; e < 3; ++e) {
        pd.pimpl[e] = ns->impl[e];
        pd.pca[e] = pa[e];
        pd.pcb[e] = pb[e];
        pd.pcc[e] = pc[e];
    }
    TimedScope ts("gradient_update", s);
    hipError_t e = launch_gradient_update(pd, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("gradient update launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

}  // extern "C"
