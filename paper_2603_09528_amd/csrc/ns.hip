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
// and rhs: 56 B per unknown (48 B for k = 1); neighbours are cache hits of
// adjacent lanes and planes.  The pressure update moves 24 B per cell.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "device_common.h"

#include "host_ops.h"
#include "internal.h"

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

struct NsPressDesc {
    int N[3];
    int per[3];
    int impl[3];
    const double* a[3];         // pressure operator's 1-D coefficients
    const double* b[3];
    const double* c[3];
    const double* phi;
    double* P;
    double cn;
};

namespace {

constexpr int NS_NT = 256;

// Advection flux difference of component C across the two faces of its
// control volume normal to direction E (E != C): the mass flux is the
// cell-width weighted mean of component E's face velocities in cells m and
// m + 1 along C; the transported value the mean of the two unknowns of C.
template <int C, int E>
__device__ __forceinline__ double ns_transverse(const NsDesc& d, const int* idx, double q0, double qm, double qp,
                                                double hC) {
    constexpr int F = 3 - C - E;
    const int ext0 = E == 0 ? d.nf[0] : d.N[0];
    const int ext1 = E == 1 ? d.nf[1] : d.N[1];
    const long long s[3] = {1, ext0, (long long)ext0 * ext1};
    const int m = idx[C], j = idx[E];
    const int m1 = m + 1 < d.N[C] ? m + 1 : 0;
    const double w0 = d.w[C][m], w1 = d.w[C][m1];
    const double* Qe = d.q[E];
    const long long base = (long long)idx[F] * s[F];
    const long long o0 = base + (long long)m * s[C], o1 = base + (long long)m1 * s[C];
    double ft = 0.0, fb = 0.0;
    if (j < d.nf[E]) ft = 0.5 * (w0 * Qe[o0 + j * s[E]] + w1 * Qe[o1 + j * s[E]]);
    const int jb = j > 0 ? j - 1 : (d.per[E] ? d.nf[E] - 1 : -1);
    if (jb >= 0) fb = 0.5 * (w0 * Qe[o0 + jb * s[E]] + w1 * Qe[o1 + jb * s[E]]);
    return -(ft * (0.5 * (q0 + qp)) - fb * (0.5 * (q0 + qm))) / (hC * d.w[E][j]);
}

template <int C>
__global__ __launch_bounds__(NS_NT) void ns_explicit_kernel(NsDesc d) {
    int ext[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) ext[e] = e == C ? d.nf[e] : d.N[e];
    const unsigned total = (unsigned)ext[0] * (unsigned)ext[1] * (unsigned)ext[2];
    const unsigned o = (unsigned)xcd_block(blockIdx.x, gridDim.x) * NS_NT + threadIdx.x;
    if (o >= total) return;
    const unsigned row = o / (unsigned)ext[0];
    int idx[3];
    idx[0] = (int)(o - row * (unsigned)ext[0]);
    idx[2] = (int)(row / (unsigned)ext[1]);
    idx[1] = (int)(row - (unsigned)idx[2] * (unsigned)ext[1]);
    const unsigned str[3] = {1u, (unsigned)ext[0], (unsigned)ext[0] * (unsigned)ext[1]};
    const double* Q = d.q[C];
    const double q0 = Q[o];
    double qm[3], qp[3], le = 0.0, li = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int p = idx[e], n = ext[e];
        qm[e] = p > 0 ? Q[o - str[e]] : (d.per[e] ? Q[o + (unsigned)(n - 1) * str[e]] : 0.0);
        qp[e] = p < n - 1 ? Q[o + str[e]] : (d.per[e] ? Q[o - (unsigned)(n - 1) * str[e]] : 0.0);
        const double lap = d.cb[e][p] * q0 + d.ca[e][p] * qm[e] + d.cc[e][p] * qp[e];
        if (d.impl[e]) li += lap;
        else le += lap;
    }
    const int m = idx[C];
    const double hC = d.h[C][m];
    // along C: fluxes through the cell centres on both sides of face m
    const double ul = 0.5 * (qm[C] + q0), uh = 0.5 * (q0 + qp[C]);
    double adv = -(uh * uh - ul * ul) / hC;
    constexpr int E1 = C == 0 ? 1 : 0, E2 = C == 2 ? 1 : 2;
    adv += ns_transverse<C, E1>(d, idx, q0, qm[E1], qp[E1], hC);
    adv += ns_transverse<C, E2>(d, idx, q0, qm[E2], qp[E2], hC);
    // pressure gradient on the face between cells m and m + 1
    const long long sp[3] = {1, d.N[0], (long long)d.N[0] * d.N[1]};
    long long pb = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e)
        if (e != C) pb += (long long)idx[e] * sp[e];
    const int m1 = m + 1 < d.N[C] ? m + 1 : 0;
    const double gp = (d.P[pb + (long long)m1 * sp[C]] - d.P[pb + (long long)m * sp[C]]) / hC;
    const double ek = adv + d.nu * le;
    double r = q0 + d.dt * (d.alpha * ek - d.gamma * gp) + d.cn * li;
    if (d.use_prev) r += d.dt * d.beta * d.e[o];
    d.e[o] = ek;
    d.rhs[o] = r;
}

__global__ __launch_bounds__(NS_NT) void ns_pressure_kernel(NsPressDesc d) {
    const unsigned total = (unsigned)d.N[0] * (unsigned)d.N[1] * (unsigned)d.N[2];
    const unsigned o = (unsigned)xcd_block(blockIdx.x, gridDim.x) * NS_NT + threadIdx.x;
    if (o >= total) return;
    const unsigned row = o / (unsigned)d.N[0];
    int idx[3];
    idx[0] = (int)(o - row * (unsigned)d.N[0]);
    idx[2] = (int)(row / (unsigned)d.N[1]);
    idx[1] = (int)(row - (unsigned)idx[2] * (unsigned)d.N[1]);
    const unsigned str[3] = {1u, (unsigned)d.N[0], (unsigned)d.N[0] * (unsigned)d.N[1]};
    const double f0 = d.phi[o];
    double li = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        if (!d.impl[e]) continue;
        const int p = idx[e], n = d.N[e];
        const double fm = p > 0 ? d.phi[o - str[e]] : (d.per[e] ? d.phi[o + (unsigned)(n - 1) * str[e]] : 0.0);
        const double fp = p < n - 1 ? d.phi[o + str[e]] : (d.per[e] ? d.phi[o - (unsigned)(n - 1) * str[e]] : 0.0);
        li += d.b[e][p] * f0 + d.a[e][p] * fm + d.c[e][p] * fp;
    }
    d.P[o] = d.P[o] + f0 - d.cn * li;
}

inline unsigned ns_blocks(long long n) { return (unsigned)((n + NS_NT - 1) / NS_NT); }

constexpr double kAlpha[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double kBeta[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

hipError_t launch_ns_explicit(int comp, const NsDesc& d, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = ns_blocks(n);
    if (comp == 0) TPT_KLAUNCH(ns_explicit_kernel<0>, dim3(nb), dim3(NS_NT), 0, s, d);
    else if (comp == 1) TPT_KLAUNCH(ns_explicit_kernel<1>, dim3(nb), dim3(NS_NT), 0, s, d);
    else TPT_KLAUNCH(ns_explicit_kernel<2>, dim3(nb), dim3(NS_NT), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_ns_pressure(const NsPressDesc& d, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    TPT_KLAUNCH(ns_pressure_kernel, dim3(ns_blocks(n)), dim3(NS_NT), 0, s, d);
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
        hipError_t e = launch_ns_explicit(c, d, ns->count[c], s);
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
    {
        TimedScope ts("gradient_update", s);
        hipError_t e = launch_gradient_update(pd, s);
        if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("gradient update launch: ") + hipGetErrorString(e));
    }
    // P^{k+1/2} = P^{k-1/2} + Phi - c L_I Phi
    NsPressDesc q{};
    const double* pa[3] = {pp->buf.ax, pp->buf.ay, pp->buf.az};
    const double* pb[3] = {pp->buf.bx, pp->buf.by, pp->buf.bz};
    const double* pc[3] = {pp->buf.cx, pp->buf.cy, pp->buf.cz};
    for (int e = 0; e < 3; ++e) {
        q.N[e] = ns->N[e];
        q.per[e] = ns->per[e];
        q.impl[e] = ns->impl[e];
        q.a[e] = pa[e];
        q.b[e] = pb[e];
        q.c[e] = pc[e];
    }
    q.phi = phi;
    q.P = p;
    q.cn = cn;
    TimedScope ts("ns_pressure_update", s);
    hipError_t e = launch_ns_pressure(q, pp->dof, s);
    if (e != hipSuccess) return fail(TPT_ERR_HIP, std::string("NS pressure launch: ") + hipGetErrorString(e));
    return TPT_OK;
}

}  // extern "C"
