// Projection step on the staggered grid (§2.1): descriptor and launchers of
// the divergence and gradient-update kernels, shared by the projection and
// the Navier-Stokes substep.
#pragma once
#include "internal.h"

namespace tpt {

// Pressure-like fields (Nz, Ny, Nx); u (Nz, Ny, Nux), v (Nz, Nvy, Nx),
// w (Nwz, Ny, Nx), with N face unknowns in a periodic direction and N - 1
// between walls.
struct ProjDesc {
    int nx, ny, nz;
    int perx, pery, perz;
    int nux, nvy, nwz;               // face unknowns per direction
    const double* wx;                // cell widths (control volumes)
    const double* wy;
    const double* wz;
    const double* dx;                // centre distances of the faces (nux / nvy / nwz)
    const double* dy;
    const double* dz;
    const double* u;
    const double* v;
    const double* w;
    double* uo;
    double* vo;
    double* wo;
    const double* phi;
    double* div;
    double scale;                    // div = scale * D(u, v, w)
    double gscale;                   // uo = u - gscale * G phi
    // optional pressure update in the same pass (Navier-Stokes substep):
    // P += phi - pcn L_I phi, L_I the pressure operator's 1-D rows (pca, pcb,
    // pcc) in the directions marked in pimpl; null P: no update
    double* P;
    double pcn;
    int pimpl[3];
    const double* pca[3];
    const double* pcb[3];
    const double* pcc[3];
};
hipError_t launch_divergence(const ProjDesc& d, hipStream_t s);
hipError_t launch_gradient_update(const ProjDesc& d, hipStream_t s);

// Projection descriptor of a cell-centred pressure plan (periodic / Neumann
// boundaries): sizes, widths and face spacings; TPT_OK or an error.
int proj_desc(const tpt_plan_s* p, ProjDesc& d);

}  // namespace tpt
