// Tangent-linear (Born) forward: source terms of the model perturbation, one thread per
// cell.  The derivative of one step along (dlam, dmu, drho) is the same step applied to
// the perturbation state plus the first-order effect of the perturbation on the
// background, which these kernels add to the perturbation state just before the
// perturbation's own pass runs (so that pass's damping acts on it as on everything else):
//   velocity:  dv     += dt db (D_S sigma) + db c s,   db = -b^2 drho_eff
//                        (c s the background force term, which carries b)
//   stress:    dsigma += dt dC E(v)                      dC from dlam and dmu
// with sigma (before the stress pass) and v (after the velocity pass) the background at
// that point of the step (Sec. 2.1 Eq.(1)-(3) with Eq.(4), differentiated).  Damped
// boundaries only.
#pragma once

#include "common.h"
#include "fwd_cell.h"

namespace fd3d {

template <typename T> struct BornOut {
    T *f[6];  // the perturbation's velocity (3) or stress (6) components
};

template <typename T>
__global__ void __launch_bounds__(256) born_vel_source(Grid<T> G, BornOut<T> dv, const T *__restrict__ drho,
                                                      Inject<T> src, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const long p = i + G.sy * j + G.sz * k;
    const T s = src.on ? src.wavelet[n] : T(0);
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;
    const long off[3] = {1, G.sy, G.sz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const bool act = c == 0 ? i <= G.nx - 2 : (c == 1 ? j <= G.ny - 2 : k <= G.nz - 2);
        if (!act) continue;
        T d;
        if (c == 0)
            d = dstag(rd<SXX>(G, i + 1, j, k), rd<SXX>(G, i, j, k), rd<SXX>(G, i + 2, j, k), rd<SXX>(G, i - 1, j, k), rdx)
              + dstag(rd<SXY>(G, i, j, k), rd<SXY>(G, i, j - 1, k), rd<SXY>(G, i, j + 1, k), rd<SXY>(G, i, j - 2, k), rdy)
              + dstag(rd<SXZ>(G, i, j, k), rd<SXZ>(G, i, j, k - 1), rd<SXZ>(G, i, j, k + 1), rd<SXZ>(G, i, j, k - 2), rdz);
        else if (c == 1)
            d = dstag(rd<SXY>(G, i, j, k), rd<SXY>(G, i - 1, j, k), rd<SXY>(G, i + 1, j, k), rd<SXY>(G, i - 2, j, k), rdx)
              + dstag(rd<SYY>(G, i, j + 1, k), rd<SYY>(G, i, j, k), rd<SYY>(G, i, j + 2, k), rd<SYY>(G, i, j - 1, k), rdy)
              + dstag(rd<SYZ>(G, i, j, k), rd<SYZ>(G, i, j, k - 1), rd<SYZ>(G, i, j, k + 1), rd<SYZ>(G, i, j, k - 2), rdz);
        else
            d = dstag(rd<SXZ>(G, i, j, k), rd<SXZ>(G, i - 1, j, k), rd<SXZ>(G, i + 1, j, k), rd<SXZ>(G, i - 2, j, k), rdx)
              + dstag(rd<SYZ>(G, i, j, k), rd<SYZ>(G, i, j - 1, k), rd<SYZ>(G, i, j + 1, k), rd<SYZ>(G, i, j - 2, k), rdy)
              + dstag(rd<SZZ>(G, i, j, k + 1), rd<SZZ>(G, i, j, k), rd<SZZ>(G, i, j, k + 2), rd<SZZ>(G, i, j, k - 1), rdz);
        const T b = buoy(G.rho[p], G.rho[p + off[c]]);
        const T db = -(b * b) * ((drho[p] + drho[p + off[c]]) * T(0.5));
        T add = dt * db * d;
        const int t = tap_of(src, VX + c, i, j, k);
        if (t >= 0) add += db * src.coef[(VX + c) * 8 + t] * s;
        dv.f[c][p] += add;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) born_stress_source(Grid<T> G, BornOut<T> ds, const T *__restrict__ dlam,
                                                         const T *__restrict__ dmu)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const long p = i + G.sy * j + G.sz * k;
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;
    const T exx = dstag(rd<VX>(G, i, j, k), rd<VX>(G, i - 1, j, k), rd<VX>(G, i + 1, j, k), rd<VX>(G, i - 2, j, k), rdx);
    const T eyy = dstag(rd<VY>(G, i, j, k), rd<VY>(G, i, j - 1, k), rd<VY>(G, i, j + 1, k), rd<VY>(G, i, j - 2, k), rdy);
    const T ezz = dstag(rd<VZ>(G, i, j, k), rd<VZ>(G, i, j, k - 1), rd<VZ>(G, i, j, k + 1), rd<VZ>(G, i, j, k - 2), rdz);
    const T tr = exx + eyy + ezz;
    const T l = dlam[p], m = dmu[p];
    ds.f[0][p] += dt * (l * tr + T(2) * m * exx);
    ds.f[1][p] += dt * (l * tr + T(2) * m * eyy);
    ds.f[2][p] += dt * (l * tr + T(2) * m * ezz);
    if (i <= G.nx - 2 && j <= G.ny - 2) {
        const T e = dstag(rd<VX>(G, i, j + 1, k), rd<VX>(G, i, j, k), rd<VX>(G, i, j + 2, k), rd<VX>(G, i, j - 1, k), rdy)
                  + dstag(rd<VY>(G, i + 1, j, k), rd<VY>(G, i, j, k), rd<VY>(G, i + 2, j, k), rd<VY>(G, i - 1, j, k), rdx);
        const T mxy = ((dmu[p] + dmu[p + 1]) + (dmu[p + G.sy] + dmu[p + 1 + G.sy])) / T(4);
        ds.f[3][p] += dt * mxy * e;
    }
    if (i <= G.nx - 2 && k <= G.nz - 2) {
        const T e = dstag(rd<VX>(G, i, j, k + 1), rd<VX>(G, i, j, k), rd<VX>(G, i, j, k + 2), rd<VX>(G, i, j, k - 1), rdz)
                  + dstag(rd<VZ>(G, i + 1, j, k), rd<VZ>(G, i, j, k), rd<VZ>(G, i + 2, j, k), rd<VZ>(G, i - 1, j, k), rdx);
        const T mxz = ((dmu[p] + dmu[p + 1]) + (dmu[p + G.sz] + dmu[p + 1 + G.sz])) / T(4);
        ds.f[4][p] += dt * mxz * e;
    }
    if (j <= G.ny - 2 && k <= G.nz - 2) {
        const T e = dstag(rd<VY>(G, i, j, k + 1), rd<VY>(G, i, j, k), rd<VY>(G, i, j, k + 2), rd<VY>(G, i, j, k - 1), rdz)
                  + dstag(rd<VZ>(G, i, j + 1, k), rd<VZ>(G, i, j, k), rd<VZ>(G, i, j + 2, k), rd<VZ>(G, i, j - 1, k), rdy);
        const T myz = ((dmu[p] + dmu[p + G.sy]) + (dmu[p + G.sz] + dmu[p + G.sy + G.sz])) / T(4);
        ds.f[5][p] += dt * myz * e;
    }
}

} // namespace fd3d
