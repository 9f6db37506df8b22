// Device helpers shared by the element kernels of the voxel hex8 mesh.
#pragma once

#include <hip/hip_runtime.h>

namespace afd {

// In place, per axis k, the node pairs (v0, v1) along k become (v0 + v1,
// v1 - v0): the tensor-product Haar transform of an element's 8 nodal
// vectors, nodes in binary order (bit k of the index = the node's side along
// axis k).  Index alpha of the result: bit k set = difference along k.
__device__ __forceinline__ void haar_fwd(double v[8][3]) {
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int st = 1 << ax;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            if (n & st) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double s = v[n][c] + v[n + st][c], d = v[n + st][c] - v[n][c];
                v[n][c] = s;
                v[n + st][c] = d;
            }
        }
    }
}

// The stress at the voxel centre, Voigt order (xx, yy, zz, yz, xz, xy), from
// the Haar-transformed displacements hv: the centroid gradient of component c
// along axis i is hv[1 << i][c] / (4 h_i) (the mean of the four edge
// differences along i); sigma = rho (lam tr(eps) I + 2 mu eps).
__device__ __forceinline__ void centroid_stress(const double hv[8][3], const double inv4h[3], double lam, double mu,
                                                double rho, double sig[6]) {
    double g[3][3];  // g[i][c] = d u_c / d x_i
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) g[i][c] = hv[1 << i][c] * inv4h[i];
    const double tr = g[0][0] + g[1][1] + g[2][2];
    sig[0] = rho * (lam * tr + 2.0 * mu * g[0][0]);
    sig[1] = rho * (lam * tr + 2.0 * mu * g[1][1]);
    sig[2] = rho * (lam * tr + 2.0 * mu * g[2][2]);
    sig[3] = rho * mu * (g[1][2] + g[2][1]);
    sig[4] = rho * mu * (g[0][2] + g[2][0]);
    sig[5] = rho * mu * (g[0][1] + g[1][0]);
}

}  // namespace afd
