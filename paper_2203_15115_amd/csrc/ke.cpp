// Element matrix of an isotropic hx*hy*hz voxel (the K^e of Eq. 3.5), in the
// two forms the kernels use.
//
// Ke[(a,i),(b,j)] = lam G^ij_ab + mu G^ji_ab + delta_ij mu sum_k G^kk_ab, with
// G^pq_ab = int dN_a/dx_p dN_b/dx_q a product over the axes of the 1-D
// integrals of linear shape functions: S = int phi' phi' (axis p = q),
// C = int phi'_a phi_b (axis p), C^T (axis q), M = int phi phi (other axes).
// In the per-axis basis (s, d) = (v0 + v1, v1 - v0) these become
// S -> diag(0, 1/h), M -> diag(h/4, h/12), C -> single entry 1/2 at (d, s),
// which gives the block-sparse form stored in KeHaar (45 nonzeros of 576).
#include <cmath>

#include "afd_internal.h"

namespace afd {

static inline double mhat(const double h[3], int k, int bit) { return bit ? h[k] / 12.0 : h[k] / 4.0; }
static inline double shat(const double h[3], int k, int bit) { return bit ? 1.0 / h[k] : 0.0; }

KeHaar make_ke_haar(const double h[3], double E, double nu) {
    const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    const double mu = E / (2.0 * (1.0 + nu));
    KeHaar kh{};
    for (int al = 0; al < 8; ++al) {
        int bits[3] = {al & 1, (al >> 1) & 1, (al >> 2) & 1};
        double g[3];
        for (int k = 0; k < 3; ++k) {
            double v = shat(h, k, bits[k]);
            for (int m = 0; m < 3; ++m)
                if (m != k) v *= mhat(h, m, bits[m]);
            g[k] = v;
        }
        for (int i = 0; i < 3; ++i) kh.dg[i][al] = (lam + 2.0 * mu) * g[i] + mu * (g[0] + g[1] + g[2] - g[i]);
    }
    for (int k = 0; k < 3; ++k)
        for (int bit = 0; bit < 2; ++bit) {
            kh.cl[k][bit] = lam * mhat(h, k, bit) / 4.0;
            kh.cm[k][bit] = mu * mhat(h, k, bit) / 4.0;
        }
    // diagonal of Ke for component c: (lam + 2 mu) int (dN/dx_c)^2 + mu sum_{k != c} int (dN/dx_k)^2,
    // int (dN/dx_k)^2 = (1/h_k) * prod_{m != k} (h_m / 3)
    double q[3];
    for (int k = 0; k < 3; ++k) {
        q[k] = 1.0 / h[k];
        for (int m = 0; m < 3; ++m)
            if (m != k) q[k] *= h[m] / 3.0;
    }
    for (int c = 0; c < 3; ++c) kh.kdiag[c] = (lam + 2.0 * mu) * q[c] + mu * (q[0] + q[1] + q[2] - q[c]);
    return kh;
}

// Dense Ke in the public local node order (bottom face counter-clockwise, then
// top face), built by applying the Haar form to unit vectors.
void make_ke_dense(const double h[3], double E, double nu, double* ke) {
    static const int LOC[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                  {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
    KeHaar kh = make_ke_haar(h, E, nu);
    for (int col = 0; col < 24; ++col) {
        double v[8][3] = {};
        int a = col / 3, c = col % 3;
        v[LOC[a][0] + 2 * LOC[a][1] + 4 * LOC[a][2]][c] = 1.0;
        for (int ax = 0; ax < 3; ++ax) {
            int st = 1 << ax;
            for (int n = 0; n < 8; ++n)
                if (!(n & st))
                    for (int cc = 0; cc < 3; ++cc) {
                        double s = v[n][cc] + v[n + st][cc], d = v[n + st][cc] - v[n][cc];
                        v[n][cc] = s;
                        v[n + st][cc] = d;
                    }
        }
        double y[8][3] = {};
        for (int al = 0; al < 8; ++al)
            for (int i = 0; i < 3; ++i) {
                double acc = kh.dg[i][al] * v[al][i];
                for (int j = 0; j < 3; ++j) {
                    if (j == i) continue;
                    int k = 3 - i - j;
                    int bi = (al >> i) & 1, bj = (al >> j) & 1, bk = (al >> k) & 1;
                    if (bi == bj) continue;
                    double cf = bi ? kh.cl[k][bk] : kh.cm[k][bk];
                    acc += cf * v[al ^ (1 << i) ^ (1 << j)][j];
                }
                y[al][i] = acc;
            }
        for (int ax = 0; ax < 3; ++ax) {
            int st = 1 << ax;
            for (int n = 0; n < 8; ++n)
                if (!(n & st))
                    for (int cc = 0; cc < 3; ++cc) {
                        double s = y[n][cc], d = y[n + st][cc];
                        y[n][cc] = s - d;
                        y[n + st][cc] = s + d;
                    }
        }
        for (int b = 0; b < 8; ++b)
            for (int cc = 0; cc < 3; ++cc)
                ke[(3 * b + cc) * 24 + col] = y[LOC[b][0] + 2 * LOC[b][1] + 4 * LOC[b][2]][cc];
    }
}

}  // namespace afd
