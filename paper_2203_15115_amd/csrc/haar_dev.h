// The element matrix of a voxel in the tensor-product Haar basis: the
// element arithmetic shared by the tiled element-by-element apply and the
// persistent small-mesh solver.  Nodes in binary order a = ax + 2 ay + 4 az;
// the unnormalised two-point transform (v0, v1) -> (v0 + v1, v1 - v0) per
// axis, its transpose (s, d) -> (s - d, s + d) on the way back, and the
// element matrix in that basis: a diagonal plus the lam / mu couplings of
// pairs of modes that differ in two axes (45 nonzeros per component block),
// with the factor 1/8 of the transforms folded into the coefficients.
#pragma once

#include "afd_internal.h"

namespace afd {
namespace {

template <typename T>
struct KH {
    T dg[3][8];   // general voxel: diagonal of the Haar-basis element matrix
    T cl[3][2];   // lam * M_k(bit) / 4
    T cm[3][2];   // mu  * M_k(bit) / 4
    T kdiag[3];
    T dgc[2][3];  // cubic voxel: dg depends only on (alpha_i, number of other set bits)
    T clc[2], cmc[2];
};

template <typename T>
KH<T> to_kh(const KeHaar& k) {
    KH<T> o;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 8; ++a) o.dg[i][a] = (T)k.dg[i][a];
    for (int i = 0; i < 3; ++i)
        for (int b = 0; b < 2; ++b) {
            o.cl[i][b] = (T)k.cl[i][b];
            o.cm[i][b] = (T)k.cm[i][b];
        }
    for (int i = 0; i < 3; ++i) o.kdiag[i] = (T)k.kdiag[i];
    // representatives (component 0): alpha_0 = bit, others = first n of bits 1, 2
    const int rep[2][3] = {{0, 2, 6}, {1, 3, 7}};
    for (int b = 0; b < 2; ++b)
        for (int n = 0; n < 3; ++n) o.dgc[b][n] = (T)k.dg[0][rep[b][n]];
    for (int b = 0; b < 2; ++b) {
        o.clc[b] = (T)k.cl[0][b];
        o.cmc[b] = (T)k.cm[0][b];
    }
    return o;
}

bool is_cubic(const KeHaar& k) {
    // all three axes share the same 1-D integrals iff the coefficient tables
    // are symmetric under axis permutation
    for (int b = 0; b < 2; ++b)
        if (k.cl[0][b] != k.cl[1][b] || k.cl[0][b] != k.cl[2][b] || k.cm[0][b] != k.cm[1][b] ||
            k.cm[0][b] != k.cm[2][b])
            return false;
    for (int i = 0; i < 3; ++i)
        for (int a = 1; a < 8; ++a) {
            const int bi = (a >> i) & 1, n = __builtin_popcount(a & ~(1 << i));
            const int rep[2][3] = {{0, 2, 6}, {1, 3, 7}};
            if (k.dg[i][a] != k.dg[0][rep[bi][n]]) return false;
        }
    return true;
}

template <typename T, bool CUB>
__device__ __forceinline__ T dgv(const KH<T>& kh, int i, int al) {
    if constexpr (CUB) return kh.dgc[(al >> i) & 1][__builtin_popcount(al & ~(1 << i))];
    else return kh.dg[i][al];
}
template <typename T, bool CUB>
__device__ __forceinline__ T clv(const KH<T>& kh, int k, int b) {
    if constexpr (CUB) return kh.clc[b];
    else return kh.cl[k][b];
}
template <typename T, bool CUB>
__device__ __forceinline__ T cmv(const KH<T>& kh, int k, int b) {
    if constexpr (CUB) return kh.cmc[b];
    else return kh.cm[k][b];
}

// forward x then y stage of a face: q = ax + 2 ay, (v0, v1) -> (v0 + v1, v1 - v0)
template <typename T>
__device__ __forceinline__ void face_fwd(T f[4][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T s0 = f[0][c] + f[1][c], d0 = f[1][c] - f[0][c];
        T s1 = f[2][c] + f[3][c], d1 = f[3][c] - f[2][c];
        f[0][c] = s0 + s1;
        f[2][c] = s1 - s0;
        f[1][c] = d0 + d1;
        f[3][c] = d1 - d0;
    }
}
// inverse y then x stage: (s, d) -> (s - d, s + d)
template <typename T>
__device__ __forceinline__ void face_inv(T f[4][3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T a0 = f[0][c] - f[2][c], a2 = f[0][c] + f[2][c];
        T a1 = f[1][c] - f[3][c], a3 = f[1][c] + f[3][c];
        f[0][c] = a0 - a1;
        f[1][c] = a0 + a1;
        f[2][c] = a2 - a3;
        f[3][c] = a2 + a3;
    }
}

// element step in the Haar basis: from the transformed bottom (bf) and top (tf)
// faces, produce the transformed bottom (yb) and top (yt) face outputs of
// rho * Ke u_e (z stage done here; x/y stages are per face)
template <typename T, bool CUB>
__device__ __forceinline__ void element_haar(const KH<T>& kh, T rho, const T bf[4][3], const T tf[4][3],
                                             T yb[4][3], T yt[4][3]) {
    T v[8][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            v[q][c] = bf[q][c] + tf[q][c];
            v[q + 4][c] = tf[q][c] - bf[q][c];
        }
    T y[8][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) y[0][c] = T(0);
    if constexpr (CUB) {
        // fold rho into the ten distinct coefficients of a cubic voxel
        T rd[2][3], rl[2], rm[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
#pragma unroll
            for (int n = 0; n < 3; ++n) rd[b][n] = rho * kh.dgc[b][n];
            rl[b] = rho * kh.clc[b];
            rm[b] = rho * kh.cmc[b];
        }
#pragma unroll
        for (int al = 1; al < 8; ++al) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T acc = rd[(al >> i) & 1][__builtin_popcount(al & ~(1 << i))] * v[al][i];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j == i) continue;
                    const int k = 3 - i - j;
                    const int bi = (al >> i) & 1, bj = (al >> j) & 1, bk = (al >> k) & 1;
                    if (bi == bj) continue;
                    acc = fma(bi ? rl[bk] : rm[bk], v[al ^ (1 << i) ^ (1 << j)][j], acc);
                }
                y[al][i] = acc;
            }
        }
    } else {
#pragma unroll
        for (int al = 1; al < 8; ++al) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T acc = dgv<T, CUB>(kh, i, al) * v[al][i];
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (j == i) continue;
                    const int k = 3 - i - j;
                    const int bi = (al >> i) & 1, bj = (al >> j) & 1, bk = (al >> k) & 1;
                    if (bi == bj) continue;
                    const T cf = bi ? clv<T, CUB>(kh, k, bk) : cmv<T, CUB>(kh, k, bk);
                    acc = fma(cf, v[al ^ (1 << i) ^ (1 << j)][j], acc);
                }
                y[al][i] = rho * acc;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            yb[q][c] = y[q][c] - y[q + 4][c];
            yt[q][c] = y[q][c] + y[q + 4][c];
        }
}

}  // namespace
}  // namespace afd
