// Element-by-element operator apply y = sum_e rho_e P_e^T Ke P_e u (the
// assembly-free matrix-vector product of Sec. 3.5), for one shared voxel Ke.
//
// Work decomposition (gfx950, wave64):
//  * a workgroup of 256 threads owns a 16x16 column of ELEMENTS in x-y and
//    marches in z over a chunk of node planes; consecutive workgroups overlap
//    by one element so that each owns 15x15 NODES exactly (no atomics, fixed
//    summation order => bitwise reproducible);
//  * per element layer the next node plane (17x17 nodes, interleaved DOFs,
//    contiguous 51-value rows => coalesced) is staged in LDS; each thread
//    keeps its element's lower four nodes in registers from the previous layer;
//  * each thread applies rho_e Ke to its element in the tensor-product Haar
//    basis (45 multiplies instead of 576) and parks the 24 results in LDS;
//  * each owned node gathers its 8 contributions in a fixed order: the upper
//    corners of layer k-1 (carried in registers) plus the lower corners of
//    layer k, and the plane is written once.
//
// Modes: APPLY (Y = A U), RESID (R = F - A X, with partial sums of r.M^-1 r and
// r.r) and DIR (the deflated CG direction P' = beta P + M^-1 R - W mu formed
// while staging, Q = A P', partial sums of p'.q).
#include <cstdio>
#include <cstdlib>

#include "afd_internal.h"

namespace afd {

namespace {

constexpr int TX = 16, TY = 16, NT = TX * TY;  // element tile (threads)
constexpr int PX = TX + 1, PY = TY + 1;        // node plane in LDS
constexpr int PLANE = PX * PY * 3;

enum { APPLY = 0, RESID = 1, DIR = 2 };

template <typename T>
struct KH {
    T dg[3][8];
    T cl[3][2];
    T cm[3][2];
    T kdiag[3];
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
    return o;
}

template <typename T>
struct MvParams {
    int nx, ny, nz;
    int tiles_x, tiles_y, zc, nchunk;
    int64_t ndof;
    const T* rho;
    const uint8_t* nmask;
    const T* U;     // APPLY: input; RESID: X; DIR: P (old)
    T* Y;           // APPLY: output; RESID: R; DIR: Q
    const T* F;     // RESID: F; DIR: R (residual)
    T* Pn;          // DIR: new direction (owned nodes written)
    const double* rinv;  // per node 1/sum rho (double)
    const float* rinv32;
    // deflation
    int deflate;
    int b[3], nb[3];
    double inv_scale;
    const double* mu;
    int ncoarse;
    CgScalars* sc;
    double* partial;  // [rhs][npart]
    int npart;
};

// y = rho * Ke v for one element; v,y indexed [bit pattern ax+2ay+4az][comp]
template <typename T>
__device__ __forceinline__ void element_apply(const KH<T>& kh, T rho, T v[8][3], T y[8][3]) {
    // forward Haar per axis: (v0, v1) -> (v0 + v1, v1 - v0)
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const int st = 1 << ax;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            if (n & st) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T s = v[n][c] + v[n + st][c];
                T d = v[n + st][c] - v[n][c];
                v[n][c] = s;
                v[n + st][c] = d;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) y[0][c] = T(0);
#pragma unroll
    for (int al = 1; al < 8; ++al) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T acc = kh.dg[i][al] * v[al][i];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (j == i) continue;
                const int k = 3 - i - j;
                const int bi = (al >> i) & 1, bj = (al >> j) & 1, bk = (al >> k) & 1;
                if (bi == bj) continue;
                const T cf = bi ? kh.cl[k][bk] : kh.cm[k][bk];
                acc = fma(cf, v[al ^ (1 << i) ^ (1 << j)][j], acc);
            }
            y[al][i] = rho * acc;
        }
    }
    // inverse per axis: (s, d) -> (s - d, s + d)
#pragma unroll
    for (int ax = 2; ax >= 0; --ax) {
        const int st = 1 << ax;
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            if (n & st) continue;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                T s = y[n][c], d = y[n + st][c];
                y[n][c] = s - d;
                y[n + st][c] = s + d;
            }
        }
    }
}

// rigid-motion value of block coarse vector mu at node (i,j,k), component c
__device__ __forceinline__ double wmu(const int b[3], const int nb[3], int nx, int ny, int nz, double inv_scale,
                                      const double* mu, int i, int j, int k, int c) {
    const int n[3] = {nx, ny, nz};
    const int p[3] = {i, j, k};
    int bidx[3];
    double x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int bb = p[a] / b[a];
        if (bb > nb[a] - 1) bb = nb[a] - 1;
        const int lo = bb * b[a];
        const int hi = (bb == nb[a] - 1) ? n[a] : lo + b[a] - 1;
        bidx[a] = bb;
        x[a] = (p[a] - 0.5 * (lo + hi)) * inv_scale;
    }
    const double* m = mu + 6 * (bidx[0] + nb[0] * (bidx[1] + nb[1] * bidx[2]));
    if (c == 0) return m[0] + m[4] * x[2] - m[5] * x[1];
    if (c == 1) return m[1] - m[3] * x[2] + m[5] * x[0];
    return m[2] + m[3] * x[1] - m[4] * x[0];
}

template <typename T>
__device__ __forceinline__ double rinv_of(const MvParams<T>& P, int64_t node) {
    if constexpr (sizeof(T) == 8) return P.rinv[node];
    else return (double)P.rinv32[node];
}

template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_matvec(MvParams<T> P, KH<T> kh) {
    __shared__ T plane[PLANE];
    __shared__ T outb[24 * NT];
    __shared__ double red[NT / 64][2];

    const int rhs = blockIdx.y;
    if constexpr (MODE != APPLY) {
        if (P.sc[rhs].done) return;
    }
    const int t = threadIdx.x;
    const int lx = t % TX, ly = t / TX;
    const int tile = blockIdx.x % (P.tiles_x * P.tiles_y);
    const int chunk = blockIdx.x / (P.tiles_x * P.tiles_y);
    const int X0 = (tile % P.tiles_x) * (TX - 1) - 1;
    const int Y0 = (tile / P.tiles_x) * (TY - 1) - 1;
    const int Z0 = chunk * P.zc;
    const int Z1 = min(Z0 + P.zc, P.nz + 1);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int64_t sy = nx + 1, sz = (int64_t)(nx + 1) * (ny + 1);
    const T* U = P.U + rhs * P.ndof;
    T* Y = P.Y + rhs * P.ndof;
    const T* F = (MODE != APPLY) ? P.F + rhs * P.ndof : nullptr;
    T* Pn = (MODE == DIR) ? P.Pn + rhs * P.ndof : nullptr;
    const double* mu = (MODE == DIR && P.deflate) ? P.mu + (int64_t)rhs * P.ncoarse : nullptr;
    T beta = T(0);
    if constexpr (MODE == DIR) beta = (T)P.sc[rhs].beta;

    const int gi = X0 + lx, gj = Y0 + ly;  // this thread's element (ex, ey) and owned node (i, j)
    const bool own = lx >= 1 && ly >= 1 && gi <= nx && gj <= ny;
    const bool elem_xy = gi >= 0 && gi < nx && gj >= 0 && gj < ny;

    // stage node plane gk into LDS (masked input; DIR: direction formed here)
    auto stage = [&](int gk) {
        for (int f = t; f < PLANE; f += NT) {
            const int row = f / (PX * 3);
            const int rem = f - row * (PX * 3);
            const int li = rem / 3;
            const int c = rem - li * 3;
            const int i = X0 + li, j = Y0 + row;
            T v = T(0);
            if (i >= 0 && i <= nx && j >= 0 && j <= ny && gk >= 0 && gk <= nz) {
                const int64_t node = i + sy * j + sz * gk;
                if (!((P.nmask[node] >> c) & 1)) {
                    if constexpr (MODE == DIR) {
                        const int64_t a = 3 * node + c;
                        double z = rinv_of(P, node) / (double)kh.kdiag[c] * (double)F[a];
                        double pv = (double)beta * (double)U[a] + z;
                        if (mu) pv -= wmu(P.b, P.nb, nx, ny, nz, P.inv_scale, mu, i, j, gk, c);
                        v = (T)pv;
                    } else {
                        v = U[3 * node + c];
                    }
                }
            }
            plane[f] = v;
        }
    };

    T lo[4][3];       // element's lower four nodes: (0,0),(1,0),(0,1),(1,1)
    T carry[3] = {T(0), T(0), T(0)};
    double acc0 = 0.0, acc1 = 0.0;

    stage(Z0 - 1);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int li = lx + (q & 1), lj = ly + (q >> 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) lo[q][c] = plane[(lj * PX + li) * 3 + c];
    }

    for (int k = Z0 - 1; k < Z1; ++k) {  // element layer k spans node planes k, k+1
        __syncthreads();
        stage(k + 1);
        __syncthreads();
        T v[8][3], y[8][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int li = lx + (q & 1), lj = ly + (q >> 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[q][c] = lo[q][c];
                const T up = plane[(lj * PX + li) * 3 + c];
                v[q + 4][c] = up;
                lo[q][c] = up;
            }
        }
        // DIR: owned nodes of plane k+1 write the new direction
        if constexpr (MODE == DIR) {
            if (own && k + 1 >= Z0 && k + 1 < Z1) {
                const int64_t node = gi + sy * gj + sz * (k + 1);
#pragma unroll
                for (int c = 0; c < 3; ++c) Pn[3 * node + c] = v[4][c];
            }
        }
        T ownk[3];  // this thread's node (gi, gj) on plane k, as staged
#pragma unroll
        for (int c = 0; c < 3; ++c) ownk[c] = v[0][c];
        const bool valid = elem_xy && k >= 0 && k < nz;
        const T r = valid ? P.rho[gi + (int64_t)nx * (gj + (int64_t)ny * k)] : T(0);
        element_apply<T>(kh, r, v, y);
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int c = 0; c < 3; ++c) outb[(n * 3 + c) * NT + t] = y[n][c];
        __syncthreads();
        if (own) {
            const int t00 = t - TX - 1, t10 = t - TX, t01 = t - 1, t11 = t;
            T bot[3], top[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bot[c] = outb[(3 * 3 + c) * NT + t00] + outb[(2 * 3 + c) * NT + t10] +
                         outb[(1 * 3 + c) * NT + t01] + outb[(0 * 3 + c) * NT + t11];
                top[c] = outb[(7 * 3 + c) * NT + t00] + outb[(6 * 3 + c) * NT + t10] +
                         outb[(5 * 3 + c) * NT + t01] + outb[(4 * 3 + c) * NT + t11];
            }
            if (k >= Z0) {  // node plane k is complete
                const int64_t node = gi + sy * gj + sz * k;
                const uint8_t m = P.nmask[node];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int64_t a = 3 * node + c;
                    const T yv = carry[c] + bot[c];
                    const bool fx = (m >> c) & 1;
                    if constexpr (MODE == APPLY) {
                        Y[a] = fx ? U[a] : yv;
                    } else if constexpr (MODE == RESID) {
                        const T rv = fx ? T(0) : (T)(F[a] - yv);
                        Y[a] = rv;
                        const double z = rinv_of(P, node) / (double)kh.kdiag[c] * (double)rv;
                        acc0 += (double)rv * z;
                        acc1 += (double)rv * (double)rv;
                    } else {  // DIR: q = A p' (p' = 0 on fixed DOFs, so q = 0 there)
                        const T qv = fx ? T(0) : yv;
                        Y[a] = qv;
                        acc0 += (double)ownk[c] * (double)qv;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) carry[c] = top[c];
        }
    }
    if constexpr (MODE != APPLY) {
        // fixed-order workgroup reduction -> one partial per workgroup
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            acc0 += __shfl_down(acc0, off, 64);
            acc1 += __shfl_down(acc1, off, 64);
        }
        __syncthreads();
        if ((t & 63) == 0) {
            red[t >> 6][0] = acc0;
            red[t >> 6][1] = acc1;
        }
        __syncthreads();
        if (t == 0) {
            double s0 = 0.0, s1 = 0.0;
            for (int w = 0; w < NT / 64; ++w) {
                s0 += red[w][0];
                s1 += red[w][1];
            }
            P.partial[(int64_t)(rhs * 2 + 0) * P.npart + blockIdx.x] = s0;
            P.partial[(int64_t)(rhs * 2 + 1) * P.npart + blockIdx.x] = s1;
        }
    }
}

int g_zc_override = -1;

void tiling(const Grid& g, int& tx, int& ty, int& zc, int& nchunk) {
    tx = (g.nx + 1 + (TX - 2)) / (TX - 1);  // ceil((nx+1)/15)
    ty = (g.ny + 1 + (TY - 2)) / (TY - 1);
    if (g_zc_override < 0) {
        const char* e = getenv("AFD_MATVEC_ZC");
        g_zc_override = e ? atoi(e) : 0;
    }
    const int planes = g.nz + 1;
    if (g_zc_override > 0) {
        zc = g_zc_override;
    } else {
        // aim at ~1024 workgroups (4 per CU) while keeping the one-layer
        // z-overlap small
        int want = (1024 + tx * ty - 1) / (tx * ty);
        if (want < 1) want = 1;
        zc = (planes + want - 1) / want;
        if (zc < 8) zc = 8;
    }
    if (zc > planes) zc = planes;
    nchunk = (planes + zc - 1) / zc;
}

template <typename T>
MvParams<T> base_params(const MatvecArgs& a) {
    MvParams<T> p{};
    p.nx = a.g.nx;
    p.ny = a.g.ny;
    p.nz = a.g.nz;
    tiling(a.g, p.tiles_x, p.tiles_y, p.zc, p.nchunk);
    p.ndof = a.g.ndof;
    if constexpr (sizeof(T) == 8) p.rho = a.rho;
    else p.rho = a.rho32;
    p.nmask = a.nmask;
    return p;
}

template <typename T, int MODE>
int launch(const MvParams<T>& p, const KH<T>& kh, int nrhs, hipStream_t s) {
    if (nrhs < 1 || nrhs > 4) {
        set_error("nrhs must be in 1..4");
        return AFD_E_INVALID_ARG;
    }
    dim3 grid(p.tiles_x * p.tiles_y * p.nchunk, nrhs);
    hipLaunchKernelGGL((k_matvec<T, MODE>), grid, dim3(NT), 0, s, p, kh);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

}  // namespace

int matvec_num_tiles(const Grid& g) {
    int tx, ty, zc, nc;
    tiling(g, tx, ty, zc, nc);
    return tx * ty * nc;
}

int launch_apply(const MatvecArgs& a, const KeHaar& kh, int fp32, int nrhs, const void* U, void* Y,
                 hipStream_t s) {
    if (fp32) {
        MvParams<float> p = base_params<float>(a);
        p.U = (const float*)U;
        p.Y = (float*)Y;
        return launch<float, APPLY>(p, to_kh<float>(kh), nrhs, s);
    }
    MvParams<double> p = base_params<double>(a);
    p.U = (const double*)U;
    p.Y = (double*)Y;
    return launch<double, APPLY>(p, to_kh<double>(kh), nrhs, s);
}

template <typename T>
static void set_dcg(MvParams<T>& p, const DcgArgs& d) {
    p.rinv = d.rinv;
    p.deflate = d.deflate;
    for (int i = 0; i < 3; ++i) {
        p.b[i] = d.blk.b[i];
        p.nb[i] = d.blk.nb[i];
    }
    p.inv_scale = d.blk.inv_scale;
    p.mu = d.mu;
    p.ncoarse = d.blk.ncoarse;
    p.sc = d.sc;
    p.partial = d.partial;
    p.npart = d.npart;
}

int launch_residual(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, int nrhs, const double* F,
                    const double* X, double* R, hipStream_t s) {
    MvParams<double> p = base_params<double>(a);
    set_dcg(p, d);
    p.U = X;
    p.Y = R;
    p.F = F;
    return launch<double, RESID>(p, to_kh<double>(kh), nrhs, s);
}

int launch_dir_apply(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, int nrhs, const double* Pold,
                     double* Pnew, const double* R, double* Q, hipStream_t s) {
    MvParams<double> p = base_params<double>(a);
    set_dcg(p, d);
    p.U = Pold;
    p.Pn = Pnew;
    p.F = R;
    p.Y = Q;
    return launch<double, DIR>(p, to_kh<double>(kh), nrhs, s);
}

int launch_residual_f32(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, const float* rinv32, int nrhs,
                        const float* F, const float* X, float* R, hipStream_t s) {
    MvParams<float> p = base_params<float>(a);
    set_dcg(p, d);
    p.rinv32 = rinv32;
    p.U = X;
    p.Y = R;
    p.F = F;
    return launch<float, RESID>(p, to_kh<float>(kh), nrhs, s);
}

int launch_dir_apply_f32(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, const float* rinv32, int nrhs,
                         const float* Pold, float* Pnew, const float* R, float* Q, hipStream_t s) {
    MvParams<float> p = base_params<float>(a);
    set_dcg(p, d);
    p.rinv32 = rinv32;
    p.U = Pold;
    p.Pn = Pnew;
    p.F = R;
    p.Y = Q;
    return launch<float, DIR>(p, to_kh<float>(kh), nrhs, s);
}

}  // namespace afd
