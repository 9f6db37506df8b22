// Modal analysis (the eigenvalue constraint of Eq. 3.21 and its sensitivity,
// Eq. 3.4): the lowest eigenpairs of K phi = lambda M phi on the free DOFs by
// subspace iteration with a block of four vectors, each step one four-column
// deflated solve (the assembly-free K^-1 of Sec. 3.5) and a Rayleigh-Ritz
// projection; M is the consistent mass matrix applied element by element
// (never assembled), each element's mass scaled by its stiffness scale.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "afd_internal.h"
#include "voxel_dev.h"

namespace afd {

namespace {

constexpr int BLK = 4;  // subspace block (the solver's right-hand sides per launch)

struct MassP {
    int nx, ny, nz;
    int64_t ndof;
    double w[4];        // h_x h_y h_z (1/3)^(3-d) (1/6)^d for d = 0..3 axes on which two corners differ
    const double* rho;
    const uint8_t* nmask;
};

// Y[r] = M U[r] on free DOFs (fixed inputs taken as zero), 0 on fixed DOFs:
// one thread per node gathers its up to 8 elements' rows of rho_e M_e u_e in a
// fixed order (no atomics, bitwise reproducible)
__global__ void k_mass_apply(MassP p, const double* U, double* Y) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1);
    const int nn = sz * (nz + 1);  // 3 nn < 2^31 (checked at mesh creation)
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int r = blockIdx.y;
    const double* u = U + (int64_t)r * p.ndof;
    const int i = n % sy, j = (n / sy) % (ny + 1), k = n / sz;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int dz = 0; dz < 2; ++dz) {
        const int ez = k - 1 + dz;
        if (ez < 0 || ez >= nz) continue;
        for (int dy = 0; dy < 2; ++dy) {
            const int ey = j - 1 + dy;
            if (ey < 0 || ey >= ny) continue;
            for (int dx = 0; dx < 2; ++dx) {
                const int ex = i - 1 + dx;
                if (ex < 0 || ex >= nx) continue;
                // this node is corner (1-dx, 1-dy, 1-dz) of element (ex, ey, ez)
                const int ax = 1 - dx, ay = 1 - dy, az = 1 - dz;
                double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
                    const int m = (ex + bx) + sy * (ey + by) + sz * (ez + bz);
                    const uint8_t mk = p.nmask[m];
                    const double wgt = p.w[(bx != ax) + (by != ay) + (bz != az)];
#pragma unroll
                    for (int c = 0; c < 3; ++c) s[c] += ((mk >> c) & 1) ? 0.0 : wgt * u[3 * (int64_t)m + c];
                }
                const double re = p.rho[ex + nx * (ey + ny * ez)];
#pragma unroll
                for (int c = 0; c < 3; ++c) acc[c] += re * s[c];
            }
        }
    }
    const uint8_t mk = p.nmask[n];
    double* y = Y + (int64_t)r * p.ndof + 3 * (int64_t)n;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c] = ((mk >> c) & 1) ? 0.0 : acc[c];
}

// S[f][e] -= lam[f] * rho_e phi_e^T M_e phi_e: the kinetic term of the
// eigenvalue sensitivity (S holds rho_e phi_e^T K_e phi_e).  In the per-axis
// Haar basis (v0 + v1, v1 - v0) the 1-D mass matrix is h diag(1/4, 1/12), so
// M_e is diagonal there: mass[alpha] = prod_k h_k (alpha_k ? 1/12 : 1/4).
struct KinP {
    int nx, ny, nz;
    int64_t ndof;
    int nf;
    double lam[BLK];
    double mass[8];
    const double* Phi;
    const double* rho;
};
__global__ void k_kinetic(KinP p, double* S) {
    const int nE = p.nx * p.ny * p.nz;  // < 2^31 (checked on the host)
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const int f = blockIdx.y;
    const int ex = e % p.nx, exy = e / p.nx, ey = exy % p.ny, ez = exy / p.ny;
    const int sy = p.nx + 1, sz = (p.nx + 1) * (p.ny + 1);
    const double* ph = p.Phi + (int64_t)f * p.ndof;
    double v[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int64_t nd = (ex + (a & 1)) + sy * (ey + ((a >> 1) & 1)) + (int64_t)sz * (ez + (a >> 2));
#pragma unroll
        for (int c = 0; c < 3; ++c) v[a][c] = ph[3 * nd + c];
    }
    haar_fwd(v);
    double kin = 0.0;
#pragma unroll
    for (int al = 0; al < 8; ++al)
#pragma unroll
        for (int c = 0; c < 3; ++c) kin = fma(p.mass[al] * v[al][c], v[al][c], kin);
    S[(int64_t)f * nE + e] -= p.lam[f] * p.rho[e] * kin;
}

// per-workgroup partials of the m x m Gram matrix G[i][j] = A[i] . B[j]
// (deterministic: the host sums the partials in a fixed order)
constexpr int GWG = 256, GNB = 512;
__global__ __launch_bounds__(GWG) void k_gram(int64_t n, int m, const double* A, const double* B, double* part) {
    __shared__ double red[GWG / 64][BLK * BLK];
    double acc[BLK * BLK];
#pragma unroll
    for (int q = 0; q < BLK * BLK; ++q) acc[q] = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)GWG + threadIdx.x; t < n; t += (int64_t)gridDim.x * GWG) {
        double a[BLK], b[BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i) {
            a[i] = i < m ? A[i * n + t] : 0.0;
            b[i] = i < m ? B[i * n + t] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < BLK; ++i)
#pragma unroll
            for (int j = 0; j < BLK; ++j) acc[i * BLK + j] = fma(a[i], b[j], acc[i * BLK + j]);
    }
#pragma unroll
    for (int q = 0; q < BLK * BLK; ++q) {
        double v = acc[q];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < BLK * BLK) {
        double s = 0.0;
        for (int w = 0; w < GWG / 64; ++w) s += red[w][threadIdx.x];
        part[(int64_t)blockIdx.x * BLK * BLK + threadIdx.x] = s;
    }
}

// X[j] = sum_i Y[i] Q[i][j] for the m columns (each thread reads its entries
// of every column before writing, so X may alias Y)
struct LinP {
    int m;
    double Q[BLK][BLK];
};
__global__ void k_lincomb(int64_t n, LinP q, const double* Y, double* X) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        double y[BLK];
#pragma unroll
        for (int i = 0; i < BLK; ++i) y[i] = i < q.m ? Y[i * n + t] : 0.0;
#pragma unroll
        for (int j = 0; j < BLK; ++j) {
            if (j >= q.m) break;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < BLK; ++i) s = fma(y[i], q.Q[i][j], s);
            X[j * n + t] = s;
        }
    }
}

// R[j] = A[j] - th[j] B[j] (the Ritz residual vectors, formed explicitly so
// that their norms do not cancel)
struct ThP {
    double th[BLK];
};
__global__ void k_resid(int64_t n, ThP t, const double* A, const double* B, double* R) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
#pragma unroll
        for (int j = 0; j < BLK; ++j) R[j * n + i] = A[j * n + i] - t.th[j] * B[j * n + i];
}

// deterministic start block: splitmix64 of (column, DOF index) mapped to
// [-1, 1), zero on fixed DOFs
__global__ void k_start_block(int64_t nnode, const uint8_t* nmask, double* X) {
    const int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (n >= nnode) return;
    const int col = blockIdx.y;
    const uint8_t mk = nmask[n];
    for (int c = 0; c < 3; ++c) {
        uint64_t z = (uint64_t)(3 * n + c) + 0x9E3779B97F4A7C15ull * (uint64_t)(col + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const double v = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
        X[(int64_t)col * 3 * nnode + 3 * n + c] = ((mk >> c) & 1) ? 0.0 : v;
    }
}

// ---- linear buckling (Eq. 3.5) ---------------------------------------
// element centroid stresses sig[6][nE] of a displacement field, zero on the
// ersatz void (scale below 1/2)
struct SigP {
    int nx, ny, nz;
    double inv4h[3];
    double lam, mu;
    const double* U;
    const double* rho;
};
__global__ void k_elem_stress(SigP p, double* sig) {
    const int nE = p.nx * p.ny * p.nz;  // < 2^31 (checked on the host)
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const int ex = e % p.nx, exy = e / p.nx, ey = exy % p.ny, ez = exy / p.ny;
    const int sy = p.nx + 1, sz = (p.nx + 1) * (p.ny + 1);
    double v[8][3];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int64_t nd = (ex + (a & 1)) + sy * (ey + ((a >> 1) & 1)) + (int64_t)sz * (ez + (a >> 2));
#pragma unroll
        for (int c = 0; c < 3; ++c) v[a][c] = p.U[3 * nd + c];
    }
    haar_fwd(v);
    double sg[6];
    const double re = p.rho[e];
    centroid_stress(v, p.inv4h, p.lam, p.mu, re, sg);
    // the ersatz void carries no prebuckling stress
#pragma unroll
    for (int q = 0; q < 6; ++q) sig[(int64_t)q * nE + e] = re < 0.5 ? 0.0 : sg[q];
}

// The geometric stiffness of element e, K_sigma,e[(a,i),(b,j)] = delta_ij
// sum_pq S_pq G^pq_ab, G^pq_ab = int dN_a/dx_p dN_b/dx_q (nodes in binary
// order): with the symmetric stress, w_ab = sum_p S_pp Gd[p]_ab +
// S_yz Go[0]_ab + S_xz Go[1]_ab + S_xy Go[2]_ab, Go = G^pq + G^qp.
struct GeoP {
    int nx, ny, nz;
    int64_t ndof;
    double Gd[3][8][8];
    double Go[3][8][8];
    const double* sig;     // [6][nE]
    const uint8_t* nmask;
};
__device__ __forceinline__ double geo_w(const GeoP& p, const double S[6], int a, int b) {
    return S[0] * p.Gd[0][a][b] + S[1] * p.Gd[1][a][b] + S[2] * p.Gd[2][a][b] + S[3] * p.Go[0][a][b] +
           S[4] * p.Go[1][a][b] + S[5] * p.Go[2][a][b];
}
// Y[r] = scale * K_sigma U[r] on free DOFs (fixed inputs taken as zero), 0 on
// fixed DOFs; one thread per node gathering its elements' rows in a fixed order
__global__ void k_geo_apply(GeoP p, double scale, const double* U, double* Y) {
    const int nx = p.nx, ny = p.ny, nz = p.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1);
    const int nn = sz * (nz + 1);
    const int nE = nx * ny * nz;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const int r = blockIdx.y;
    const double* u = U + (int64_t)r * p.ndof;
    const int i = n % sy, j = (n / sy) % (ny + 1), k = n / sz;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int dz = 0; dz < 2; ++dz) {
        const int ez = k - 1 + dz;
        if (ez < 0 || ez >= nz) continue;
        for (int dy = 0; dy < 2; ++dy) {
            const int ey = j - 1 + dy;
            if (ey < 0 || ey >= ny) continue;
            for (int dx = 0; dx < 2; ++dx) {
                const int ex = i - 1 + dx;
                if (ex < 0 || ex >= nx) continue;
                const int e = ex + nx * (ey + ny * ez);
                const int a = (1 - dx) + 2 * (1 - dy) + 4 * (1 - dz);  // this node's corner of e
                double S[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) S[q] = p.sig[(int64_t)q * nE + e];
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const int m = (ex + (b & 1)) + sy * (ey + ((b >> 1) & 1)) + sz * (ez + (b >> 2));
                    const uint8_t mk = p.nmask[m];
                    const double w = geo_w(p, S, a, b);
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[c] += ((mk >> c) & 1) ? 0.0 : w * u[3 * (int64_t)m + c];
                }
            }
        }
    }
    const uint8_t mk = p.nmask[n];
    double* y = Y + (int64_t)r * p.ndof + 3 * (int64_t)n;
#pragma unroll
    for (int c = 0; c < 3; ++c) y[c] = ((mk >> c) & 1) ? 0.0 : scale * acc[c];
}

// G[f][e] = phi_e^T K_sigma,e phi_e (field f of Phi)
__global__ void k_geo_energy(GeoP p, const double* Phi, double* G) {
    const int nE = p.nx * p.ny * p.nz;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nE) return;
    const int f = blockIdx.y;
    const int ex = e % p.nx, exy = e / p.nx, ey = exy % p.ny, ez = exy / p.ny;
    const int sy = p.nx + 1, sz = (p.nx + 1) * (p.ny + 1);
    const double* ph = Phi + (int64_t)f * p.ndof;
    double v[8][3], S[6];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int64_t nd = (ex + (a & 1)) + sy * (ey + ((a >> 1) & 1)) + (int64_t)sz * (ez + (a >> 2));
#pragma unroll
        for (int c = 0; c < 3; ++c) v[a][c] = ph[3 * nd + c];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) S[q] = p.sig[(int64_t)q * nE + e];
    double acc = 0.0;
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            const double w = geo_w(p, S, a, b);
            acc += w * (v[a][0] * v[b][0] + v[a][1] * v[b][1] + v[a][2] * v[b][2]);
        }
    G[(int64_t)f * nE + e] = acc;
}

// G^pq_ab for the voxel, nodes in binary order
void geo_tables(const double h[3], GeoP& p) {
    auto one = [&](int ax, int p_, int q_, int ia, int ib) {
        const double hh = h[ax];
        if (ax == p_ && ax == q_) return (ia == ib ? 1.0 : -1.0) / hh;              // int phi_a' phi_b'
        if (ax == p_) return (ia == 0 ? -0.5 : 0.5);                                  // int phi_a' phi_b
        if (ax == q_) return (ib == 0 ? -0.5 : 0.5);                                  // int phi_a phi_b'
        return hh * (ia == ib ? 2.0 : 1.0) / 6.0;                                     // int phi_a phi_b
    };
    auto G = [&](int p_, int q_, int a, int b) {
        double v = 1.0;
        for (int ax = 0; ax < 3; ++ax) v *= one(ax, p_, q_, (a >> ax) & 1, (b >> ax) & 1);
        return v;
    };
    const int off[3][2] = {{1, 2}, {0, 2}, {0, 1}};  // yz, xz, xy
    for (int a = 0; a < 8; ++a)
        for (int b = 0; b < 8; ++b) {
            for (int d = 0; d < 3; ++d) p.Gd[d][a][b] = G(d, d, a, b);
            for (int o = 0; o < 3; ++o)
                p.Go[o][a][b] = G(off[o][0], off[o][1], a, b) + G(off[o][1], off[o][0], a, b);
        }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// symmetric eigen-decomposition of a small matrix by cyclic Jacobi rotations:
// A (m x m, destroyed) -> eigenvalues d, eigenvectors V (columns)
void jacobi_eig(int m, double A[BLK][BLK], double d[BLK], double V[BLK][BLK]) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) (i == j ? diag : off) += A[i][j] * A[i][j];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                if (A[p][q] == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {  // A <- J^T A J
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < m; ++i) d[i] = A[i][i];
}

}  // namespace

int mass_apply(const Grid& g, const double h[3], const double* rho, const uint8_t* nmask, int nrhs, const double* U,
               double* Y, hipStream_t s) {
    if (nrhs < 1 || nrhs > 4) {
        set_error("apply_M: nrhs 1..4");
        return AFD_E_INVALID_ARG;
    }
    MassP p;
    p.nx = g.nx, p.ny = g.ny, p.nz = g.nz;
    p.ndof = g.ndof;
    const double vol = h[0] * h[1] * h[2];
    for (int d = 0; d < 4; ++d) p.w[d] = vol * std::pow(1.0 / 3.0, 3 - d) * std::pow(1.0 / 6.0, d);
    p.rho = rho;
    p.nmask = nmask;
    hipLaunchKernelGGL(k_mass_apply, dim3((unsigned)((g.nnode + 255) / 256), nrhs), dim3(256), 0, s, p, U, Y);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

namespace {

// The largest eigenvalues mu of B x = mu K x (K positive definite on the free
// DOFs; B = M for modes, -K_sigma for buckling) by subspace iteration on a
// block of BLK vectors: Z = B X, Y = K^-1 Z (one BLK-column deflated solve,
// warm-started from X mu), Rayleigh-Ritz (Kr = Y^T Z = Y^T K Y, Br = Y^T B Y;
// Kr = L L^T, L^-1 Br L^-T = V diag(mu) V^T, Q = L^-T V), X = Y Q (K-orthonormal),
// until the Ritz residuals ||B x - mu K x|| / (|mu| ||K x||) of the first nev
// pairs (B X = (B Y) Q and K X = Z Q from the solves, formed as vectors) meet
// tol.  X (BLK x n_dof, caller's) holds the Ritz vectors on return, mu the
// Ritz values in descending order.
struct Subspace {
    afd_mesh* mesh;
    int64_t nd;
    hipStream_t s;
    double *Y = nullptr, *Z = nullptr, *W = nullptr, *part = nullptr;
    std::vector<double> hp;
    int alloc() {
        const size_t vec = (size_t)BLK * nd;
        if (afd::dev_malloc((void**)&Y, vec * 8) != hipSuccess || afd::dev_malloc((void**)&Z, vec * 8) != hipSuccess ||
            afd::dev_malloc((void**)&W, vec * 8) != hipSuccess ||
            afd::dev_malloc((void**)&part, (size_t)GNB * BLK * BLK * 8) != hipSuccess) {
            set_error("eigen: out of device memory");
            return AFD_E_OOM;
        }
        hp.resize((size_t)GNB * BLK * BLK);
        return AFD_OK;
    }
    void release() {
        (void)hipStreamSynchronize(s);
        for (double* q : {Y, Z, W, part})
            if (q) (void)afd::dev_free(q);
    }
    int gram(const double* A, const double* B, double G[BLK][BLK]) {
        hipLaunchKernelGGL(k_gram, dim3(GNB), dim3(GWG), 0, s, nd, BLK, A, B, part);
        AFD_HIP_TRY(hipGetLastError());
        AFD_HIP_TRY(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, s));
        AFD_HIP_TRY(hipStreamSynchronize(s));
        for (int q = 0; q < BLK * BLK; ++q) {
            double acc = 0.0;
            for (int b = 0; b < GNB; ++b) acc += hp[(size_t)b * BLK * BLK + q];
            G[q / BLK][q % BLK] = acc;
        }
        return AFD_OK;
    }
    int lincomb(const double* src, const double Q[BLK][BLK], double* dst) {
        LinP lp;
        lp.m = BLK;
        for (int i = 0; i < BLK; ++i)
            for (int j = 0; j < BLK; ++j) lp.Q[i][j] = Q[i][j];
        hipLaunchKernelGGL(k_lincomb, dim3(2048), dim3(256), 0, s, nd, lp, src, dst);
        AFD_HIP_TRY(hipGetLastError());
        return AFD_OK;
    }
    // out[j] = ||A_j - th_j B_j|| / (|th_j| ||B_j||), j < n, the vectors formed in R
    int residuals(const double* A, const double* B, const double* th, double* R, int n, double* out) {
        ThP t;
        for (int j = 0; j < BLK; ++j) t.th[j] = th[j];
        hipLaunchKernelGGL(k_resid, dim3(2048), dim3(256), 0, s, nd, t, A, B, R);
        AFD_HIP_TRY(hipGetLastError());
        double G1[BLK][BLK], G3[BLK][BLK];
        AFD_TRY(gram(R, R, G1));
        AFD_TRY(gram(B, B, G3));
        for (int j = 0; j < n; ++j) out[j] = std::sqrt(G1[j][j]) / (std::fabs(th[j]) * std::sqrt(G3[j][j]));
        return AFD_OK;
    }
};

template <typename ApplyB>
int subspace_largest(Subspace& sp, const Grid& g, const uint8_t* nmask, ApplyB applyB, const afd_solve_opts* inner,
                     int nev, double tol, int max_iter, double* X, double mu[BLK], double res[BLK], int& it, int& cg,
                     bool& conv, const EigenBlock* start, double inexact) {
    hipStream_t s = sp.s;
    const bool warm = start && start->valid;
    if (warm) {  // the block of an earlier run (e.g. of the previous topology of a loop)
        AFD_HIP_TRY(hipMemcpyAsync(X, start->X, (size_t)BLK * g.ndof * 8, hipMemcpyDeviceToDevice, s));
    } else {
        hipLaunchKernelGGL(k_start_block, dim3((unsigned)((g.nnode + 255) / 256), BLK), dim3(256), 0, s, g.nnode,
                           nmask, X);
        AFD_HIP_TRY(hipGetLastError());
    }
    afd_solve_opts so = *inner;
    so.mem_kind = AFD_MEM_DEVICE;
    so.pairs = nullptr;
    so.npairs = 0;
    std::vector<afd_solve_stats> ss(BLK);
    for (int j = 0; j < BLK; ++j) mu[j] = warm ? start->mu[j] : 0.0, res[j] = 1.0;
    it = 0, cg = 0, conv = false;
    while (it < max_iter && !conv) {
        ++it;
        // Z = B X; Y = K^-1 Z, warm-started from X mu (K^-1 B x = mu x for an eigenpair)
        AFD_TRY(applyB(X, sp.Z));
        // inexact inner solves: to `inexact` times the smallest Ritz residual
        // of the wanted pairs so far, never looser than `inexact` nor tighter
        // than the caller's rtol (the residuals are measured with the
        // operators, so the stopping test stays exact)
        double rmin = 1.0;
        for (int j = 0; j < nev; ++j) rmin = std::min(rmin, res[j]);
        so.rtol = std::max(inner->rtol, inexact * rmin);
        if (it > 1 || warm) {
            double D[BLK][BLK] = {};
            for (int j = 0; j < BLK; ++j) D[j][j] = mu[j];
            AFD_TRY(sp.lincomb(X, D, sp.Y));
            so.x0 = sp.Y;
        } else {
            so.x0 = nullptr;
        }
        AFD_TRY(afd_solve(sp.mesh, &so, BLK, sp.Z, sp.Y, nullptr, nullptr, ss.data()));
        for (int j = 0; j < BLK; ++j) cg += ss[j].iterations;
        double Kr[BLK][BLK], Br[BLK][BLK];
        AFD_TRY(sp.gram(sp.Y, sp.Z, Kr));
        AFD_TRY(applyB(sp.Y, sp.W));
        AFD_TRY(sp.gram(sp.Y, sp.W, Br));
        for (int i = 0; i < BLK; ++i)  // symmetric parts (rounding and inexact solves)
            for (int j = i + 1; j < BLK; ++j) {
                Kr[i][j] = Kr[j][i] = 0.5 * (Kr[i][j] + Kr[j][i]);
                Br[i][j] = Br[j][i] = 0.5 * (Br[i][j] + Br[j][i]);
            }
        double L[BLK][BLK] = {};
        for (int j = 0; j < BLK; ++j) {
            double d = Kr[j][j];
            for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
            if (!(d > 0)) {
                set_error("eigen: the subspace lost rank (K-Gram matrix not positive definite)");
                return AFD_E_BREAKDOWN;
            }
            L[j][j] = std::sqrt(d);
            for (int i = j + 1; i < BLK; ++i) {
                double v = Kr[i][j];
                for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
                L[i][j] = v / L[j][j];
            }
        }
        double Li[BLK][BLK] = {};  // L^-1
        for (int j = 0; j < BLK; ++j) {
            Li[j][j] = 1.0 / L[j][j];
            for (int i = j + 1; i < BLK; ++i) {
                double v = 0.0;
                for (int k = j; k < i; ++k) v -= L[i][k] * Li[k][j];
                Li[i][j] = v / L[i][i];
            }
        }
        double C[BLK][BLK], T1[BLK][BLK];
        for (int i = 0; i < BLK; ++i)
            for (int j = 0; j < BLK; ++j) {
                double v = 0.0;
                for (int k = 0; k < BLK; ++k) v += Li[i][k] * Br[k][j];
                T1[i][j] = v;
            }
        for (int i = 0; i < BLK; ++i)
            for (int j = 0; j < BLK; ++j) {
                double v = 0.0;
                for (int k = 0; k < BLK; ++k) v += T1[i][k] * Li[j][k];
                C[i][j] = v;
            }
        double d[BLK], V[BLK][BLK];
        jacobi_eig(BLK, C, d, V);
        int ord[BLK] = {0, 1, 2, 3};
        std::sort(ord, ord + BLK, [&](int a, int b) { return d[a] > d[b]; });
        double Q[BLK][BLK];
        for (int j = 0; j < BLK; ++j) {
            for (int i = 0; i < BLK; ++i) {
                double v = 0.0;
                for (int k = i; k < BLK; ++k) v += Li[k][i] * V[k][ord[j]];  // (L^-T V)[i][j]
                Q[i][j] = v;
            }
            mu[j] = d[ord[j]];
        }
        // X = Y Q; B X = W Q into Y, K X = Z Q into W; residual vectors in Z
        AFD_TRY(sp.lincomb(sp.Y, Q, X));
        AFD_TRY(sp.lincomb(sp.W, Q, sp.Y));
        AFD_TRY(sp.lincomb(sp.Z, Q, sp.W));
        AFD_TRY(sp.residuals(sp.Y, sp.W, mu, sp.Z, nev, res));
        conv = true;
        for (int j = 0; j < nev; ++j) conv = conv && res[j] <= tol;
    }
    return AFD_OK;
}

}  // namespace

int modal_subspace(afd_mesh* mesh, const Grid& g, const double h[3], const double* rho, const uint8_t* nmask,
                   const afd_solve_opts* inner, int nev, double tol, int max_iter, double* lam_out, double* Phi,
                   double* S, afd_modal_stats* st, hipStream_t s, EigenBlock* block) {
    if (nev < 1 || nev > BLK - 1 || !(tol > 0) || max_iter < 1 || !lam_out || !Phi || !inner) {
        set_error("modal: nev 1..3, tol > 0, max_iter >= 1, non-null lambda, Phi, solve options");
        return AFD_E_INVALID_ARG;
    }
    if (g.nelem >= ((int64_t)1 << 31)) {
        set_error("modal: more than 2^31 elements");
        return AFD_E_INVALID_ARG;
    }
    const double t0 = now_s();
    Subspace sp{mesh, g.ndof, s};
    double* X = nullptr;
    int rc = sp.alloc();
    if (rc == AFD_OK && afd::dev_malloc((void**)&X, (size_t)BLK * g.ndof * 8) != hipSuccess) {
        set_error("modal: out of device memory");
        rc = AFD_E_OOM;
    }
    auto done = [&](int code) {
        sp.release();
        if (X) (void)afd::dev_free(X);
        if (st) st->t = now_s() - t0;
        return code;
    };
    if (rc) return done(rc);
    double mu[BLK], res[BLK];
    int it = 0, cg = 0;
    bool conv = false;
    auto applyM = [&](const double* in, double* out) { return mass_apply(g, h, rho, nmask, BLK, in, out, s); };
    // 1e-1: the mass pencil's iteration count does not grow with looser inner
    // solves (128x64x64: 9 subspace iterations at 1e-2 and at 1e-1, 4,256 ->
    // 3,383 CG iterations)
    if ((rc = subspace_largest(sp, g, nmask, applyM, inner, nev, tol, max_iter, X, mu, res, it, cg, conv, block,
                               1e-1)))
        return done(rc);
    if (block && block->X) {  // the K-orthonormal Ritz block and its values, for a later start
        if (hipMemcpyAsync(block->X, X, (size_t)BLK * g.ndof * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            set_error("modal: copy of the Ritz block failed");
            return done(AFD_E_HIP);
        }
        for (int j = 0; j < BLK; ++j) block->mu[j] = mu[j];
        block->valid = true;
    }
    // lambda = 1 / mu; phi = x / sqrt(mu) (M-normalised: x^T M x = mu x^T K x = mu)
    double D[BLK][BLK] = {};
    for (int j = 0; j < BLK; ++j) {
        if (!(mu[j] > 0)) {
            set_error("modal: a non-positive Ritz value (M or K not definite on the free DOFs)");
            return done(AFD_E_BREAKDOWN);
        }
        D[j][j] = 1.0 / std::sqrt(mu[j]);
    }
    double lam[BLK];
    for (int j = 0; j < BLK; ++j) lam[j] = 1.0 / mu[j];
    if ((rc = sp.lincomb(X, D, X))) return done(rc);
    // reported residuals with the operators: ||K phi - lambda M phi|| / (lambda ||M phi||)
    if ((rc = afd_apply_K(mesh, AFD_FP64, BLK, X, sp.Y))) return done(rc);
    if ((rc = mass_apply(g, h, rho, nmask, BLK, X, sp.W, s))) return done(rc);
    if ((rc = sp.residuals(sp.Y, sp.W, lam, sp.Z, nev, res))) return done(rc);
    for (int j = 0; j < nev; ++j) {
        lam_out[j] = lam[j];
        if (st) st->rel_residual[j] = res[j];
    }
    if (hipMemcpyAsync(Phi, X, (size_t)nev * g.ndof * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("modal: copy failed");
        return done(AFD_E_HIP);
    }
    if (S) {  // T_lambda(e) = rho_e phi_e^T (K_e - lambda M_e) phi_e
        if ((rc = afd_sensitivity(mesh, nev, X, 0, nullptr, S))) return done(rc);
        KinP kp;
        memset(&kp, 0, sizeof(kp));
        kp.nx = g.nx, kp.ny = g.ny, kp.nz = g.nz;
        kp.ndof = g.ndof;
        kp.nf = nev;
        for (int j = 0; j < nev; ++j) kp.lam[j] = lam[j];
        for (int al = 0; al < 8; ++al) {
            double m = 1.0;
            for (int ax = 0; ax < 3; ++ax) m *= h[ax] * (((al >> ax) & 1) ? 1.0 / 12.0 : 0.25);
            kp.mass[al] = m;
        }
        kp.Phi = X;
        kp.rho = rho;
        hipLaunchKernelGGL(k_kinetic, dim3((unsigned)((g.nelem + 255) / 256), nev), dim3(256), 0, s, kp, S);
        if (hipGetLastError() != hipSuccess) {
            set_error("modal: sensitivity kernel failed");
            return done(AFD_E_HIP);
        }
    }
    if (st) {
        st->iterations = it;
        st->cg_iterations = cg;
        st->converged = conv ? 1 : 0;
    }
    if (!conv) {
        set_error("modal: the Ritz residuals did not meet tol within max_iter");
        return done(AFD_E_NOT_CONVERGED);
    }
    return done(AFD_OK);
}

int geo_apply(const Grid& g, const double h[3], double E, double nu, const double* rho, const uint8_t* nmask,
              const double* U0, int nrhs, const double* X, double* Y, hipStream_t s) {
    if (nrhs < 1 || nrhs > BLK || !U0 || !X || !Y) {
        set_error("apply_Kg: nrhs 1..4 and non-null U0, X, Y");
        return AFD_E_INVALID_ARG;
    }
    if (g.nelem >= ((int64_t)1 << 31)) {
        set_error("apply_Kg: more than 2^31 elements");
        return AFD_E_INVALID_ARG;
    }
    double* sig = nullptr;
    if (afd::dev_malloc((void**)&sig, (size_t)6 * g.nelem * 8) != hipSuccess) {
        set_error("apply_Kg: out of device memory");
        return AFD_E_OOM;
    }
    SigP sp6;
    sp6.nx = g.nx, sp6.ny = g.ny, sp6.nz = g.nz;
    for (int a = 0; a < 3; ++a) sp6.inv4h[a] = 1.0 / (4.0 * h[a]);
    sp6.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    sp6.mu = E / (2.0 * (1.0 + nu));
    sp6.U = U0;
    sp6.rho = rho;
    hipLaunchKernelGGL(k_elem_stress, dim3((unsigned)((g.nelem + 255) / 256)), dim3(256), 0, s, sp6, sig);
    GeoP gp;
    memset(&gp, 0, sizeof(gp));
    gp.nx = g.nx, gp.ny = g.ny, gp.nz = g.nz;
    gp.ndof = g.ndof;
    geo_tables(h, gp);
    gp.sig = sig;
    gp.nmask = nmask;
    hipLaunchKernelGGL(k_geo_apply, dim3((unsigned)((g.nnode + 255) / 256), nrhs), dim3(256), 0, s, gp, 1.0, X, Y);
    const hipError_t e = hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)afd::dev_free(sig);
    if (e != hipSuccess) {
        set_error("apply_Kg: kernel launch failed");
        return AFD_E_HIP;
    }
    return AFD_OK;
}

int buckling_subspace(afd_mesh* mesh, const Grid& g, const double h[3], double E, double nu, const double* rho,
                      const uint8_t* nmask, const double* U, const afd_solve_opts* inner, int nev, double tol,
                      int max_iter, double* lam_out, double* Phi, double* S, afd_modal_stats* st, hipStream_t s,
                      EigenBlock* block) {
    if (nev < 1 || nev > BLK - 1 || !(tol > 0) || max_iter < 1 || !lam_out || !Phi || !inner || !U) {
        set_error("buckling: nev 1..3, tol > 0, max_iter >= 1, non-null U, lambda, Phi, solve options");
        return AFD_E_INVALID_ARG;
    }
    if (g.nelem >= ((int64_t)1 << 31)) {
        set_error("buckling: more than 2^31 elements");
        return AFD_E_INVALID_ARG;
    }
    const double t0 = now_s();
    Subspace sp{mesh, g.ndof, s};
    double *X = nullptr, *sig = nullptr, *Gf = nullptr;
    int rc = sp.alloc();
    if (rc == AFD_OK && (afd::dev_malloc((void**)&X, (size_t)BLK * g.ndof * 8) != hipSuccess ||
                         afd::dev_malloc((void**)&sig, (size_t)6 * g.nelem * 8) != hipSuccess ||
                         (S && afd::dev_malloc((void**)&Gf, (size_t)nev * g.nelem * 8) != hipSuccess))) {
        set_error("buckling: out of device memory");
        rc = AFD_E_OOM;
    }
    auto done = [&](int code) {
        sp.release();
        for (double* q : {X, sig, Gf})
            if (q) (void)afd::dev_free(q);
        if (st) st->t = now_s() - t0;
        return code;
    };
    if (rc) return done(rc);
    // the prebuckling stresses, one per element (centroid)
    SigP sp6;
    sp6.nx = g.nx, sp6.ny = g.ny, sp6.nz = g.nz;
    for (int a = 0; a < 3; ++a) sp6.inv4h[a] = 1.0 / (4.0 * h[a]);
    sp6.lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    sp6.mu = E / (2.0 * (1.0 + nu));
    sp6.U = U;
    sp6.rho = rho;
    hipLaunchKernelGGL(k_elem_stress, dim3((unsigned)((g.nelem + 255) / 256)), dim3(256), 0, s, sp6, sig);
    GeoP gp;
    memset(&gp, 0, sizeof(gp));
    gp.nx = g.nx, gp.ny = g.ny, gp.nz = g.nz;
    gp.ndof = g.ndof;
    geo_tables(h, gp);
    gp.sig = sig;
    gp.nmask = nmask;
    const unsigned nb = (unsigned)((g.nnode + 255) / 256);
    auto applyNegKg = [&](const double* in, double* out) -> int {
        hipLaunchKernelGGL(k_geo_apply, dim3(nb, BLK), dim3(256), 0, s, gp, -1.0, in, out);
        AFD_HIP_TRY(hipGetLastError());
        return AFD_OK;
    };
    double mu[BLK], res[BLK];
    int it = 0, cg = 0;
    bool conv = false;
    // 1e-2: looser inner solves cost the buckling pencil more subspace
    // iterations than they save (128x64x64: 41 at 1e-2, 47 at 3e-2, 49 at 1e-1)
    if ((rc = subspace_largest(sp, g, nmask, applyNegKg, inner, nev, tol, max_iter, X, mu, res, it, cg, conv,
                               block, 1e-2)))
        return done(rc);
    if (block && block->X) {  // the K-orthonormal Ritz block and its values, for a later start
        if (hipMemcpyAsync(block->X, X, (size_t)BLK * g.ndof * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
            set_error("buckling: copy of the Ritz block failed");
            return done(AFD_E_HIP);
        }
        for (int j = 0; j < BLK; ++j) block->mu[j] = mu[j];
        block->valid = true;
    }
    double lam[BLK] = {0, 0, 0, 0};
    for (int j = 0; j < nev; ++j) {
        if (!(mu[j] > 0)) {
            set_error("buckling: fewer positive load factors than requested (the loads put too little in compression)");
            return done(AFD_E_BREAKDOWN);
        }
        lam[j] = 1.0 / mu[j];
    }
    // reported residuals: ||K phi + lambda K_sigma phi|| / ||K phi|| (phi^T K phi = 1)
    if ((rc = afd_apply_K(mesh, AFD_FP64, BLK, X, sp.Y))) return done(rc);
    if ((rc = applyNegKg(X, sp.W))) return done(rc);
    for (int j = 0; j < nev; ++j) {
        lam_out[j] = lam[j];
    }
    if ((rc = sp.residuals(sp.W, sp.Y, mu, sp.Z, nev, res))) return done(rc);
    if (st)
        for (int j = 0; j < nev; ++j) st->rel_residual[j] = res[j];
    if (hipMemcpyAsync(Phi, X, (size_t)nev * g.ndof * 8, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("buckling: copy failed");
        return done(AFD_E_HIP);
    }
    if (S) {  // T_P(e) = lambda phi_e^T (rho_e K_e + lambda K_sigma,e) phi_e
        if ((rc = afd_sensitivity(mesh, nev, X, 0, nullptr, S))) return done(rc);
        hipLaunchKernelGGL(k_geo_energy, dim3((unsigned)((g.nelem + 255) / 256), nev), dim3(256), 0, s, gp, X, Gf);
        AFD_HIP_TRY(hipGetLastError());
        for (int j = 0; j < nev; ++j) {
            const double* grp[2] = {S + (size_t)j * g.nelem, Gf + (size_t)j * g.nelem};
            const int rows[2] = {1, 1};
            const double coef[2] = {lam[j], lam[j] * lam[j]};
            if ((rc = launch_combine(g.nelem, 2, grp, rows, coef, S + (size_t)j * g.nelem, s))) return done(rc);
        }
    }
    if (st) {
        st->iterations = it;
        st->cg_iterations = cg;
        st->converged = conv ? 1 : 0;
    }
    if (!conv) {
        set_error("buckling: the Ritz residuals did not meet tol within max_iter");
        return done(AFD_E_NOT_CONVERGED);
    }
    return done(AFD_OK);
}

}  // namespace afd
