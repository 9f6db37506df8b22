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

int modal_subspace(afd_mesh* mesh, const Grid& g, const double h[3], const double* rho, const uint8_t* nmask,
                   const afd_solve_opts* inner, int nev, double tol, int max_iter, double* lam_out, double* Phi,
                   double* S, afd_modal_stats* st, hipStream_t s) {
    if (nev < 1 || nev > BLK - 1 || !(tol > 0) || max_iter < 1 || !lam_out || !Phi || !inner) {
        set_error("modal: nev 1..3, tol > 0, max_iter >= 1, non-null lambda, Phi, solve options");
        return AFD_E_INVALID_ARG;
    }
    if (g.nelem >= ((int64_t)1 << 31)) {
        set_error("modal: more than 2^31 elements");
        return AFD_E_INVALID_ARG;
    }
    const double t0 = now_s();
    const int64_t nd = g.ndof;
    double *X = nullptr, *Y = nullptr, *Zk = nullptr, *Zm = nullptr, *part = nullptr;
    const size_t vec = (size_t)BLK * nd;
    if (hipMalloc((void**)&X, vec * 8) != hipSuccess || hipMalloc((void**)&Y, vec * 8) != hipSuccess ||
        hipMalloc((void**)&Zk, vec * 8) != hipSuccess || hipMalloc((void**)&Zm, vec * 8) != hipSuccess ||
        hipMalloc((void**)&part, (size_t)GNB * BLK * BLK * 8) != hipSuccess) {
        for (double* q : {X, Y, Zk, Zm, part})
            if (q) (void)hipFree(q);
        set_error("modal: out of device memory");
        return AFD_E_OOM;
    }
    int rc = AFD_OK;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);
        for (double* q : {X, Y, Zk, Zm, part}) (void)hipFree(q);
        if (st) st->t = now_s() - t0;
        return code;
    };
    std::vector<double> hp((size_t)GNB * BLK * BLK);
    auto gram = [&](const double* A, const double* B, double G[BLK][BLK]) -> int {
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
    };
    auto lincomb = [&](const double* src, const double Q[BLK][BLK], double* dst) -> int {
        LinP lp;
        lp.m = BLK;
        for (int i = 0; i < BLK; ++i)
            for (int j = 0; j < BLK; ++j) lp.Q[i][j] = Q[i][j];
        hipLaunchKernelGGL(k_lincomb, dim3(2048), dim3(256), 0, s, nd, lp, src, dst);
        AFD_HIP_TRY(hipGetLastError());
        return AFD_OK;
    };
    // ||A_j - theta_j B_j|| / (theta_j ||B_j||) for the first nev columns, the
    // residual vectors formed in R
    auto residuals = [&](const double* A, const double* B, const double* th, double* R, double* out) -> int {
        ThP t;
        for (int j = 0; j < BLK; ++j) t.th[j] = th[j];
        hipLaunchKernelGGL(k_resid, dim3(2048), dim3(256), 0, s, nd, t, A, B, R);
        AFD_HIP_TRY(hipGetLastError());
        double G1[BLK][BLK], G3[BLK][BLK];
        AFD_TRY(gram(R, R, G1));
        AFD_TRY(gram(B, B, G3));
        for (int j = 0; j < nev; ++j) out[j] = std::sqrt(G1[j][j]) / (std::fabs(th[j]) * std::sqrt(G3[j][j]));
        return AFD_OK;
    };
    hipLaunchKernelGGL(k_start_block, dim3((unsigned)((g.nnode + 255) / 256), BLK), dim3(256), 0, s, g.nnode, nmask,
                       X);
    if (hipGetLastError() != hipSuccess) {
        set_error("modal: start block kernel failed");
        return done(AFD_E_HIP);
    }
    afd_solve_opts so = *inner;
    so.mem_kind = AFD_MEM_DEVICE;
    so.pairs = nullptr;
    so.npairs = 0;
    std::vector<afd_solve_stats> ss(BLK);
    double theta[BLK] = {0, 0, 0, 0}, res[BLK] = {1, 1, 1, 1};
    int it = 0, cg = 0;
    bool conv = false;
    while (it < max_iter && !conv) {
        ++it;
        // Zk = M X; Y = K^-1 Zk, warm-started from X / theta (K^-1 M x = x / lambda for an eigenpair)
        if ((rc = mass_apply(g, h, rho, nmask, BLK, X, Zk, s))) return done(rc);
        if (it > 1) {
            double D[BLK][BLK] = {};
            for (int j = 0; j < BLK; ++j) D[j][j] = theta[j] > 0 ? 1.0 / theta[j] : 0.0;
            if ((rc = lincomb(X, D, Y))) return done(rc);
            so.x0 = Y;
        } else {
            so.x0 = nullptr;
        }
        if ((rc = afd_solve(mesh, &so, BLK, Zk, Y, nullptr, nullptr, ss.data()))) return done(rc);
        for (int j = 0; j < BLK; ++j) cg += ss[j].iterations;
        // Rayleigh-Ritz: Kr = Y^T K Y = Y^T Zk, Mr = Y^T M Y = Y^T Zm
        double Kr[BLK][BLK], Mr[BLK][BLK];
        if ((rc = gram(Y, Zk, Kr))) return done(rc);
        if ((rc = mass_apply(g, h, rho, nmask, BLK, Y, Zm, s))) return done(rc);
        if ((rc = gram(Y, Zm, Mr))) return done(rc);
        for (int i = 0; i < BLK; ++i)  // symmetric parts (rounding and inexact solves)
            for (int j = i + 1; j < BLK; ++j) {
                Kr[i][j] = Kr[j][i] = 0.5 * (Kr[i][j] + Kr[j][i]);
                Mr[i][j] = Mr[j][i] = 0.5 * (Mr[i][j] + Mr[j][i]);
            }
        // Mr = L L^T; C = L^-1 Kr L^-T = V diag(theta) V^T; Q = L^-T V (M-orthonormal Ritz vectors)
        double L[BLK][BLK] = {};
        for (int j = 0; j < BLK; ++j) {
            double d = Mr[j][j];
            for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
            if (!(d > 0)) {
                set_error("modal: the subspace lost rank (M-Gram matrix not positive definite)");
                return done(AFD_E_BREAKDOWN);
            }
            L[j][j] = std::sqrt(d);
            for (int i = j + 1; i < BLK; ++i) {
                double v = Mr[i][j];
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
                for (int k = 0; k < BLK; ++k) v += Li[i][k] * Kr[k][j];
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
        std::sort(ord, ord + BLK, [&](int a, int b) { return d[a] < d[b]; });
        double Q[BLK][BLK];
        for (int j = 0; j < BLK; ++j) {
            for (int i = 0; i < BLK; ++i) {
                double v = 0.0;
                for (int k = i; k < BLK; ++k) v += Li[k][i] * V[k][ord[j]];  // (L^-T V)[i][j]
                Q[i][j] = v;
            }
            theta[j] = d[ord[j]];
        }
        // X = Y Q; K X = Zk Q (from the solves) and M X = Zm Q give the Ritz residuals
        if ((rc = lincomb(Y, Q, X)) || (rc = lincomb(Zk, Q, Y)) || (rc = lincomb(Zm, Q, Zk))) return done(rc);
        if ((rc = residuals(Y, Zk, theta, Zm, res))) return done(rc);
        conv = true;
        for (int j = 0; j < nev; ++j) conv = conv && res[j] <= tol;
    }
    // the reported residuals with the operator itself: ||K phi - lambda M phi|| / (lambda ||M phi||)
    if ((rc = afd_apply_K(mesh, AFD_FP64, BLK, X, Y))) return done(rc);
    if ((rc = mass_apply(g, h, rho, nmask, BLK, X, Zk, s))) return done(rc);
    if ((rc = residuals(Y, Zk, theta, Zm, res))) return done(rc);
    for (int j = 0; j < nev; ++j) {
        lam_out[j] = theta[j];
        if (st) st->rel_residual[j] = res[j];
    }
    AFD_HIP_TRY(hipMemcpyAsync(Phi, X, (size_t)nev * nd * 8, hipMemcpyDeviceToDevice, s));
    if (S) {  // T_lambda(e) = rho_e phi_e^T (K_e - lambda M_e) phi_e
        if ((rc = afd_sensitivity(mesh, nev, X, 0, nullptr, S))) return done(rc);
        KinP kp;
        memset(&kp, 0, sizeof(kp));
        kp.nx = g.nx, kp.ny = g.ny, kp.nz = g.nz;
        kp.ndof = nd;
        kp.nf = nev;
        for (int j = 0; j < nev; ++j) kp.lam[j] = theta[j];
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
        set_error("modal: the Ritz values did not settle within max_iter");
        return done(AFD_E_NOT_CONVERGED);
    }
    return done(AFD_OK);
}

}  // namespace afd
