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
// Modes: APPLY (Y = A U) and RESID (R = F - A X, with partial sums of r.M^-1 r
// and r.r).
//
// Kernels (same tiles, element arithmetic and summation order):
//  * k_matvec: register-staged planes, both modes (the residual form, and apply
//    variant 0);
//  * k_apply_tm: plain apply with tile-major densities and fixity words and
//    every input staged by global_load_lds DMA (variants 2 and 3);
//  * k_apply_bl: the same staging by untyped buffer loads, out-of-range lanes
//    reading zero, with partial vmcnt waits (variants 4 and 6; 6 is the
//    default plain apply, and its DOT form is the solver's direction apply).
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "afd_internal.h"
#include "haar_dev.h"

namespace afd {

namespace {

constexpr int TX = 16, TY = 16, NT = TX * TY;  // element tile (threads)
constexpr int PX = TX + 1, PY = TY + 1;        // node plane in LDS
constexpr int PLANE = PX * PY * 3;

enum { APPLY = 0, RESID = 1 };

template <typename T>
struct MvParams {
    int nx, ny, nz;
    int tiles_x, tiles_y, zc, nchunk;
    int ndof;
    const T* rho;
    const uint8_t* nmask;
    const T* U;     // APPLY: input; RESID: X
    T* Y;           // APPLY: output; RESID: R
    const T* F;     // RESID: F
    int variant;             // plain-apply kernel variant
    const T* rho_t;          // tile-major densities (plain apply)
    const uint16_t* fm_t;    // tile-major face fixity words (plain apply)
    const double* rinv;  // per node 1/sum rho (double)
    const float* rinv32;
    CgScalars* sc;
    double* partial;  // [(rhs*2 + which) * npart + i]
    int npart;
};

template <typename T>
__device__ __forceinline__ double rinv_of(const MvParams<T>& P, int node) {
    if constexpr (sizeof(T) == 8) return P.rinv[node];
    else return (double)P.rinv32[node];
}

// 64-bit row shift by one lane inside each 16-lane DPP row (lane 0 of a row
// receives 0: bound_ctrl zeroes reads from outside the row, so the old value
// of the destination needs no initialisation)
__device__ __forceinline__ double dpp_shr1(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x111, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x111, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float dpp_shr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map dispatch index b to a logical tile so that every XCD receives a
// contiguous range of tiles (x-fastest, then y, then z-chunk): neighbouring
// tiles, which re-read each other's halo node planes, then share an L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int x = b % NXCD, k = b / NXCD;
    const int base = nb / NXCD, rem = nb % NXCD;
    return x * base + min(x, rem) + k;
}

constexpr int PNODES = PX * PY;                   // 289 nodes per staged plane
constexpr int NSLOT = (PNODES + NT - 1) / NT;     // 2 node slots per thread

template <typename T, int MODE, bool CUB>
__global__ __launch_bounds__(NT) void k_matvec(MvParams<T> P, KH<T> kh) {
    __shared__ T plane[2][PLANE];
    __shared__ T xch[3][NT];
    __shared__ double red[NT / 64][2];

    const int rhs = blockIdx.y;
    if constexpr (MODE != APPLY) {
        if (P.sc[rhs].done) return;
    }
    const int t = threadIdx.x;
    const int lx = t % TX, ly = t / TX;
    const int L = xcd_tile(blockIdx.x, gridDim.x);
    const int tile = L % (P.tiles_x * P.tiles_y);
    const int chunk = L / (P.tiles_x * P.tiles_y);
    const int X0 = (tile % P.tiles_x) * (TX - 1) - 1;
    const int Y0 = (tile / P.tiles_x) * (TY - 1) - 1;
    const int Z0 = chunk * P.zc;
    const int Z1 = min(Z0 + P.zc, P.nz + 1);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1);
    const int64_t roff = (int64_t)rhs * P.ndof;  // nrhs * ndof may exceed 2^31
    const T* U = P.U + roff;
    T* Y = P.Y + roff;
    const T* F = (MODE != APPLY) ? P.F + roff : nullptr;

    const int gi = X0 + lx, gj = Y0 + ly;  // this thread's element (ex, ey) and owned node (i, j)
    const bool own = lx >= 1 && ly >= 1 && gi <= nx && gj <= ny;
    const bool elem_xy = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
    const int own_node = gi + sy * gj;     // plane offset of the owned node (if own)

    // node slots this thread stages: fixed (i, j), so set up once
    int soff[NSLOT];     // plane offset, -1 outside the mesh / unused
#pragma unroll
    for (int q = 0; q < NSLOT; ++q) {
        const int n = t + q * NT;
        soff[q] = -1;
        if (n < PNODES) {
            const int row = n / PX, li = n - row * PX;
            const int i = X0 + li, j = Y0 + row;
            if (i >= 0 && i <= nx && j >= 0 && j <= ny) soff[q] = i + sy * j;
        }
    }
    // global loads of plane gk into registers (masked)
    auto fetch = [&](int gk, T reg[NSLOT][3]) {
        const bool pv_ok = gk >= 0 && gk <= nz;
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) reg[q][c] = T(0);
            if (soff[q] >= 0 && pv_ok) {
                const int node = soff[q] + sz * gk;
                const int m = P.nmask[node];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T v = U[3 * node + c];
                    reg[q][c] = ((m >> c) & 1) ? T(0) : v;
                }
            }
        }
    };
    auto put = [&](int buf, const T reg[NSLOT][3]) {
#pragma unroll
        for (int q = 0; q < NSLOT; ++q) {
            const int n = t + q * NT;
            if (n < PNODES) {
#pragma unroll
                for (int c = 0; c < 3; ++c) plane[buf][3 * n + c] = reg[q][c];
            }
        }
    };
    auto rho_at = [&](int k) -> T {
        return (elem_xy && k >= 0 && k < nz) ? P.rho[gi + nx * (gj + ny * k)] : T(0);
    };
    // this thread's element face (4 nodes) of plane in buffer b
    auto read_face = [&](int b, T f[4][3]) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int li = lx + (q & 1), lj = ly + (q >> 1);
#pragma unroll
            for (int c = 0; c < 3; ++c) f[q][c] = plane[b][(lj * PX + li) * 3 + c];
        }
    };

    T bf[4][3];                // transformed lower face of the current layer
    T ctop[4][3];              // transformed upper-face output of the previous layer
    double acc0 = 0.0, acc1 = 0.0;
    T reg[NSLOT][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) ctop[q][c] = T(0);

    fetch(Z0 - 1, reg);
    put(0, reg);
    fetch(Z0, reg);
    put(1, reg);
    __syncthreads();
    read_face(0, bf);
    face_fwd<T>(bf);
    T rho_cur = rho_at(Z0 - 1);
    int buf = 1;  // buffer holding plane k+1

    // outputs of plane k are stored after the first barrier of layer k+1, so
    // that the barrier's wait for outstanding memory operations does not
    // wait for stores issued just before it
    T pend[3];
    int pend_a = -1;
    int own_m_next = (own && Z0 - 1 >= 0) ? (int)P.nmask[own_node + sz * (Z0 - 1)] : 0;
    for (int k = Z0 - 1; k < Z1; ++k) {  // element layer k spans node planes k, k+1
        const bool more = k + 2 <= Z1;
        if (more) fetch(k + 2, reg);  // prefetch while this layer computes
        const int own_m = own_m_next;  // fixity of the owned node on plane k
        if (own && k + 1 <= nz) own_m_next = P.nmask[own_node + sz * (k + 1)];
        const T rho_nxt = rho_at(k + 1);
        __syncthreads();  // plane k+1 staged; previous exchange consumed
        if (pend_a >= 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) Y[pend_a + c] = pend[c];
            pend_a = -1;
        }
        T tf[4][3];
        read_face(buf, tf);
        face_fwd<T>(tf);
        T yb[4][3], yt[4][3];
        element_haar<T, CUB>(kh, rho_cur, bf, tf, yb, yt);
        // plane k: lower-face output of layer k plus upper-face output of layer k-1
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                yb[q][c] += ctop[q][c];
                ctop[q][c] = yt[q][c];
                bf[q][c] = tf[q][c];
            }
        face_inv<T>(yb);  // nodal contributions of this element column to its 4 face nodes
        // node (lx, ly) = corner (0,0) of face (lx,ly) + (1,0) of (lx-1,ly)
        //               + (0,1) of (lx,ly-1) + (1,1) of (lx-1,ly-1)
        T s0[3], s1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s0[c] = yb[0][c] + dpp_shr1(yb[1][c]);
            s1[c] = yb[2][c] + dpp_shr1(yb[3][c]);
            xch[c][t] = s1[c];
        }
        __syncthreads();
        if (own && k >= Z0) {  // node plane k is complete
            const int node = own_node + sz * k;
            const int m = own_m;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int a = 3 * node + c;
                const T yv = s0[c] + xch[c][t - TX];
                const bool fx = (m >> c) & 1;
                if constexpr (MODE == APPLY) {
                    pend[c] = fx ? U[a] : yv;
                } else {  // RESID
                    const T rv = fx ? T(0) : (T)(F[a] - yv);
                    pend[c] = rv;
                    const double z = rinv_of(P, node) / (double)kh.kdiag[c] * (double)rv;
                    acc0 += (double)rv * z;
                    acc1 += (double)rv * (double)rv;
                }
            }
            pend_a = 3 * node;
        }
        // stage plane k+2 into the buffer that held plane k (read last layer)
        if (more) put(buf ^ 1, reg);
        buf ^= 1;
        rho_cur = rho_nxt;
    }
    if (pend_a >= 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Y[pend_a + c] = pend[c];
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
            P.partial[(rhs * 2 + 0) * P.npart + blockIdx.x] = s0;
            P.partial[(rhs * 2 + 1) * P.npart + blockIdx.x] = s1;
        }
        // slots beyond this grid (sized for the larger of the FP64/FP32 grids) read as zero
        if (blockIdx.x == 0)
            for (int i = gridDim.x + t; i < P.npart; i += NT) {
                P.partial[(rhs * 2 + 0) * P.npart + i] = 0.0;
                P.partial[(rhs * 2 + 1) * P.npart + i] = 0.0;
            }
    }
}

// ---------------------------------------------------------------------------
// Helpers of the LDS-DMA staged apply below.  Barriers are plain s_barrier
// with explicit waits: a fenced __syncthreads would also wait for the plane
// loads in flight.
template <typename T>
struct DmaShape {
    static constexpr int DW = sizeof(T) / 4;          // dwords per value
    static constexpr int NDW = PLANE * DW;            // dwords per staged plane
    static constexpr int J = (NDW + NT - 1) / NT;     // DMA instructions per wave per plane
    static constexpr int ROWDW = PX * 3 * DW;         // dwords per staged node row
};

__device__ __forceinline__ void wait_all_and_barrier() {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Tile-major side arrays of the plain apply, rebuilt whenever the densities
// or the fixity change: per (tile, element layer) the 16x16 densities of the
// tile's elements, and per (tile, node plane) a 12-bit fixity word for each
// of the 16x16 node positions, bit 3q + c set when component c of face
// corner q (node (lx + (q & 1), ly + (q >> 1))) is fixed.  Entries outside
// the mesh are zero.  Both are contiguous per tile and layer, so the apply
// stages them with aligned LDS DMA instead of many narrow loads.
template <typename T>
__global__ void k_tile_rho(int nx, int ny, int nz, int tiles_x, int ntile, const double* rho, T* out) {
    const int64_t n = (int64_t)ntile * nz * NT;
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n; f += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(f % NT);
        const int64_t r = f / NT;
        const int k = (int)(r % nz), tile = (int)(r / nz);
        const int gi = (tile % tiles_x) * (TX - 1) - 1 + t % TX, gj = (tile / tiles_x) * (TY - 1) - 1 + t / TX;
        T v = T(0);
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) v = (T)rho[gi + (int64_t)nx * (gj + (int64_t)ny * k)];
        out[f] = v;
    }
}
__global__ void k_tile_fmask(int nx, int ny, int nz, int tiles_x, int ntile, const uint8_t* nmask, uint16_t* out) {
    const int64_t n = (int64_t)ntile * (nz + 1) * NT;
    const int64_t sy = nx + 1, sz = (int64_t)(nx + 1) * (ny + 1);
    for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < n; f += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(f % NT);
        const int64_t r = f / NT;
        const int k = (int)(r % (nz + 1)), tile = (int)(r / (nz + 1));
        const int gi = (tile % tiles_x) * (TX - 1) - 1 + t % TX, gj = (tile / tiles_x) * (TY - 1) - 1 + t / TX;
        int word = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = gi + (q & 1), j = gj + (q >> 1);
            if (i >= 0 && i <= nx && j >= 0 && j <= ny) word |= (nmask[i + sy * j + sz * k] & 7) << (3 * q);
        }
        out[f] = (uint16_t)word;
    }
}

// Plain apply with every input staged by LDS DMA.  Same tiles and element
// arithmetic as above; the z march proceeds in steps of D layers: at the top
// of a step the node planes, fixity words and densities needed one step
// later are put in flight (rings of 2D + 1 planes and 2D density layers),
// and one wait + barrier per step lands them.  Staged planes stay raw: each
// thread zeroes the fixed components of its own face after reading it, which
// also hands it the unmasked value of its own node for the identity rows.
// The y exchange of layer k is completed after the barrier at the top of
// layer k + 1, so each layer has a single barrier.  LDS reads are inline
// assembly with their own lgkmcnt wait: the compiler would otherwise put a
// vmcnt(0) before each of them (it cannot tell that the DMAs in flight
// target other ring slots), which would cap the prefetch distance at one
// layer.

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ uint32_t lds_off(const T* p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) T*)p;
}

// Face of a staged plane at LDS byte address a (node (lx, ly); corners
// q = ax + 2 ay, three components; node rows PX * 3 values apart), the
// density at ar and the fixity word at am, with one wait.
__device__ __forceinline__ void lds_face(uint32_t a, uint32_t ar, uint32_t am, double f[4][3], double& rho,
                                         int& fm) {
    dv2 r0, r1, r2, r3, r4, r5;
    double rr;
    uint32_t mm;
    asm volatile(
        "ds_read2_b64 %0, %8 offset1:1\n\t"
        "ds_read2_b64 %1, %8 offset0:2 offset1:3\n\t"
        "ds_read2_b64 %2, %8 offset0:4 offset1:5\n\t"
        "ds_read2_b64 %3, %8 offset0:51 offset1:52\n\t"
        "ds_read2_b64 %4, %8 offset0:53 offset1:54\n\t"
        "ds_read2_b64 %5, %8 offset0:55 offset1:56\n\t"
        "ds_read_b64 %6, %9\n\t"
        "ds_read_u16 %7, %10\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(rr), "=&v"(mm)
        : "v"(a), "v"(ar), "v"(am));
    f[0][0] = r0.x; f[0][1] = r0.y; f[0][2] = r1.x;
    f[1][0] = r1.y; f[1][1] = r2.x; f[1][2] = r2.y;
    f[2][0] = r3.x; f[2][1] = r3.y; f[2][2] = r4.x;
    f[3][0] = r4.y; f[3][1] = r5.x; f[3][2] = r5.y;
    rho = rr;
    fm = (int)mm;
}
__device__ __forceinline__ void lds_face(uint32_t a, uint32_t ar, uint32_t am, float f[4][3], float& rho, int& fm) {
    fv2 r0, r1, r2, r3, r4, r5;
    float rr;
    uint32_t mm;
    asm volatile(
        "ds_read2_b32 %0, %8 offset1:1\n\t"
        "ds_read2_b32 %1, %8 offset0:2 offset1:3\n\t"
        "ds_read2_b32 %2, %8 offset0:4 offset1:5\n\t"
        "ds_read2_b32 %3, %8 offset0:51 offset1:52\n\t"
        "ds_read2_b32 %4, %8 offset0:53 offset1:54\n\t"
        "ds_read2_b32 %5, %8 offset0:55 offset1:56\n\t"
        "ds_read_b32 %6, %9\n\t"
        "ds_read_u16 %7, %10\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(rr), "=&v"(mm)
        : "v"(a), "v"(ar), "v"(am));
    f[0][0] = r0.x; f[0][1] = r0.y; f[0][2] = r1.x;
    f[1][0] = r1.y; f[1][1] = r2.x; f[1][2] = r2.y;
    f[2][0] = r3.x; f[2][1] = r3.y; f[2][2] = r4.x;
    f[3][0] = r4.y; f[3][1] = r5.x; f[3][2] = r5.y;
    rho = rr;
    fm = (int)mm;
}
// bottom face and its fixity only (start of a chunk)
template <typename T>
__device__ __forceinline__ void lds_face0(uint32_t a, uint32_t am, T f[4][3], int& fm) {
    T rho_unused;
    lds_face(a, a, am, f, rho_unused, fm);
}
// lds_face plus, from another staged plane (byte address ab of the same
// node), the three unmasked components of the own node and its fixity word
__device__ __forceinline__ void lds_face_own(uint32_t a, uint32_t ar, uint32_t am, uint32_t ab, uint32_t amb,
                                             double f[4][3], double& rho, int& fm, double own[3], int& fmb) {
    dv2 r0, r1, r2, r3, r4, r5, o01;
    double rr, o2;
    uint32_t mm, mb;
    asm volatile(
        "ds_read2_b64 %0, %11 offset1:1\n\t"
        "ds_read2_b64 %1, %11 offset0:2 offset1:3\n\t"
        "ds_read2_b64 %2, %11 offset0:4 offset1:5\n\t"
        "ds_read2_b64 %3, %11 offset0:51 offset1:52\n\t"
        "ds_read2_b64 %4, %11 offset0:53 offset1:54\n\t"
        "ds_read2_b64 %5, %11 offset0:55 offset1:56\n\t"
        "ds_read_b64 %6, %12\n\t"
        "ds_read_u16 %7, %13\n\t"
        "ds_read2_b64 %8, %14 offset1:1\n\t"
        "ds_read_b64 %9, %14 offset:16\n\t"
        "ds_read_u16 %10, %15\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(rr), "=&v"(mm), "=&v"(o01),
          "=&v"(o2), "=&v"(mb)
        : "v"(a), "v"(ar), "v"(am), "v"(ab), "v"(amb));
    f[0][0] = r0.x; f[0][1] = r0.y; f[0][2] = r1.x;
    f[1][0] = r1.y; f[1][1] = r2.x; f[1][2] = r2.y;
    f[2][0] = r3.x; f[2][1] = r3.y; f[2][2] = r4.x;
    f[3][0] = r4.y; f[3][1] = r5.x; f[3][2] = r5.y;
    rho = rr;
    fm = (int)mm;
    own[0] = o01.x; own[1] = o01.y; own[2] = o2;
    fmb = (int)mb;
}
__device__ __forceinline__ void lds_face_own(uint32_t a, uint32_t ar, uint32_t am, uint32_t ab, uint32_t amb,
                                             float f[4][3], float& rho, int& fm, float own[3], int& fmb) {
    fv2 r0, r1, r2, r3, r4, r5, o01;
    float rr, o2;
    uint32_t mm, mb;
    asm volatile(
        "ds_read2_b32 %0, %11 offset1:1\n\t"
        "ds_read2_b32 %1, %11 offset0:2 offset1:3\n\t"
        "ds_read2_b32 %2, %11 offset0:4 offset1:5\n\t"
        "ds_read2_b32 %3, %11 offset0:51 offset1:52\n\t"
        "ds_read2_b32 %4, %11 offset0:53 offset1:54\n\t"
        "ds_read2_b32 %5, %11 offset0:55 offset1:56\n\t"
        "ds_read_b32 %6, %12\n\t"
        "ds_read_u16 %7, %13\n\t"
        "ds_read2_b32 %8, %14 offset1:1\n\t"
        "ds_read_b32 %9, %14 offset:8\n\t"
        "ds_read_u16 %10, %15\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(rr), "=&v"(mm), "=&v"(o01),
          "=&v"(o2), "=&v"(mb)
        : "v"(a), "v"(ar), "v"(am), "v"(ab), "v"(amb));
    f[0][0] = r0.x; f[0][1] = r0.y; f[0][2] = r1.x;
    f[1][0] = r1.y; f[1][1] = r2.x; f[1][2] = r2.y;
    f[2][0] = r3.x; f[2][1] = r3.y; f[2][2] = r4.x;
    f[3][0] = r4.y; f[3][1] = r5.x; f[3][2] = r5.y;
    rho = rr;
    fm = (int)mm;
    own[0] = o01.x; own[1] = o01.y; own[2] = o2;
    fmb = (int)mb;
}
// three components of one exchange slot: [c][NT] layout, a = slot of c = 0
__device__ __forceinline__ void lds_xch(uint32_t a, double x[3]) {
    dv2 r01;
    double r2;
    asm volatile(
        "ds_read2st64_b64 %0, %2 offset1:4\n\t"
        "ds_read_b64 %1, %2 offset:4096\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r01), "=&v"(r2)
        : "v"(a));
    x[0] = r01.x;
    x[1] = r01.y;
    x[2] = r2;
}
__device__ __forceinline__ void lds_xch(uint32_t a, float x[3]) {
    fv2 r01;
    float r2;
    asm volatile(
        "ds_read2st64_b32 %0, %2 offset1:4\n\t"
        "ds_read_b32 %1, %2 offset:2048\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r01), "=&v"(r2)
        : "v"(a));
    x[0] = r01.x;
    x[1] = r01.y;
    x[2] = r2;
}
static_assert(PX * 3 == 51 && NT == 256, "assembly offsets assume 17-node rows and 256-slot exchange planes");
// write the three components of this thread's exchange slot ([c][NT]
// layout, a = slot of c = 0).  Assembly, so that the compiler, which cannot
// tell the exchange planes from the targets of buffer-load DMAs in flight,
// does not put a vmcnt wait in front of it.
__device__ __forceinline__ void lds_xch_put(uint32_t a, double x0, double x1, double x2) {
    asm volatile(
        "ds_write2st64_b64 %0, %1, %2 offset1:4\n\t"
        "ds_write_b64 %0, %3 offset:4096"
        :
        : "v"(a), "v"(x0), "v"(x1), "v"(x2)
        : "memory");
}
__device__ __forceinline__ void lds_xch_put(uint32_t a, float x0, float x1, float x2) {
    asm volatile(
        "ds_write2st64_b32 %0, %1, %2 offset1:4\n\t"
        "ds_write_b32 %0, %3 offset:2048"
        :
        : "v"(a), "v"(x0), "v"(x1), "v"(x2)
        : "memory");
}


// DOT: also the per-workgroup partial of P.Q over owned nodes (slot 0 of
// this right-hand side; unused slots zeroed by workgroup 0), and converged
// right-hand sides skipped (the solver's direction apply)
template <typename T, bool CUB, int D, bool DOT = false>
__global__ __launch_bounds__(NT) void k_apply_tm(MvParams<T> P, KH<T> kh) {
    using S = DmaShape<T>;
    constexpr int R = 2 * D + 1;   // node-plane slots: D + 1 in use, D in flight
    constexpr int RR = 2 * D;      // density-layer slots
    __shared__ __attribute__((aligned(16))) T ring[R][PLANE];
    __shared__ __attribute__((aligned(16))) T rring[RR][NT];
    __shared__ __attribute__((aligned(16))) uint16_t mring[R][NT];
    __shared__ __attribute__((aligned(16))) T xch[2][3][NT];
    __shared__ double dred[NT / 64];

    const int rhs = blockIdx.y;
    if constexpr (DOT) {
        if (P.sc[rhs].done) return;
    }
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    const int lx = t % TX, ly = t / TX;
    const int L = xcd_tile(blockIdx.x, gridDim.x);
    const int ntile = P.tiles_x * P.tiles_y;
    const int tile = L % ntile;
    const int chunk = L / ntile;
    const int X0 = (tile % P.tiles_x) * (TX - 1) - 1;
    const int Y0 = (tile / P.tiles_x) * (TY - 1) - 1;
    const int Z0 = chunk * P.zc;
    const int Z1 = min(Z0 + P.zc, P.nz + 1);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1);
    const int64_t roff = (int64_t)rhs * P.ndof;  // nrhs * ndof may exceed 2^31
    const T* U = P.U + roff;
    T* Y = P.Y + roff;
    const uint32_t* Udw = reinterpret_cast<const uint32_t*>(U);
    const uint32_t* Rdw = reinterpret_cast<const uint32_t*>(P.rho_t) + (size_t)tile * nz * NT * S::DW;
    const uint32_t* Mdw = reinterpret_cast<const uint32_t*>(P.fm_t) + (size_t)tile * (nz + 1) * (NT / 2);

    const int gi = X0 + lx, gj = Y0 + ly;
    const bool own = lx >= 1 && ly >= 1 && gi <= nx && gj <= ny;
    const int own_node = gi + sy * gj;

    int goff[S::J];  // node-plane DMA plan: instruction j of wave w moves dwords (4j + w) * 64 + lane
#pragma unroll
    for (int j = 0; j < S::J; ++j) {
        const int f = (4 * j + w) * 64 + lane;
        goff[j] = -1;
        if (f < S::NDW) {
            const int row = f / S::ROWDW, c = f - row * S::ROWDW;
            const int i = X0 + c / (3 * S::DW), jj = Y0 + row;
            if (i >= 0 && i <= nx && jj >= 0 && jj <= ny) goff[j] = (X0 + sy * jj) * 3 * S::DW + c;
        }
    }
    const int kfirst = Z0 - 1;
    auto pslot = [&](int g) { return (g - kfirst) % R; };
    auto rslot = [&](int k) { return (k - kfirst) % RR; };
    auto issue_plane = [&](int g) {  // node plane g and its fixity words
        uint32_t* dst = reinterpret_cast<uint32_t*>(&ring[pslot(g)][0]);
        uint32_t* mdst = reinterpret_cast<uint32_t*>(&mring[pslot(g)][0]);
        if (g >= 0 && g <= nz) {
            const int base = g * sz * 3 * S::DW;
#pragma unroll
            for (int j = 0; j < S::J; ++j) {
                if (goff[j] >= 0)
                    __builtin_amdgcn_global_load_lds(
                        (const void*)(Udw + base + goff[j]),
                        (__attribute__((address_space(3))) void*)(dst + (4 * j + w) * 64), 4, 0, 0);
            }
            if (w < 2)
                __builtin_amdgcn_global_load_lds((const void*)(Mdw + g * (NT / 2) + t),
                                                 (__attribute__((address_space(3))) void*)(mdst + w * 64), 4, 0, 0);
        } else {
            for (int f = t; f < S::NDW; f += NT) dst[f] = 0u;
            if (t < NT / 2) mdst[t] = 0u;
        }
    };
    auto issue_rho = [&](int k) {  // density layer k
        uint32_t* dst = reinterpret_cast<uint32_t*>(&rring[rslot(k)][0]);
        if (k >= 0 && k < nz) {
#pragma unroll
            for (int j = 0; j < S::DW; ++j)
                __builtin_amdgcn_global_load_lds((const void*)(Rdw + (size_t)k * NT * S::DW + (4 * j + w) * 64 + lane),
                                                 (__attribute__((address_space(3))) void*)(dst + (4 * j + w) * 64), 4,
                                                 0, 0);
        } else {
#pragma unroll
            for (int j = 0; j < S::DW; ++j) dst[j * NT + t] = 0u;
        }
    };
    // zero the fixed components of a face (bit 3q + c of fm); a wave-uniform
    // branch, so that the many waves without any fixed face node skip it
    auto mask_face = [&](int fm, T f[4][3]) {
        if (__builtin_amdgcn_ballot_w64(fm != 0)) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if ((fm >> (3 * q + c)) & 1) f[q][c] = T(0);
        }
    };
    const uint32_t face_off = (uint32_t)((ly * PX + lx) * 3 * sizeof(T));
    const uint32_t ring_base = lds_off(&ring[0][0]) + face_off;
    const uint32_t rring_base = lds_off(&rring[0][0]) + (uint32_t)(t * sizeof(T));
    const uint32_t mring_base = lds_off(&mring[0][0]) + (uint32_t)(t * 2);
    const uint32_t xch_base = lds_off(&xch[0][0][0]) + (uint32_t)(max(t - TX, 0) * sizeof(T));
    constexpr uint32_t PLANE_B = PLANE * sizeof(T), RL_B = NT * sizeof(T), ML_B = NT * 2, XB_B = 3 * NT * sizeof(T);

    for (int f = t; f < R * PLANE; f += NT) (&ring[0][0])[f] = T(0);
    lds_barrier();

    // prologue: planes kfirst .. kfirst + D, densities of layers kfirst .. kfirst + D - 1
#pragma unroll
    for (int j = 0; j <= D; ++j)
        if (kfirst + j <= Z1) issue_plane(kfirst + j);
#pragma unroll
    for (int d = 0; d < D; ++d) issue_rho(kfirst + d);
    wait_all_and_barrier();

    T bf[4][3], ctop[4][3];
    int fm0;
    lds_face0<T>(ring_base + pslot(kfirst) * PLANE_B, mring_base + pslot(kfirst) * ML_B, bf, fm0);
    mask_face(fm0, bf);
    face_fwd<T>(bf);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) ctop[q][c] = T(0);
    T rawb[3] = {T(0), T(0), T(0)};  // unmasked own-node values of the bottom plane
    int mownb = 0;                    // and their fixity bits
    T pend[3] = {T(0), T(0), T(0)};   // plane k - 1 output before the y exchange
    T pin[3] = {T(0), T(0), T(0)};    // DOT: the input at that node
    int pend_m = 0, pend_a = -1, pend_x = 0;
    double dot = 0.0;

    for (int k0 = kfirst; k0 < Z1; k0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int k = k0 + d;
            if (k < Z1) {
                if (d == 0) wait_all_and_barrier();  // planes k0 + 1 .. k0 + D and their densities landed
                else lds_barrier();
                if (pend_a >= 0) {  // finish plane k - 1 with the row below's exchange
                    T xr[3];
                    lds_xch(xch_base + pend_x * XB_B, xr);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const T yv = ((pend_m >> c) & 1) ? pend[c] : pend[c] + xr[c];
                        Y[pend_a + c] = yv;
                        if constexpr (DOT) dot += (double)pin[c] * (double)yv;
                    }
                    pend_a = -1;
                }
                if (d == 0) {  // next step's planes and densities
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        if (k0 + D + 1 + j <= Z1) issue_plane(k0 + D + 1 + j);
                        if (k0 + D + j < Z1) issue_rho(k0 + D + j);
                    }
                }
                T tf[4][3], rho_k;
                int fmt;
                lds_face(ring_base + pslot(k + 1) * PLANE_B, rring_base + rslot(k) * RL_B,
                         mring_base + pslot(k + 1) * ML_B, tf, rho_k, fmt);
                T rawt[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) rawt[c] = tf[0][c];
                mask_face(fmt, tf);
                face_fwd<T>(tf);
                T yb[4][3], yt[4][3];
                element_haar<T, CUB>(kh, rho_k, bf, tf, yb, yt);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        yb[q][c] += ctop[q][c];
                        ctop[q][c] = yt[q][c];
                        bf[q][c] = tf[q][c];
                    }
                face_inv<T>(yb);
                const int xb = k & 1;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T s0 = yb[0][c] + dpp_shr1(yb[1][c]);
                    xch[xb][c][t] = yb[2][c] + dpp_shr1(yb[3][c]);
                    pend[c] = ((mownb >> c) & 1) ? rawb[c] : s0;
                }
                if (own && k >= Z0) {
                    pend_a = 3 * (own_node + sz * k);
                    pend_m = mownb;
                    pend_x = xb;
                    if constexpr (DOT) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) pin[c] = ((mownb >> c) & 1) ? T(0) : rawb[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) rawb[c] = rawt[c];
                mownb = fmt & 7;
            }
        }
    }
    lds_barrier();
    if (pend_a >= 0) {
        T xr[3];
        lds_xch(xch_base + pend_x * XB_B, xr);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T yv = ((pend_m >> c) & 1) ? pend[c] : pend[c] + xr[c];
            Y[pend_a + c] = yv;
            if constexpr (DOT) dot += (double)pin[c] * (double)yv;
        }
    }
    if constexpr (DOT) {
        // fixed-order workgroup reduction -> one partial per workgroup
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) dot += __shfl_down(dot, off, 64);
        if (lane == 0) dred[w] = dot;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int q = 0; q < NT / 64; ++q) sum += dred[q];
            P.partial[(rhs * 2 + 0) * P.npart + blockIdx.x] = sum;
            P.partial[(rhs * 2 + 1) * P.npart + blockIdx.x] = 0.0;
        }
        if (blockIdx.x == 0)
            for (int i = gridDim.x + t; i < P.npart; i += NT) {
                P.partial[(rhs * 2 + 0) * P.npart + i] = 0.0;
                P.partial[(rhs * 2 + 1) * P.npart + i] = 0.0;
            }
    }
}

// The same apply with the staging issued as untyped buffer loads into LDS.
// A load whose byte offset lies beyond the range of its buffer resource
// returns zero, so every wave issues the same loads for every layer (node
// positions outside the mesh, planes outside the chunk and the pad of a ring
// slot are simply out of range), and each wave knows how many of its loads
// are younger than the plane it needs.  That allows a partial vmcnt wait and
// hence a prefetch distance of DIST layers with one layer per step: at the
// top of layer k the wave waits for the loads of plane k + 1, issued DIST
// layers earlier, while the DIST - 1 younger batches stay in flight.  Vector
// loads return in order; stores in between do not matter, because the wait
// counts only the loads of the younger batches.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ void dma_dword(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t* lds_wave) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_wave, 4, voff, 0, 0,
                                             0);
}
template <int N>
__device__ __forceinline__ void wait_vm_and_barrier() {
    static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
    asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}
constexpr uint32_t OOB = 0x80000000u;  // beyond every buffer range used below

template <typename T, bool CUB, int DIST, bool DOT = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_apply_bl(MvParams<T> P, KH<T> kh) {
    using S = DmaShape<T>;
    // plane ring: planes k and k + 1 being read, DIST in flight; density ring:
    // layer k being read, DIST in flight.  Both are rounded up to 4 slots, so
    // that with the loop below unrolled by 4 every slot is a constant offset.
    constexpr int R = 4;
    constexpr int RR = DIST + 1 <= 2 ? 2 : 4;
    static_assert(DIST + 2 <= R && DIST + 1 <= RR, "ring too small for the prefetch distance");
    constexpr int SLOT = S::J * NT;    // dwords per plane slot (whole-wave DMA, pad included)
    constexpr int NB = S::J + S::DW;   // loads per wave and layer (waves 0 and 1 issue one more)
    __shared__ __attribute__((aligned(16))) uint32_t ring[R][SLOT];
    __shared__ __attribute__((aligned(16))) T rring[RR][NT];
    __shared__ __attribute__((aligned(16))) uint16_t mring[R][NT];
    __shared__ __attribute__((aligned(16))) T xch[2][3][NT];
    __shared__ double dred[NT / 64];

    const int rhs = blockIdx.y;
    if constexpr (DOT) {
        if (P.sc[rhs].done) return;
    }
    const int t = threadIdx.x, lane = t & 63;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int lx = t % TX, ly = t / TX;
    const int L = xcd_tile(blockIdx.x, gridDim.x);
    const int ntile = P.tiles_x * P.tiles_y;
    const int tile = L % ntile;
    const int chunk = L / ntile;
    const int X0 = (tile % P.tiles_x) * (TX - 1) - 1;
    const int Y0 = (tile / P.tiles_x) * (TY - 1) - 1;
    const int Z0 = chunk * P.zc;
    const int Z1 = min(Z0 + P.zc, P.nz + 1);
    const int nx = P.nx, ny = P.ny, nz = P.nz;
    const int sy = nx + 1, sz = (nx + 1) * (ny + 1);
    const int64_t roff = (int64_t)rhs * P.ndof;  // nrhs * ndof may exceed 2^31
    const T* U = P.U + roff;
    T* Y = P.Y + roff;
    const T* Rt = P.rho_t + (size_t)tile * nz * NT;
    const uint16_t* Mt = P.fm_t + (size_t)tile * (nz + 1) * NT;
    const uint32_t plane_bytes = (uint32_t)(3u * (uint32_t)sz * sizeof(T));

    const int gi = X0 + lx, gj = Y0 + ly;
    const bool own = lx >= 1 && ly >= 1 && gi <= nx && gj <= ny;
    const int own_node = gi + sy * gj;

    uint32_t voff[S::J];  // plane DMA: instruction j of wave w moves dword (4j + w) * 64 + lane of the slot
#pragma unroll
    for (int j = 0; j < S::J; ++j) {
        const int f = (4 * j + w) * 64 + lane;
        voff[j] = OOB;
        if (f < S::NDW) {
            const int row = f / S::ROWDW, c = f - row * S::ROWDW;
            const int i = X0 + c / (3 * S::DW), jj = Y0 + row;
            if (i >= 0 && i <= nx && jj >= 0 && jj <= ny) voff[j] = (uint32_t)(((X0 + sy * jj) * 3 * S::DW + c) * 4);
        }
    }
    const int kfirst = Z0 - 1;
    auto slot = [&](int g) { return (g - kfirst) & (R - 1); };  // g >= kfirst
    auto rslot = [&](int k) { return (k - kfirst) & (RR - 1); };
    // node plane g with its fixity words (zeros outside 0..min(nz, Z1))
    auto issue_plane = [&](int g) {
        const bool in = g >= 0 && g <= Z1 && g <= nz;
        const int gc = in ? g : 0;
        const __amdgpu_buffer_rsrc_t ru = raw_rsrc(U + (size_t)gc * sz * 3, in ? plane_bytes : 0u);
        uint32_t* dst = &ring[slot(g)][0] + w * 64;
#pragma unroll
        for (int j = 0; j < S::J; ++j) dma_dword(ru, voff[j], dst + 4 * j * 64);
        if (w < 2) {
            const __amdgpu_buffer_rsrc_t rm = raw_rsrc(Mt + (size_t)gc * NT, in ? NT * 2u : 0u);
            dma_dword(rm, (uint32_t)(t * 4), reinterpret_cast<uint32_t*>(&mring[slot(g)][0]) + w * 64);
        }
    };
    // densities of element layer k (zeros outside 0..min(nz, Z1) - 1)
    auto issue_rho = [&](int k) {
        const bool in = k >= 0 && k < Z1 && k < nz;
        const __amdgpu_buffer_rsrc_t rr = raw_rsrc(Rt + (size_t)(in ? k : 0) * NT, in ? (uint32_t)(NT * sizeof(T)) : 0u);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&rring[rslot(k)][0]) + w * 64;
#pragma unroll
        for (int j = 0; j < S::DW; ++j) dma_dword(rr, (uint32_t)((j * NT + t) * 4), dst + 4 * j * 64);
    };
    auto mask_face = [&](int fm, T f[4][3]) {
        if (__builtin_amdgcn_ballot_w64(fm != 0)) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if ((fm >> (3 * q + c)) & 1) f[q][c] = T(0);
        }
    };
    const uint32_t face_off = (uint32_t)((ly * PX + lx) * 3 * sizeof(T));
    const uint32_t ring_base = lds_off(&ring[0][0]) + face_off;
    const uint32_t rring_base = lds_off(&rring[0][0]) + (uint32_t)(t * sizeof(T));
    const uint32_t mring_base = lds_off(&mring[0][0]) + (uint32_t)(t * 2);
    const uint32_t xch_base = lds_off(&xch[0][0][0]) + (uint32_t)(max(t - TX, 0) * sizeof(T));
    const uint32_t xch_put = lds_off(&xch[0][0][0]) + (uint32_t)(t * sizeof(T));
    constexpr uint32_t PLANE_B = SLOT * 4, RL_B = NT * sizeof(T), ML_B = NT * 2, XB_B = 3 * NT * sizeof(T);

    // prologue: plane kfirst, then DIST batches (plane kfirst + 1 + d, densities kfirst + d)
    issue_plane(kfirst);
#pragma unroll
    for (int d = 0; d < DIST; ++d) {
        issue_plane(kfirst + 1 + d);
        issue_rho(kfirst + d);
    }
    wait_vm_and_barrier<(DIST - 1) * NB>();  // plane kfirst and the first batch landed (read at layer kfirst)

    // state carried from layer k - 1 to layer k, in two alternating sets (the
    // loop below is unrolled by hand so that no registers are copied): the
    // transformed bottom face and the top-face output of layer k - 1.  The
    // unmasked own-node values of the bottom plane and their fixity bits are
    // re-read from its ring slot, which is refilled only at the top of
    // layer k + 1.
    T bfA[4][3], ctA[4][3], bfB[4][3], ctB[4][3];
    int fm0;
    lds_face0<T>(ring_base + slot(kfirst) * PLANE_B, mring_base + slot(kfirst) * ML_B, bfA, fm0);
    mask_face(fm0, bfA);
    face_fwd<T>(bfA);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) ctA[q][c] = T(0);
    T pend[3] = {T(0), T(0), T(0)};   // plane k - 1 output of the own node before the y exchange
    T pin[3] = {T(0), T(0), T(0)};    // DOT: the input at that node (zero where fixed)
    int pend_m = 0;                   // and its fixity bits
    double dot = 0.0;
    // completes the own node of plane g (computed in layer g) with the
    // contribution of the row below (fixed DOFs keep their input value)
    auto finish = [&](int g) {
        T xr[3], yv[3];
        lds_xch(xch_base + (g & 1) * XB_B, xr);
#pragma unroll
        for (int c = 0; c < 3; ++c) yv[c] = pend[c] + xr[c];
        if (__builtin_amdgcn_ballot_w64(pend_m != 0)) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((pend_m >> c) & 1) yv[c] = pend[c];
        }
        T* y = Y + 3 * ((size_t)own_node + (size_t)sz * g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            y[c] = yv[c];
            if constexpr (DOT) dot += (double)pin[c] * (double)yv[c];
        }
    };

    // element layer k: state in (bfc, ctc), state for layer k + 1 out to (bfn, ctn)
    auto layer = [&](int k, const T (&bfc)[4][3], const T (&ctc)[4][3], T (&bfn)[4][3], T (&ctn)[4][3]) {
        // plane k + 1 and densities k landed; every wave is done with layer k - 1
        // (at k = kfirst: with the bottom face, whose slot is refilled next)
        wait_vm_and_barrier<(DIST - 1) * NB>();
        if (own && k - 1 >= Z0) finish(k - 1);  // plane k - 1, with the row below's exchange
        issue_plane(k + 1 + DIST);  // into the slot of plane k - 1, done with before the barrier
        issue_rho(k + DIST);        // into the slot of densities k - 1
        __builtin_amdgcn_s_setprio(0);
        T rho_k, rbc[3];
        int fmt, mbc;
        lds_face_own(ring_base + slot(k + 1) * PLANE_B, rring_base + rslot(k) * RL_B, mring_base + slot(k + 1) * ML_B,
                     ring_base + slot(k) * PLANE_B, mring_base + slot(k) * ML_B, bfn, rho_k, fmt, rbc, mbc);
        mbc &= 7;
        mask_face(fmt, bfn);
        face_fwd<T>(bfn);
        T yb[4][3];
        element_haar<T, CUB>(kh, rho_k, bfc, bfn, yb, ctn);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) yb[q][c] += ctc[q][c];
        face_inv<T>(yb);
        const int xb = k & 1;
        T up[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pend[c] = yb[0][c] + dpp_shr1(yb[1][c]);
            up[c] = yb[2][c] + dpp_shr1(yb[3][c]);
        }
        lds_xch_put(xch_put + xb * XB_B, up[0], up[1], up[2]);
        // from here through the barrier to the next plane's loads this wave
        // goes ahead of the other resident workgroups' arithmetic (measured:
        // 29.4 -> 28.3 us at 192x96x96, 38 -> 34.5 us for 4 right-hand sides
        // at 128x64x64); the priority drops again once the loads are out
        __builtin_amdgcn_s_setprio(1);
        if (__builtin_amdgcn_ballot_w64(mbc != 0)) {  // identity rows of fixed DOFs: the input value
#pragma unroll
            for (int c = 0; c < 3; ++c)
                if ((mbc >> c) & 1) pend[c] = rbc[c];
        }
        pend_m = mbc;
        if constexpr (DOT) {
#pragma unroll
            for (int c = 0; c < 3; ++c) pin[c] = ((mbc >> c) & 1) ? T(0) : rbc[c];
        }
    };
    for (int k = kfirst;; k += 4) {
        layer(k, bfA, ctA, bfB, ctB);
        if (k + 1 >= Z1) break;
        layer(k + 1, bfB, ctB, bfA, ctA);
        if (k + 2 >= Z1) break;
        layer(k + 2, bfA, ctA, bfB, ctB);
        if (k + 3 >= Z1) break;
        layer(k + 3, bfB, ctB, bfA, ctA);
        if (k + 4 >= Z1) break;
    }
    wait_vm_and_barrier<0>();  // the trailing out-of-range batches too, before the LDS is released
    if (own && Z1 - 1 >= Z0) finish(Z1 - 1);
    if constexpr (DOT) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) dot += __shfl_down(dot, off, 64);
        if (lane == 0) dred[w] = dot;
        __syncthreads();
        if (t == 0) {
            double sum = 0.0;
            for (int q = 0; q < NT / 64; ++q) sum += dred[q];
            P.partial[(rhs * 2 + 0) * P.npart + blockIdx.x] = sum;
            P.partial[(rhs * 2 + 1) * P.npart + blockIdx.x] = 0.0;
        }
        if (blockIdx.x == 0)
            for (int i = gridDim.x + t; i < P.npart; i += NT) {
                P.partial[(rhs * 2 + 0) * P.npart + i] = 0.0;
                P.partial[(rhs * 2 + 1) * P.npart + i] = 0.0;
            }
    }
}

// plain-apply kernel: 0 register staging; 2 / 3 the tile-major DMA kernel with
// 1 / 2 layers per step; 4 / 6 the buffer-load kernel with a prefetch distance
// of 2 / 1 layers (6 is the default; the autotuner or afd_mesh_apply_config
// pick another per mesh)
bool valid_variant(int v) { return v == 0 || v == 2 || v == 3 || v == 4 || v == 6; }
constexpr int DEFAULT_VARIANT = 6;
int apply_variant() { return DEFAULT_VARIANT; }
// buffer-load kernels address a node plane with 32-bit byte offsets
template <typename T>
int usable_variant(int v, const Grid& g) {
    if (v >= 4 && (int64_t)3 * (g.nx + 1) * (g.ny + 1) * (int64_t)sizeof(T) >= (int64_t)OOB) return 2;
    return v;
}

template <typename T>
int apply_occupancy(int variant) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (variant) {
        case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_matvec<T, APPLY, true>, NT, 0); break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_apply_tm<T, true, 2>, NT, 0); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_apply_bl<T, true, 2>, NT, 0); break;
        case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_apply_bl<T, true, 1>, NT, 0); break;
        default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_apply_tm<T, true, 1>, NT, 0); break;
    }
    return (e == hipSuccess && n > 0) ? n : 0;
}

int g_slots[8][2];  // resident 256-thread workgroups per (apply variant, FP32) on this device, 0 = unknown

// z-chunking: as many chunks as fit in one round of resident workgroups of
// the given kernel variant, so that no partly filled second round trails the
// launch; at least 4 node planes per chunk.  zc_req > 0 forces the chunk.
// z chunking: by default enough chunks for one round of workgroups over the
// chip, counting the right-hand sides (grid.y) of the launch
void tiling(const Grid& g, int fp32, int variant, int zc_req, int& tx, int& ty, int& zc, int& nchunk, int nrhs = 1) {
    tx = (g.nx + 1 + (TX - 2)) / (TX - 1);  // ceil((nx+1)/15)
    ty = (g.ny + 1 + (TY - 2)) / (TY - 1);
    if (!valid_variant(variant)) variant = apply_variant();
    if (g_slots[variant][fp32] <= 0) {
        int dev = 0, cus = 256, per = fp32 ? 4 : 2;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int n = fp32 ? apply_occupancy<float>(variant) : apply_occupancy<double>(variant);
        if (n > 0) per = n;
        g_slots[variant][fp32] = cus * per;
    }
    const int planes = g.nz + 1;
    if (zc_req > 0) {
        zc = zc_req;
    } else {
        int want = g_slots[variant][fp32] / (tx * ty * std::max(1, nrhs));
        if (want < 1) want = 1;
        const int maxc = (planes + 3) / 4;
        if (want > maxc) want = maxc;
        zc = (planes + want - 1) / want;
    }
    if (zc > planes) zc = planes;
    if (zc < 1) zc = 1;
    nchunk = (planes + zc - 1) / zc;
}

// plain = the plain apply (its kernel variant and chunking may be tuned per
// mesh); the fused solver modes keep the default tiling, which also sizes the
// partial-sum buffers
template <typename T>
MvParams<T> base_params(const MatvecArgs& a, int nrhs, bool plain = false) {
    MvParams<T> p{};
    p.nx = a.g.nx;
    p.ny = a.g.ny;
    p.nz = a.g.nz;
    const int f = sizeof(T) == 4 ? 1 : 0;
    p.variant = usable_variant<T>(plain ? (a.apply_variant[f] >= 0 ? a.apply_variant[f] : apply_variant()) : 0, a.g);
    tiling(a.g, f, plain ? p.variant : -1, plain ? a.apply_zc[f] : 0, p.tiles_x, p.tiles_y, p.zc, p.nchunk, nrhs);
    p.ndof = (int)a.g.ndof;
    if constexpr (sizeof(T) == 8) {
        p.rho = a.rho;
        p.rho_t = a.rho_t;
    } else {
        p.rho = a.rho32;
        p.rho_t = a.rho32_t;
    }
    p.nmask = a.nmask;
    p.fm_t = a.fm_t;
    return p;
}

template <typename T, int MODE>
int launch(const MvParams<T>& p, const KeHaar& khd, int nrhs, hipStream_t s) {
    if (nrhs < 1 || nrhs > 4) {
        set_error("nrhs must be in 1..4");
        return AFD_E_INVALID_ARG;
    }
    dim3 grid(p.tiles_x * p.tiles_y * p.nchunk, nrhs);
    const KH<T> kh = to_kh<T>(khd);
    const bool cub = is_cubic(khd);
    const int v = MODE == APPLY ? p.variant : 0;
    if (v >= 1) {
        switch (v) {
            case 3:
                if (cub) hipLaunchKernelGGL((k_apply_tm<T, true, 2>), grid, dim3(NT), 0, s, p, kh);
                else hipLaunchKernelGGL((k_apply_tm<T, false, 2>), grid, dim3(NT), 0, s, p, kh);
                break;
            case 4:
                if (cub) hipLaunchKernelGGL((k_apply_bl<T, true, 2>), grid, dim3(NT), 0, s, p, kh);
                else hipLaunchKernelGGL((k_apply_bl<T, false, 2>), grid, dim3(NT), 0, s, p, kh);
                break;
            case 6:
                if (cub) hipLaunchKernelGGL((k_apply_bl<T, true, 1>), grid, dim3(NT), 0, s, p, kh);
                else hipLaunchKernelGGL((k_apply_bl<T, false, 1>), grid, dim3(NT), 0, s, p, kh);
                break;
            default:
                if (cub) hipLaunchKernelGGL((k_apply_tm<T, true, 1>), grid, dim3(NT), 0, s, p, kh);
                else hipLaunchKernelGGL((k_apply_tm<T, false, 1>), grid, dim3(NT), 0, s, p, kh);
                break;
        }
    } else if (cub) {
        hipLaunchKernelGGL((k_matvec<T, MODE, true>), grid, dim3(NT), 0, s, p, kh);
    } else {
        hipLaunchKernelGGL((k_matvec<T, MODE, false>), grid, dim3(NT), 0, s, p, kh);
    }
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

}  // namespace

int matvec_num_tiles(const Grid& g) {
    // partial-sum slots: the larger of the FP64 and FP32 grids
    int tx, ty, zc, nc, best = 0;
    for (int f = 0; f < 2; ++f) {
        tiling(g, f, -1, 0, tx, ty, zc, nc);
        best = std::max(best, tx * ty * nc);
    }
    return best;
}

void apply_tiling(const Grid& g, int fp32, int variant, int zc_req, int nrhs, int* zc, int* nchunk) {
    int tx, ty;
    tiling(g, fp32, variant, zc_req, tx, ty, *zc, *nchunk, nrhs);
}

int64_t tile_layout_sizes(const Grid& g, int64_t* nrho) {
    const int tx = (g.nx + 1 + (TX - 2)) / (TX - 1), ty = (g.ny + 1 + (TY - 2)) / (TY - 1);
    if (nrho) *nrho = (int64_t)tx * ty * g.nz * NT;
    return (int64_t)tx * ty * (g.nz + 1) * NT;
}

int launch_tile_rho(const Grid& g, const double* rho, double* rho_t, float* rho32_t, hipStream_t s) {
    const int tx = (g.nx + 1 + (TX - 2)) / (TX - 1), ty = (g.ny + 1 + (TY - 2)) / (TY - 1);
    hipLaunchKernelGGL(k_tile_rho<double>, dim3(2048), dim3(256), 0, s, g.nx, g.ny, g.nz, tx, tx * ty, rho, rho_t);
    hipLaunchKernelGGL(k_tile_rho<float>, dim3(2048), dim3(256), 0, s, g.nx, g.ny, g.nz, tx, tx * ty, rho, rho32_t);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_tile_fmask(const Grid& g, const uint8_t* nmask, uint16_t* fm_t, hipStream_t s) {
    const int tx = (g.nx + 1 + (TX - 2)) / (TX - 1), ty = (g.ny + 1 + (TY - 2)) / (TY - 1);
    hipLaunchKernelGGL(k_tile_fmask, dim3(2048), dim3(256), 0, s, g.nx, g.ny, g.nz, tx, tx * ty, nmask, fm_t);
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_apply(const MatvecArgs& a, const KeHaar& kh, int fp32, int nrhs, const void* U, void* Y,
                 hipStream_t s) {
    if (fp32) {
        MvParams<float> p = base_params<float>(a, nrhs, true);
        p.U = (const float*)U;
        p.Y = (float*)Y;
        return launch<float, APPLY>(p, kh, nrhs, s);
    }
    MvParams<double> p = base_params<double>(a, nrhs, true);
    p.U = (const double*)U;
    p.Y = (double*)Y;
    return launch<double, APPLY>(p, kh, nrhs, s);
}

template <typename T>
static void set_dcg(MvParams<T>& p, const DcgArgs& d) {
    p.rinv = d.rinv;
    p.sc = d.sc;
    p.partial = d.partial;
    p.npart = d.npart;
}

int launch_residual(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, int nrhs, const double* F,
                    const double* X, double* R, hipStream_t s) {
    MvParams<double> p = base_params<double>(a, nrhs);
    set_dcg(p, d);
    p.U = X;
    p.Y = R;
    p.F = F;
    return launch<double, RESID>(p, kh, nrhs, s);
}

template <typename T>
int launch_dot_t(const MatvecArgs& a, const KeHaar& khd, const DcgArgs& d, int nrhs, const T* U, T* Y,
                 hipStream_t s) {
    if (nrhs < 1 || nrhs > 4) {
        set_error("nrhs must be in 1..4");
        return AFD_E_INVALID_ARG;
    }
    MvParams<T> p = base_params<T>(a, nrhs);  // default tiling: the partial-sum buffer is sized for it
    set_dcg(p, d);
    p.U = U;
    p.Y = Y;
    if (p.tiles_x * p.tiles_y * p.nchunk > p.npart) {
        set_error("apply_dot: grid larger than the partial-sum buffer");
        return AFD_E_INVALID_ARG;
    }
    dim3 grid(p.tiles_x * p.tiles_y * p.nchunk, nrhs);
    const KH<T> kh = to_kh<T>(khd);
    const bool cub = is_cubic(khd);
    switch (usable_variant<T>(apply_variant(), a.g)) {  // the staging of the default plain apply
        case 4:
            if (cub) hipLaunchKernelGGL((k_apply_bl<T, true, 2, true>), grid, dim3(NT), 0, s, p, kh);
            else hipLaunchKernelGGL((k_apply_bl<T, false, 2, true>), grid, dim3(NT), 0, s, p, kh);
            break;
        case 6:
            if (cub) hipLaunchKernelGGL((k_apply_bl<T, true, 1, true>), grid, dim3(NT), 0, s, p, kh);
            else hipLaunchKernelGGL((k_apply_bl<T, false, 1, true>), grid, dim3(NT), 0, s, p, kh);
            break;
        default:
            if (cub) hipLaunchKernelGGL((k_apply_tm<T, true, 1, true>), grid, dim3(NT), 0, s, p, kh);
            else hipLaunchKernelGGL((k_apply_tm<T, false, 1, true>), grid, dim3(NT), 0, s, p, kh);
            break;
    }
    AFD_HIP_TRY(hipGetLastError());
    return AFD_OK;
}

int launch_apply_dot(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, int fp32, int nrhs, const void* P,
                     void* Q, hipStream_t s) {
    if (fp32) return launch_dot_t<float>(a, kh, d, nrhs, (const float*)P, (float*)Q, s);
    return launch_dot_t<double>(a, kh, d, nrhs, (const double*)P, (double*)Q, s);
}

int launch_residual_f32(const MatvecArgs& a, const KeHaar& kh, const DcgArgs& d, const float* rinv32, int nrhs,
                        const float* F, const float* X, float* R, hipStream_t s) {
    MvParams<float> p = base_params<float>(a, nrhs);
    set_dcg(p, d);
    p.rinv32 = rinv32;
    p.U = X;
    p.Y = R;
    p.F = F;
    return launch<float, RESID>(p, kh, nrhs, s);
}

}  // namespace afd
