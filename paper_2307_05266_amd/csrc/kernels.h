// HIP kernels (gfx950) for the staggered Stokes Schur-complement solver.
//
// Data layout in HBM (N^3 voxels, x fastest, periodic):
//   cell vectors  : N^3 doubles
//   face vectors  : 3 planes of N^3 doubles, plane c = velocity on the lower
//                   c-faces (between X - e_c and X); inactive faces hold 0
//   code          : one byte per voxel describing its three lower faces:
//                   code = s_x + 6 s_y + 36 s_z, s_c = 0 for an inactive face,
//                   else 1 + t_c with t_c in 0..4 the number of tangential
//                   neighbour faces whose two voxels are both solid, so the
//                   diagonal of A on that face is 5 + s_c = 6 + t_c
//   bits          : remaining-fluid bitmask, 32 voxels per word along x
//   label         : component id per voxel (uint16), only when more than one
//                   component carries flow
//
// Every kernel keeps the invariant "inactive faces and solid cells hold 0",
// so a neighbour that is not an unknown contributes nothing to a stencil.
//
// Sweeps: the box is cut into columns of BX x BY voxels (BX = 64 or 32,
// 256 threads); each block marches a run of z-planes.  Block ids are
// remapped so each of the 8 XCDs (private L2 each) receives a contiguous
// range of columns, which keeps y- and z-neighbour rows in one L2.
//
// Reductions are deterministic: each block writes one partial per quantity,
// the last block to arrive (atomic ticket) adds the partials in block order
// and finishes the scalar recurrences on the device, so inner CG loops run
// without host round trips.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stokes {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 4096;      // partial slots per reduced quantity
constexpr int kMaxParts = 4;          // quantities reduced by one kernel
constexpr int kMaxCompLds = 2048;     // components handled by the projection kernels

struct Sweep {
    int N;
    int bxlog;        // BX = 1 << bxlog, BY = kBlock >> bxlog
    int gx, gy, gz;   // blocks along x, y and z
    int lz;           // z-planes per block
    int nblk;         // gx * gy * gz
};

// Inner CG state, resident in device memory.
struct CgState {
    double rho;       // (r, z)
    double alpha, beta;
    double z0;        // ||z_0||
    double zrel;      // ||z_j|| / ||z_0||
    double dq;        // (d, q)
    double eps;
    int it;           // operator applications so far
    int done;         // 1: stop (converged, capped or broken down)
    int status;       // 0 ok, 1 iteration cap, -4 breakdown
    int maxit;
};

// Reduction scratch shared by the kernels of one context (stream ordered).
struct Reduce {
    double* part;       // [kMaxParts][kMaxBlocks]
    unsigned* ticket;   // arrival counter, returned to 0 by the last block
    double* out;        // [8] results of host-side dots
};

__constant__ double kInvDiagA[6] = {0.0, 1.0 / 6.0, 1.0 / 7.0, 1.0 / 8.0, 1.0 / 9.0, 1.0 / 10.0};

__device__ __forceinline__ int sx_of(int code) { return code % 6; }
__device__ __forceinline__ int sy_of(int code) { return (code / 6) % 6; }
__device__ __forceinline__ int sz_of(int code) { return code / 36; }

__device__ __forceinline__ int xcd_remap(int b, int nblk) {
    if ((nblk & 7) != 0) return b;
    return (b & 7) * (nblk >> 3) + (b >> 3);
}

struct Column {
    int lb;          // logical block id
    int i, j;        // this thread's column
    int k0, k1;      // z-run
    bool valid;
};

__device__ __forceinline__ Column sweep_column(const Sweep& s) {
    Column c;
    c.lb = xcd_remap((int)blockIdx.x, s.nblk);
    const int bx = c.lb % s.gx;
    const int t = c.lb / s.gx;
    const int by = t % s.gy;
    const int bz = t / s.gy;
    c.i = (bx << s.bxlog) + ((int)threadIdx.x & ((1 << s.bxlog) - 1));
    c.j = by * (kBlock >> s.bxlog) + ((int)threadIdx.x >> s.bxlog);
    c.k0 = bz * s.lz;
    c.k1 = min(s.N, c.k0 + s.lz);
    c.valid = c.i < s.N && c.j < s.N;
    return c;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sums of NP values; result valid in thread 0.
template <int NP>
__device__ __forceinline__ void block_sum(double (&v)[NP]) {
    __shared__ double lds[kMaxParts][kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        v[n] = wave_sum(v[n]);
        if (lane == 0) lds[n][w] = v[n];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < NP; ++n) {
            double a = lds[n][0];
            for (int q = 1; q < kWaves; ++q) a += lds[n][q];
            v[n] = a;
        }
    }
    __syncthreads();
}

// Write this block's partials and take a ticket.  Returns true in every
// thread of the last block to arrive; that block then holds the totals
// (added in block order) in v[] of thread 0.
template <int NP>
__device__ __forceinline__ bool reduce_across_blocks(double (&v)[NP], const Reduce& red, int lb, int nblk) {
    __shared__ int am_last;
    block_sum<NP>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < NP; ++n)
            __hip_atomic_store(&red.part[n * kMaxBlocks + lb], v[n], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        unsigned prev = atomicAdd(red.ticket, 1u);
        am_last = (prev == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!am_last) return false;
    __threadfence();
    double acc[NP];
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        acc[n] = 0.0;
        // thread t adds partials t, t + 256, ... in order; then the block tree
        for (int b = threadIdx.x; b < nblk; b += kBlock)
            acc[n] += __hip_atomic_load(&red.part[n * kMaxBlocks + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    block_sum<NP>(acc);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < NP; ++n) v[n] = acc[n];
        __hip_atomic_store(red.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

__device__ __forceinline__ int64_t vidx(int N, int i, int j, int k) {
    return (int64_t)i + (int64_t)N * ((int64_t)j + (int64_t)N * k);
}

// ---------------------------------------------------------------------------
// Setup: face codes from the remaining-fluid bitmask
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fluid_bit(const uint32_t* bits, int N, int wpr, int i, int j, int k) {
    i = (i + N) % N;
    j = (j + N) % N;
    k = (k + N) % N;
    const uint32_t w = bits[((int64_t)k * N + j) * wpr + (i >> 5)];
    return (w >> (i & 31)) & 1;
}

__global__ void k_face_codes(Sweep s, const uint32_t* __restrict__ bits, int wpr, uint8_t* __restrict__ code) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int N = s.N;
    const int i = c.i, j = c.j;
    for (int k = c.k0; k < c.k1; ++k) {
        int sc[3];
        const int me = fluid_bit(bits, N, wpr, i, j, k);
        for (int a = 0; a < 3; ++a) {
            const int di = a == 0, dj = a == 1, dk = a == 2;
            const int lo = fluid_bit(bits, N, wpr, i - di, j - dj, k - dk);
            if (!(me && lo)) { sc[a] = 0; continue; }
            int t = 0;
            for (int b = 0; b < 3; ++b) {
                if (b == a) continue;
                const int ei = b == 0, ej = b == 1, ek = b == 2;
                for (int sg = -1; sg <= 1; sg += 2) {
                    const int f1 = fluid_bit(bits, N, wpr, i + sg * ei, j + sg * ej, k + sg * ek);
                    const int f2 = fluid_bit(bits, N, wpr, i - di + sg * ei, j - dj + sg * ej, k - dk + sg * ek);
                    t += (!f1 && !f2);
                }
            }
            sc[a] = 1 + t;
        }
        code[vidx(N, i, j, k)] = (uint8_t)(sc[0] + 6 * sc[1] + 36 * sc[2]);
    }
}

// ---------------------------------------------------------------------------
// Plain operators (no reductions)
// ---------------------------------------------------------------------------
struct Nbr {
    int64_t X, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nbr neighbours(int N, int i, int j, int k) {
    Nbr n;
    const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
    const int jm = j == 0 ? N - 1 : j - 1, jp = j == N - 1 ? 0 : j + 1;
    const int km = k == 0 ? N - 1 : k - 1, kp = k == N - 1 ? 0 : k + 1;
    n.X = vidx(N, i, j, k);
    n.xm = vidx(N, im, j, k);
    n.xp = vidx(N, ip, j, k);
    n.ym = vidx(N, i, jm, k);
    n.yp = vidx(N, i, jp, k);
    n.zm = vidx(N, i, j, km);
    n.zp = vidx(N, i, j, kp);
    return n;
}

// (A u)_F = (5 + s_F) u_F - sum of the six neighbour faces of the same plane
__device__ __forceinline__ double apply_A_face(const double* __restrict__ u, const Nbr& n, int s) {
    const double nb = u[n.xm] + u[n.xp] + u[n.ym] + u[n.yp] + u[n.zm] + u[n.zp];
    return (double)(5 + s) * u[n.X] - nb;
}

__global__ void k_apply_A(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ u,
                          double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        const int cd = code[n.X];
        const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
        for (int a = 0; a < 3; ++a)
            out[a * n3 + n.X] = sc[a] ? apply_A_face(u + a * n3, n, sc[a]) : 0.0;
    }
}

// (B^T p)(c, X) = p_X - p_{X - e_c} on active faces
__global__ void k_apply_BT(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ p,
                           double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        const int cd = code[n.X];
        const double pX = p[n.X];
        out[n.X] = sx_of(cd) ? pX - p[n.xm] : 0.0;
        out[n3 + n.X] = sy_of(cd) ? pX - p[n.ym] : 0.0;
        out[2 * n3 + n.X] = sz_of(cd) ? pX - p[n.zm] : 0.0;
    }
}

// (B u)_X = sum_c [u(c, X) - u(c, X + e_c)]  (0 in solid cells by the invariant)
// f - B^T p on active faces (right-hand side of the velocity recovery)
__global__ void k_force_minus_BT(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ p, double f0,
                                 double f1, double f2, double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        const int cd = code[n.X];
        const double pX = p[n.X];
        out[n.X] = sx_of(cd) ? f0 - (pX - p[n.xm]) : 0.0;
        out[n3 + n.X] = sy_of(cd) ? f1 - (pX - p[n.ym]) : 0.0;
        out[2 * n3 + n.X] = sz_of(cd) ? f2 - (pX - p[n.zm]) : 0.0;
    }
}

__global__ void k_apply_B(Sweep s, const double* __restrict__ u, double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        out[n.X] = (u[n.X] - u[n.xp]) + (u[n3 + n.X] - u[n3 + n.yp]) + (u[2 * n3 + n.X] - u[2 * n3 + n.zp]);
    }
}

// SIMPLE matrix: (Shat p)_X = sum over active faces F of X of (p_X - p_nbr) / diag(A)_F
__device__ __forceinline__ double apply_Shat_cell(const double* __restrict__ p, const uint8_t* __restrict__ code,
                                                  const Nbr& n, int cdX, double* diag_out) {
    const double pX = p[n.X];
    const int sxl = sx_of(cdX), syl = sy_of(cdX), szl = sz_of(cdX);
    const int sxh = sx_of(code[n.xp]), syh = sy_of(code[n.yp]), szh = sz_of(code[n.zp]);
    const double wxl = kInvDiagA[sxl], wyl = kInvDiagA[syl], wzl = kInvDiagA[szl];
    const double wxh = kInvDiagA[sxh], wyh = kInvDiagA[syh], wzh = kInvDiagA[szh];
    double acc = 0.0;
    acc += wxl * (pX - p[n.xm]);
    acc += wxh * (pX - p[n.xp]);
    acc += wyl * (pX - p[n.ym]);
    acc += wyh * (pX - p[n.yp]);
    acc += wzl * (pX - p[n.zm]);
    acc += wzh * (pX - p[n.zp]);
    if (diag_out) *diag_out = ((wxl + wxh) + (wyl + wyh)) + (wzl + wzh);
    return acc;
}

__device__ __forceinline__ double diag_Shat_cell(const uint8_t* __restrict__ code, const Nbr& n, int cdX) {
    return ((kInvDiagA[sx_of(cdX)] + kInvDiagA[sx_of(code[n.xp])]) +
            (kInvDiagA[sy_of(cdX)] + kInvDiagA[sy_of(code[n.yp])])) +
           (kInvDiagA[sz_of(cdX)] + kInvDiagA[sz_of(code[n.zp])]);
}

__global__ void k_apply_Shat(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ p,
                             double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        out[n.X] = apply_Shat_cell(p, code, n, code[n.X], nullptr);
    }
}

__global__ void k_diag_A(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const int64_t X = vidx(s.N, c.i, c.j, k);
        const int cd = code[X];
        const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
        for (int a = 0; a < 3; ++a) out[a * n3 + X] = sc[a] ? (double)(5 + sc[a]) : 0.0;
    }
}

__global__ void k_diag_Shat(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ out) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        out[n.X] = diag_Shat_cell(code, n, code[n.X]);
    }
}

// zero the entries that are not unknowns (inactive faces / solid cells)
__global__ void k_mask_faces(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ u) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const int64_t X = vidx(s.N, c.i, c.j, k);
        const int cd = code[X];
        if (!sx_of(cd)) u[X] = 0.0;
        if (!sy_of(cd)) u[n3 + X] = 0.0;
        if (!sz_of(cd)) u[2 * n3 + X] = 0.0;
    }
}

__global__ void k_mask_cells(Sweep s, const uint32_t* __restrict__ bits, int wpr, double* __restrict__ p) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        if (!fluid_bit(bits, s.N, wpr, c.i, c.j, k)) p[vidx(s.N, c.i, c.j, k)] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Inner CG with A (faces), Jacobi preconditioner diag(A) = 5 + s
// ---------------------------------------------------------------------------
// x = 0, r = b (b == nullptr: the uniform force on active faces), z = D^-1 r,
// d = z; rho = (r, z), z0 = ||z||.
__global__ void k_cgA_init(Sweep s, const uint8_t* __restrict__ code, const double* b, double f0, double f1,
                           double f2, double* __restrict__ x, double* r, double* __restrict__ d, CgState* st,
                           Reduce red, double eps, int maxit) {
    const Column c = sweep_column(s);
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        const double fc[3] = {f0, f1, f2};
        for (int k = c.k0; k < c.k1; ++k) {
            const int64_t X = vidx(s.N, c.i, c.j, k);
            const int cd = code[X];
            const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t F = a * n3 + X;
                const double bv = sc[a] ? (b ? b[F] : fc[a]) : 0.0;
                const double z = bv * kInvDiagA[sc[a]];
                x[F] = 0.0;
                r[F] = bv;
                d[F] = z;
                acc[0] += bv * z;
                acc[1] += z * z;
            }
        }
    }
    if (reduce_across_blocks<2>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        st->rho = acc[0];
        st->z0 = sqrt(acc[1]);
        st->zrel = 1.0;
        st->alpha = st->beta = st->dq = 0.0;
        st->eps = eps;
        st->maxit = maxit;
        st->it = 0;
        st->status = 0;
        st->done = !(st->z0 > 0.0);
        if (!isfinite(acc[0]) || !isfinite(acc[1])) { st->status = -4; st->done = 1; }
    }
}

// q = A d and (d, q); the last block sets alpha = rho / (d, q)
__global__ void k_cgA_stencil(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ d,
                              double* __restrict__ q, CgState* st, Reduce red) {
    if (st->done) return;
    const Column c = sweep_column(s);
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    double acc[1] = {0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const Nbr n = neighbours(s.N, c.i, c.j, k);
            const int cd = code[n.X];
            const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double* da = d + a * n3;
                const double v = sc[a] ? apply_A_face(da, n, sc[a]) : 0.0;
                q[a * n3 + n.X] = v;
                acc[0] += da[n.X] * v;
            }
        }
    }
    if (reduce_across_blocks<1>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        st->dq = acc[0];
        if (!(acc[0] > 0.0) || !isfinite(acc[0])) {
            st->status = -4;
            st->done = 1;
        } else {
            st->alpha = st->rho / acc[0];
        }
    }
}

// x += alpha d, r -= alpha q, z = D^-1 r; (r, z), ||z||; the last block tests
// ||z|| / ||z0|| < eps and otherwise forms beta = (r, z)_new / (r, z)_old
__global__ void k_cgA_update(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ x,
                             double* __restrict__ r, const double* __restrict__ d, const double* __restrict__ q,
                             CgState* st, Reduce red) {
    if (st->done) return;
    const Column c = sweep_column(s);
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const int64_t X = vidx(s.N, c.i, c.j, k);
            const int cd = code[X];
            const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int64_t F = a * n3 + X;
                x[F] += alpha * d[F];
                const double rn = r[F] - alpha * q[F];
                r[F] = rn;
                const double z = rn * kInvDiagA[sc[a]];
                acc[0] += rn * z;
                acc[1] += z * z;
            }
        }
    }
    if (reduce_across_blocks<2>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        st->it += 1;
        st->zrel = sqrt(acc[1]) / st->z0;
        if (!isfinite(acc[0]) || !isfinite(acc[1])) {
            st->status = -4;
            st->done = 1;
        } else if (st->zrel < st->eps) {
            st->done = 1;
        } else if (st->it >= st->maxit) {
            st->status = 1;
            st->done = 1;
        } else {
            st->beta = acc[0] / st->rho;
            st->rho = acc[0];
        }
    }
}

// d = D^-1 r + beta d
__global__ void k_cgA_dir(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ r,
                          double* __restrict__ d, const CgState* st) {
    if (st->done) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    const double beta = st->beta;
    for (int k = c.k0; k < c.k1; ++k) {
        const int64_t X = vidx(s.N, c.i, c.j, k);
        const int cd = code[X];
        const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int64_t F = a * n3 + X;
            d[F] = r[F] * kInvDiagA[sc[a]] + beta * d[F];
        }
    }
}

// ---------------------------------------------------------------------------
// Inner CG with the SIMPLE matrix (cells), Jacobi preconditioner diag(Shat)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double inv_or_zero(double v) { return v > 0.0 ? 1.0 / v : 0.0; }

__global__ void k_cgS_init(Sweep s, const uint8_t* __restrict__ code, const double* b, double* __restrict__ x,
                           double* r, double* __restrict__ d, CgState* st, Reduce red, double eps, int maxit) {
    const Column c = sweep_column(s);
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const Nbr n = neighbours(s.N, c.i, c.j, k);
            const double bv = b[n.X];
            const double z = bv * inv_or_zero(diag_Shat_cell(code, n, code[n.X]));
            x[n.X] = 0.0;
            r[n.X] = bv;
            d[n.X] = z;
            acc[0] += bv * z;
            acc[1] += z * z;
        }
    }
    if (reduce_across_blocks<2>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        st->rho = acc[0];
        st->z0 = sqrt(acc[1]);
        st->zrel = 1.0;
        st->alpha = st->beta = st->dq = 0.0;
        st->eps = eps;
        st->maxit = maxit;
        st->it = 0;
        st->status = 0;
        st->done = !(st->z0 > 0.0);
        if (!isfinite(acc[0]) || !isfinite(acc[1])) { st->status = -4; st->done = 1; }
    }
}

__global__ void k_cgS_stencil(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ d,
                              double* __restrict__ q, CgState* st, Reduce red) {
    if (st->done) return;
    const Column c = sweep_column(s);
    double acc[1] = {0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const Nbr n = neighbours(s.N, c.i, c.j, k);
            const double v = apply_Shat_cell(d, code, n, code[n.X], nullptr);
            q[n.X] = v;
            acc[0] += d[n.X] * v;
        }
    }
    if (reduce_across_blocks<1>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        st->dq = acc[0];
        if (!(acc[0] > 0.0) || !isfinite(acc[0])) {
            st->status = -4;
            st->done = 1;
        } else {
            st->alpha = st->rho / acc[0];
        }
    }
}

__global__ void k_cgS_update(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ x,
                             double* __restrict__ r, const double* __restrict__ d, const double* __restrict__ q,
                             CgState* st, Reduce red) {
    if (st->done) return;
    const Column c = sweep_column(s);
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const Nbr n = neighbours(s.N, c.i, c.j, k);
            x[n.X] += alpha * d[n.X];
            const double rn = r[n.X] - alpha * q[n.X];
            r[n.X] = rn;
            const double z = rn * inv_or_zero(diag_Shat_cell(code, n, code[n.X]));
            acc[0] += rn * z;
            acc[1] += z * z;
        }
    }
    if (reduce_across_blocks<2>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        st->it += 1;
        st->zrel = sqrt(acc[1]) / st->z0;
        if (!isfinite(acc[0]) || !isfinite(acc[1])) {
            st->status = -4;
            st->done = 1;
        } else if (st->zrel < st->eps) {
            st->done = 1;
        } else if (st->it >= st->maxit) {
            st->status = 1;
            st->done = 1;
        } else {
            st->beta = acc[0] / st->rho;
            st->rho = acc[0];
        }
    }
}

__global__ void k_cgS_dir(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ r,
                          double* __restrict__ d, const CgState* st) {
    if (st->done) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const double beta = st->beta;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s.N, c.i, c.j, k);
        d[n.X] = r[n.X] * inv_or_zero(diag_Shat_cell(code, n, code[n.X])) + beta * d[n.X];
    }
}

// ---------------------------------------------------------------------------
// Outer-loop vector work (scalars from the host)
// ---------------------------------------------------------------------------
// up to three dot products of cell vectors, totals to red.out[0..2]
__global__ void k_dots(Sweep s, const double* a0, const double* b0, const double* a1, const double* b1,
                       const double* a2, const double* b2, Reduce red) {
    const Column c = sweep_column(s);
    double acc[3] = {0.0, 0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const int64_t X = vidx(s.N, c.i, c.j, k);
            acc[0] += a0[X] * b0[X];
            if (a1) acc[1] += a1[X] * b1[X];
            if (a2) acc[2] += a2[X] * b2[X];
        }
    }
    if (reduce_across_blocks<3>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        red.out[0] = acc[0];
        red.out[1] = acc[1];
        red.out[2] = acc[2];
    }
}

// sums of the three velocity planes, totals to red.out[0..2]
__global__ void k_face_sums(Sweep s, const double* __restrict__ u, Reduce red) {
    const Column c = sweep_column(s);
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    double acc[3] = {0.0, 0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const int64_t X = vidx(s.N, c.i, c.j, k);
            acc[0] += u[X];
            acc[1] += u[n3 + X];
            acc[2] += u[2 * n3 + X];
        }
    }
    if (reduce_across_blocks<3>(acc, red, c.lb, s.nblk) && threadIdx.x == 0) {
        red.out[0] = acc[0];
        red.out[1] = acc[1];
        red.out[2] = acc[2];
    }
}

// p += alpha d, r -= alpha q
__global__ void k_outer_update(Sweep s, double* __restrict__ p, double* __restrict__ r, const double* __restrict__ d,
                               const double* __restrict__ q, double alpha) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int64_t X = vidx(s.N, c.i, c.j, k);
        p[X] += alpha * d[X];
        r[X] -= alpha * q[X];
    }
}

// u += a v on all three planes
__global__ void k_axpy_faces(Sweep s, double* __restrict__ u, const double* __restrict__ v, double a) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const int64_t n3 = (int64_t)s.N * s.N * s.N;
    for (int k = c.k0; k < c.k1; ++k) {
        const int64_t X = vidx(s.N, c.i, c.j, k);
        u[X] += a * v[X];
        u[n3 + X] += a * v[n3 + X];
        u[2 * n3 + X] += a * v[2 * n3 + X];
    }
}

// d = z + beta d
__global__ void k_dir_cells(Sweep s, double* __restrict__ d, const double* __restrict__ z, double beta) {
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int64_t X = vidx(s.N, c.i, c.j, k);
        d[X] = z[X] + beta * d[X];
    }
}

// ---------------------------------------------------------------------------
// Per-component mean removal (the constant pressure nullspace of each
// component).  One component: sums over the fluid bitmask.  Several: every
// wave adds its 64 values per distinct label into its own LDS bins (fixed
// order), blocks write per-component partials, a second kernel adds them in
// block order.  Flat grid: block b owns a contiguous range of voxels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int label_at(const uint16_t* label, const uint32_t* bits, int N, int wpr, int64_t X) {
    if (label) {
        const int l = label[X];
        return l == 0xFFFF ? -1 : l;
    }
    const int i = (int)(X % N);
    const int64_t row = X / N;
    return ((bits[row * wpr + (i >> 5)] >> (i & 31)) & 1) ? 0 : -1;
}

__global__ void k_comp_sum(const double* __restrict__ x, const uint16_t* __restrict__ label,
                           const uint32_t* __restrict__ bits, int N, int wpr, int64_t n3, int K, int64_t chunk,
                           double* __restrict__ part) {
    extern __shared__ double bins[];  // [kWaves][K]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = threadIdx.x; q < kWaves * K; q += kBlock) bins[q] = 0.0;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = min(n3, beg + chunk);
    for (int64_t base = beg + 64 * w; base < end; base += kBlock) {
        const int64_t X = base + lane;
        int l = -1;
        double v = 0.0;
        if (X < end) {
            l = label_at(label, bits, N, wpr, X);
            if (l >= 0) v = x[X];
        }
        unsigned long long todo = __ballot(l >= 0);
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const int L = __shfl(l, leader, 64);
            const bool mine = (l == L);
            const double sum = wave_sum(mine ? v : 0.0);
            if (lane == 0) bins[w * K + L] += sum;
            todo &= ~__ballot(mine);
        }
    }
    __syncthreads();
    for (int L = threadIdx.x; L < K; L += kBlock) {
        double a = bins[L];
        for (int q = 1; q < kWaves; ++q) a += bins[q * K + L];
        part[(int64_t)blockIdx.x * K + L] = a;
    }
}

__global__ void k_comp_mean(const double* __restrict__ part, int nblk, int K, const double* __restrict__ count,
                            double* __restrict__ mean) {
    const int L = blockIdx.x * kBlock + threadIdx.x;
    if (L >= K) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += part[(int64_t)b * K + L];
    mean[L] = a / count[L];
}

__global__ void k_comp_sub(double* __restrict__ x, const uint16_t* __restrict__ label,
                           const uint32_t* __restrict__ bits, int N, int wpr, int64_t n3,
                           const double* __restrict__ mean) {
    for (int64_t X = (int64_t)blockIdx.x * kBlock + threadIdx.x; X < n3; X += (int64_t)gridDim.x * kBlock) {
        const int l = label_at(label, bits, N, wpr, X);
        if (l >= 0) x[X] -= mean[l];
    }
}

}  // namespace stokes
