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
// Reductions are deterministic and need neither atomics nor fences: each
// block writes one partial per quantity with a plain store; the next kernel
// (after the kernel boundary has made those stores visible) has every block
// add all partials in block order, so every block derives bit-identical CG
// scalars on its own and inner loops run without host round trips.  (A
// device-scope fence per block would write back the XCD's L2 each time.)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stokes {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 4096;      // partial slots per reduced quantity
constexpr int kMaxCompLds = 2048;     // components handled by the projection kernels

// z-planes whose loads a thread issues together before computing them
constexpr int kZBatch = 4;     // cell kernels
constexpr int kZBatchA = 2;    // face kernels (three planes of unknowns per voxel)

// partial slots of the inner CG loops
constexpr int kRZ = 0, kZZ = 1, kDQ = 2, kNumSlots = 3;

// Batched contexts: B members (independent geometries of one size) whose
// device buffers sit at one fixed byte stride from each other; a launch covers
// every member, with grid y = member, and each block shifts its pointers by
// member * stride.  A plain context is one member with stride 0.
constexpr int kMaxBatch = 32;

struct Sweep {
    int N;
    int bxlog;        // BX = 1 << bxlog, BY = kBlock >> bxlog
    int gx, gy, gz;   // blocks along x, y and z
    int lz;           // z-planes per block
    int nblk;         // gx * gy * gz (per member)
    int N2;           // N * N
    int n3;           // N^3 (< 2^31 for N <= 800)
    int nbatch;       // members (grid y)
    unsigned active;  // outer-loop kernels: bit m set = member m takes part
    size_t bstride;   // bytes from one member's buffers to the next one's
};

// Per-member scalars of an outer-loop kernel (by value).
struct MemberScalars {
    double v[kMaxBatch];
};

// Pointer arithmetic on the pointer itself (not through an integer), so the
// compiler still knows what it points into (its no-alias facts survive); a
// null pointer stays null.
template <class P>
__device__ __forceinline__ void shift1(P& p, size_t o) {
    p = (P)(const_cast<char*>(reinterpret_cast<const char*>(p)) + (p ? o : (size_t)0));
}

// Point each pointer at this block's member (grid y) of a batched context.
template <class... P>
__device__ __forceinline__ void shift_all(size_t o, P&... p) {
    (shift1(p, o), ...);
}

// The same for pointers that are never null (no select on the offset).
template <class P>
__device__ __forceinline__ void shift1_nn(P& p, size_t o) {
    p = (P)(const_cast<char*>(reinterpret_cast<const char*>(p)) + o);
}
template <class... P>
__device__ __forceinline__ void shift_nn(size_t o, P&... p) {
    (shift1_nn(p, o), ...);
}

// Outer-loop kernels skip the members that sit out the current step.
__device__ __forceinline__ bool member_active(unsigned active) { return (active >> blockIdx.y) & 1u; }

// Inner CG state, resident in device memory.  Scalars are written by block 0
// only; rho is double-buffered by iteration parity because the other blocks
// of the kernel that writes rho_j still read rho_{j-1}.
struct CgState {
    double rho[2];    // (r_j, z_j) at [j & 1]
    double z0;        // ||z_0||
    double alpha, beta;
    double zrel;      // ||z_j|| / ||z_0||
    double dq;        // (d_j, A d_j)
    double eps;
    int it;           // operator applications so far = index j of the next iteration
    int jcur;         // j of the iteration in progress (set by its direction kernel)
    int done;         // 1: stop (converged, capped or broken down)
    int status;       // 0 ok, 1 iteration cap, -4 breakdown
    int maxit;
};

// 1 / diag(A) = 1 / (5 + s) on an active face (s = 1..5), 0 on an inactive one.
// Selects rather than a table: a per-lane table index would turn every use
// into a dependent memory load.
__device__ __forceinline__ double inv_diag_A(int s) {
    double v = 0.0;
    v = s == 1 ? 1.0 / 6.0 : v;
    v = s == 2 ? 1.0 / 7.0 : v;
    v = s == 3 ? 1.0 / 8.0 : v;
    v = s == 4 ? 1.0 / 9.0 : v;
    v = s == 5 ? 1.0 / 10.0 : v;
    return v;
}

__device__ __forceinline__ int sx_of(int code) { return code % 6; }
__device__ __forceinline__ int sy_of(int code) { return (code / 6) % 6; }
__device__ __forceinline__ int sz_of(int code) { return code / 36; }

__device__ __forceinline__ int xcd_remap(int b, int nblk) {
    if ((nblk & 7) != 0) return b;
    return (b & 7) * (nblk >> 3) + (b >> 3);
}

// One thread's column: (i, j) and a run of z-planes [k0, k1), with the
// periodic in-plane neighbour offsets.
struct Column {
    int lb;                  // logical block id
    int i, j, k0, k1;
    bool valid;
    int X0;                  // i + N j
    int oxm, oxp, oym, oyp;  // offsets to the x/y neighbours (wrapped)
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
    const int N = s.N;
    c.X0 = c.i + N * c.j;
    c.oxm = c.i == 0 ? N - 1 : -1;
    c.oxp = c.i == N - 1 ? -(N - 1) : 1;
    c.oym = c.j == 0 ? (N - 1) * N : -N;
    c.oyp = c.j == N - 1 ? -(N - 1) * N : N;
    return c;
}

// Seven-point neighbourhood of voxel (i, j, k) as flat indices within one plane.
struct Nbr {
    int X, xm, xp, ym, yp, zm, zp;
};

__device__ __forceinline__ Nbr neighbours(const Sweep& s, const Column& c, int k) {
    Nbr n;
    n.X = c.X0 + k * s.N2;
    n.xm = n.X + c.oxm;
    n.xp = n.X + c.oxp;
    n.ym = n.X + c.oym;
    n.yp = n.X + c.oyp;
    n.zm = n.X + (k == 0 ? (s.N - 1) * s.N2 : -s.N2);
    n.zp = n.X + (k == s.N - 1 ? -(s.N - 1) * s.N2 : s.N2);
    return n;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block sums of NP values; the totals are returned in every thread.
template <int NP>
__device__ __forceinline__ void block_sum_all(double (&v)[NP]) {
    __shared__ double lds[kNumSlots + 1][kWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        v[n] = wave_sum(v[n]);
        if (lane == 0) lds[n][w] = v[n];
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        double a = lds[n][0];
        for (int q = 1; q < kWaves; ++q) a += lds[n][q];
        v[n] = a;
    }
    __syncthreads();
}

// Write this block's partials for slots slot0 .. slot0+NP-1.
template <int NP>
__device__ __forceinline__ void write_partials(double (&v)[NP], double* part, int slot0, int lb) {
    block_sum_all<NP>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int n = 0; n < NP; ++n) part[(slot0 + n) * kMaxBlocks + lb] = v[n];
    }
}

// Totals of the partials left by the previous kernel, added in block order;
// identical bits in every block.
template <int NP>
__device__ __forceinline__ void read_totals(const double* part, const int (&slots)[NP], int nblk, double (&tot)[NP]) {
#pragma unroll
    for (int n = 0; n < NP; ++n) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nblk; b += kBlock) a += part[slots[n] * kMaxBlocks + b];
        tot[n] = a;
    }
    block_sum_all<NP>(tot);
}

// ---------------------------------------------------------------------------
// Setup: face codes from the remaining-fluid bitmask; inverse diagonal of the
// SIMPLE matrix
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fluid_bit(const uint32_t* bits, int N, int wpr, int i, int j, int k) {
    i = (i + N) % N;
    j = (j + N) % N;
    k = (k + N) % N;
    const uint32_t w = bits[((int64_t)k * N + j) * wpr + (i >> 5)];
    return (w >> (i & 31)) & 1;
}

__global__ void k_face_codes(Sweep s, const uint32_t* __restrict__ bits, int wpr, uint8_t* __restrict__ code) {
    shift_nn((size_t)blockIdx.y * s.bstride, bits, code);
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
        code[c.X0 + k * s.N2] = (uint8_t)(sc[0] + 6 * sc[1] + 36 * sc[2]);
    }
}

// diag(B diag(A)^-1 B^T) at a voxel: sum over its six faces of 1 / diag(A)_F
__device__ __forceinline__ double diag_Shat_cell(const uint8_t* __restrict__ code, const Nbr& n, int cdX) {
    return ((inv_diag_A(sx_of(cdX)) + inv_diag_A(sx_of(code[n.xp]))) +
            (inv_diag_A(sy_of(cdX)) + inv_diag_A(sy_of(code[n.yp])))) +
           (inv_diag_A(sz_of(cdX)) + inv_diag_A(sz_of(code[n.zp])));
}

__global__ void k_inv_diag_Shat(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ inv) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, inv);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        const double dS = diag_Shat_cell(code, n, code[n.X]);
        inv[n.X] = dS > 0.0 ? 1.0 / dS : 0.0;
    }
}

// The states of a voxel's six faces in 16 bits: its code (lower faces, bits
// 0-7) and, in the same encoding, its upper faces -- the x-state of the +x
// neighbour's code, the y-state of the +y neighbour's and the z-state of the
// +z neighbour's (bits 8-15).  Lets a sweep form the SIMPLE matrix's stencil
// and diagonal at a voxel from one load.
__global__ void k_code2(Sweep s, const uint8_t* __restrict__ code, uint16_t* __restrict__ code2) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, code2);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        const int up = sx_of(code[n.xp]) + 6 * sy_of(code[n.yp]) + 36 * sz_of(code[n.zp]);
        code2[n.X] = (uint16_t)(code[n.X] | (up << 8));
    }
}

// ---------------------------------------------------------------------------
// Plain operators (no reductions)
// ---------------------------------------------------------------------------
// (A u)_F = (5 + s_F) u_F - sum of the six neighbour faces of the same plane
__device__ __forceinline__ double apply_A_face(const double* __restrict__ u, const Nbr& n, int s) {
    const double nb = ((u[n.xm] + u[n.xp]) + (u[n.ym] + u[n.yp])) + (u[n.zm] + u[n.zp]);
    return (double)(5 + s) * u[n.X] - nb;
}

__global__ void k_apply_A(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ u,
                          double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, u, out);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        const int cd = code[n.X];
        const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
        for (int a = 0; a < 3; ++a)
            out[(size_t)a * s.n3 + n.X] = sc[a] ? apply_A_face(u + (size_t)a * s.n3, n, sc[a]) : 0.0;
    }
}

// (B^T p)(c, X) = p_X - p_{X - e_c} on active faces
__global__ void k_apply_BT(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ p,
                           double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, p, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    double* ox = out;
    double* oy = out + (size_t)s.n3;
    double* oz = out + 2 * (size_t)s.n3;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        const int cd = code[n.X];
        const double pX = p[n.X];
        ox[n.X] = sx_of(cd) ? pX - p[n.xm] : 0.0;
        oy[n.X] = sy_of(cd) ? pX - p[n.ym] : 0.0;
        oz[n.X] = sz_of(cd) ? pX - p[n.zm] : 0.0;
    }
}

// f - B^T p on active faces (right-hand side of the velocity recovery)
__global__ void k_force_minus_BT(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ p, double f0,
                                 double f1, double f2, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, p, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    double* ox = out;
    double* oy = out + (size_t)s.n3;
    double* oz = out + 2 * (size_t)s.n3;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        const int cd = code[n.X];
        const double pX = p[n.X];
        ox[n.X] = sx_of(cd) ? f0 - (pX - p[n.xm]) : 0.0;
        oy[n.X] = sy_of(cd) ? f1 - (pX - p[n.ym]) : 0.0;
        oz[n.X] = sz_of(cd) ? f2 - (pX - p[n.zm]) : 0.0;
    }
}

// (B u)_X = sum_c [u(c, X) - u(c, X + e_c)]  (0 in solid cells by the invariant)
__global__ void k_apply_B(Sweep s, const double* __restrict__ u, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, u, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const double* ux = u;
    const double* uy = u + (size_t)s.n3;
    const double* uz = u + 2 * (size_t)s.n3;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        out[n.X] = ((ux[n.X] - ux[n.xp]) + (uy[n.X] - uy[n.yp])) + (uz[n.X] - uz[n.zp]);
    }
}

// SIMPLE matrix: (Shat p)_X = sum over active faces F of X of (p_X - p_nbr) / diag(A)_F
__device__ __forceinline__ double apply_Shat_cell(const double pX, const double pxm, const double pxp,
                                                  const double pym, const double pyp, const double pzm,
                                                  const double pzp, const uint8_t* __restrict__ code, const Nbr& n,
                                                  int cdX) {
    const double wxl = inv_diag_A(sx_of(cdX)), wyl = inv_diag_A(sy_of(cdX)), wzl = inv_diag_A(sz_of(cdX));
    const double wxh = inv_diag_A(sx_of(code[n.xp])), wyh = inv_diag_A(sy_of(code[n.yp])),
                 wzh = inv_diag_A(sz_of(code[n.zp]));
    return ((wxl * (pX - pxm) + wxh * (pX - pxp)) + (wyl * (pX - pym) + wyh * (pX - pyp))) +
           (wzl * (pX - pzm) + wzh * (pX - pzp));
}

__global__ void k_apply_Shat(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ p,
                             double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, p, out);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        out[n.X] = apply_Shat_cell(p[n.X], p[n.xm], p[n.xp], p[n.ym], p[n.yp], p[n.zm], p[n.zp], code, n, code[n.X]);
    }
}

__global__ void k_diag_A(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, out);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        const int cd = code[X];
        const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
        for (int a = 0; a < 3; ++a) out[(size_t)a * s.n3 + X] = sc[a] ? (double)(5 + sc[a]) : 0.0;
    }
}

__global__ void k_diag_Shat(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, out);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        out[n.X] = diag_Shat_cell(code, n, code[n.X]);
    }
}

// zero the entries that are not unknowns (inactive faces / solid cells)
__global__ void k_mask_faces(Sweep s, const uint8_t* __restrict__ code, double* __restrict__ u) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, u);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        const int cd = code[X];
        if (!sx_of(cd)) u[X] = 0.0;
        if (!sy_of(cd)) u[(size_t)s.n3 + X] = 0.0;
        if (!sz_of(cd)) u[2 * (size_t)s.n3 + X] = 0.0;
    }
}

__global__ void k_mask_cells(Sweep s, const uint32_t* __restrict__ bits, int wpr, double* __restrict__ p) {
    shift_nn((size_t)blockIdx.y * s.bstride, bits, p);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        if (!fluid_bit(bits, s.N, wpr, c.i, c.j, k)) p[c.X0 + k * s.N2] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Inner Jacobi-PCG (Saad, Alg. 9.1) in three kernels per iteration j:
//   dir     : beta_j = rho_j / rho_{j-1} from the update's partials, the
//             convergence test ||z_j|| / ||z_0|| < eps, d_j = z_j + beta_j d_{j-1}
//             (pointwise, z = D^-1 r recomputed)
//   stencil : q = M d_j, partial (d_j, q)
//   update  : alpha_j = rho_j / (d_j, q); x += alpha d, r -= alpha q,
//             z = D^-1 r; partials (r, z), (z, z)
// A separate pointwise direction pass costs one more vector pass than
// recomputing the direction at the six neighbours inside the stencil, but
// keeps the stencil at one input array (measured faster on gfx950).
// ---------------------------------------------------------------------------
// Returns true when this iteration should not run; block 0 records why.
// The iteration index j lives in the state, so a launch sequence is the same
// for every iteration (and can be replayed as a graph): the direction kernel
// takes j = it and publishes it as jcur for the update kernel, whose block 0
// advances it (no kernel both reads and writes the field another block reads).
// j == 0: d_0 = z_0, and z0 = ||z_0|| is recorded.
__device__ __forceinline__ bool cg_dir_scalars(CgState* st, const double* part, int nblk, double* beta_out,
                                               int* j_out) {
    const int j = st->it;
    *j_out = j;
    const int slots[2] = {kRZ, kZZ};
    double tot[2];
    read_totals<2>(part, slots, nblk, tot);
    const double rho = tot[0];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        if (lead) { st->status = -4; st->done = 1; st->it = j; }
        return true;
    }
    const double zn = sqrt(tot[1]);
    double beta = 0.0, zrel = 1.0;
    if (j == 0) {
        if (lead) { st->z0 = zn; st->zrel = 1.0; }
        if (!(zn > 0.0)) {
            if (lead) { st->done = 1; st->it = 0; }
            return true;
        }
    } else {
        zrel = zn / st->z0;
        if (zrel < st->eps || j >= st->maxit) {
            if (lead) {
                st->zrel = zrel;
                st->it = j;
                if (!(zrel < st->eps)) st->status = 1;
                st->done = 1;
            }
            return true;
        }
        beta = rho / st->rho[(j - 1) & 1];
    }
    if (lead) {
        st->rho[j & 1] = rho;
        st->beta = beta;
        st->zrel = zrel;
        st->jcur = j;
    }
    *beta_out = beta;
    return false;
}

__device__ __forceinline__ bool cg_update_scalars(CgState* st, const double* part, int nblk, double* alpha_out) {
    const int j = st->jcur;
    const int slots[1] = {kDQ};
    double tot[1];
    read_totals<1>(part, slots, nblk, tot);
    const double dq = tot[0];
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    if (!(dq > 0.0) || !isfinite(dq)) {
        if (lead) { st->dq = dq; st->status = -4; st->done = 1; st->it = j; }
        return true;
    }
    const double alpha = st->rho[j & 1] / dq;
    if (lead) {
        st->dq = dq;
        st->alpha = alpha;
        st->it = j + 1;
    }
    *alpha_out = alpha;
    return false;
}

// The inner-CG kernels are templates on the storage and arithmetic type T of
// x, r, d, q (double, or float for the mixed-precision path); partial dot
// products are always accumulated in double.
template <class T>
__device__ __forceinline__ T inv_diag_A_t(int s) {
    T v = T(0);
    v = s == 1 ? T(1.0 / 6.0) : v;
    v = s == 2 ? T(1.0 / 7.0) : v;
    v = s == 3 ? T(1.0 / 8.0) : v;
    v = s == 4 ? T(1.0 / 9.0) : v;
    v = s == 5 ? T(1.0 / 10.0) : v;
    return v;
}

// Per-block LDS table of the face data a voxel code encodes, so the stencils
// look it up instead of decoding the code and selecting 1 / (5 + s) (about
// fifteen instructions per face on this part): for a code c and plane a,
// inv[a][c] = 1 / diag(A) of the voxel's lower a-face and dg[a][c] = diag(A) =
// 5 + s (both 0 on an inactive face).  Filled by the block's threads; the
// caller synchronises before the first use.
constexpr int kCodes = 216;
template <class T>
struct FaceTab {
    T inv[3][kCodes];
    T dg[3][kCodes];
};

template <class T>
__device__ __forceinline__ void face_tab_fill(FaceTab<T>& t) {
    for (int c = (int)threadIdx.x; c < kCodes; c += (int)blockDim.x) {
        const int sc[3] = {sx_of(c), sy_of(c), sz_of(c)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            t.inv[a][c] = inv_diag_A_t<T>(sc[a]);
            t.dg[a][c] = sc[a] ? T(5 + sc[a]) : T(0);
        }
    }
}

// ---- A (faces), Jacobi diag(A) = 5 + s -------------------------------------
// x = 0, r = b (b == nullptr: the uniform force on active faces); partials of
// (r, z), (z, z) with z = D^-1 r.  b is always an FP64 vector of the outer loop.
template <class T>
__global__ void k_cgA_init(Sweep s, const uint8_t* __restrict__ code, const double* b, double f0, double f1,
                           double f2, T* __restrict__ x, T* r, CgState* st, double* part, double eps, int maxit) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, x, r, st, part);
    shift_all((size_t)blockIdx.y * s.bstride, b);
    if (!member_active(s.active)) {
        // this member sits the solve out: it is done before its first iteration
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->it = 0;
            st->status = 0;
            st->done = 1;
        }
        return;
    }
    const Column c = sweep_column(s);
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        const double fc[3] = {f0, f1, f2};
        for (int k = c.k0; k < c.k1; ++k) {
            const int X = c.X0 + k * s.N2;
            const int cd = code[X];
            const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t F = (size_t)a * s.n3 + X;
                const T bv = (T)(sc[a] ? (b ? b[F] : fc[a]) : 0.0);
                const T z = bv * inv_diag_A_t<T>(sc[a]);
                x[F] = T(0);
                r[F] = bv;
                acc[0] += (double)bv * (double)z;
                acc[1] += (double)z * (double)z;
            }
        }
    }
    write_partials<2>(acc, part, kRZ, c.lb);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->eps = eps;
        st->maxit = maxit;
        st->it = 0;
        st->status = 0;
        st->done = 0;
        st->alpha = st->beta = st->dq = 0.0;
    }
}

// plane a's face state from a voxel's code
__device__ __forceinline__ int s_of(int code, int a) { return a == 0 ? sx_of(code) : (a == 1 ? sy_of(code) : sz_of(code)); }

// zpre == nullptr: Jacobi, z = D^-1 r; otherwise z is read from zpre (the
// multigrid-preconditioned residual, three planes)
template <class T>
__global__ void k_cgA_dir(Sweep s, const uint8_t* __restrict__ code, const T* __restrict__ r, T* __restrict__ d,
                          CgState* st, double* part, const T* __restrict__ zpre) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, r, d, st, part);
    shift_all((size_t)blockIdx.y * s.bstride, zpre);
    if (st->done) return;
    double beta_d;
    int j;
    if (cg_dir_scalars(st, part, s.nblk, &beta_d, &j)) return;
    const T beta = (T)beta_d;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const bool first = j == 0;
    for (int k0 = c.k0; k0 < c.k1; k0 += kZBatch) {
        // loads of up to kZBatch planes first, so they are in flight together
        T rv[kZBatch][3], dv[kZBatch][3];
        int cd[kZBatch];
#pragma unroll
        for (int u = 0; u < kZBatch; ++u) {
            // planes past the run re-read the first plane; their results are dropped
            const int X = c.X0 + (k0 + u < c.k1 ? k0 + u : c.k0) * s.N2;
            cd[u] = code[X];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                rv[u][a] = zpre ? zpre[(size_t)a * s.n3 + X] : r[(size_t)a * s.n3 + X];
                dv[u][a] = d[(size_t)a * s.n3 + X];
            }
        }
#pragma unroll
        for (int u = 0; u < kZBatch; ++u) {
            const bool in = k0 + u < c.k1;
            const int X = c.X0 + (in ? k0 + u : c.k0) * s.N2;
            const int sc[3] = {sx_of(cd[u]), sy_of(cd[u]), sz_of(cd[u])};
            T dn[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T z = zpre ? rv[u][a] : rv[u][a] * inv_diag_A_t<T>(sc[a]);
                dn[a] = first ? z : z + beta * dv[u][a];
            }
            if (in)
                for (int a = 0; a < 3; ++a) d[(size_t)a * s.n3 + X] = dn[a];
        }
    }
}

template <class T>
__global__ void k_cgA_update(Sweep s, const uint8_t* __restrict__ code, T* __restrict__ x, T* __restrict__ r,
                             const T* __restrict__ d, const T* __restrict__ q, CgState* st, double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, x, r, d, q, st, part);
    if (st->done) return;
    double alpha_d;
    if (cg_update_scalars(st, part, s.nblk, &alpha_d)) return;
    const T alpha = (T)alpha_d;
    const Column c = sweep_column(s);
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        for (int k0 = c.k0; k0 < c.k1; k0 += kZBatchA) {
            T xv[kZBatchA][3], rv[kZBatchA][3], dv[kZBatchA][3], qv[kZBatchA][3];
            int cd[kZBatchA];
#pragma unroll
            for (int u = 0; u < kZBatchA; ++u) {
                const int X = c.X0 + (k0 + u < c.k1 ? k0 + u : c.k0) * s.N2;
                cd[u] = code[X];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const size_t F = (size_t)a * s.n3 + X;
                    xv[u][a] = x[F];
                    rv[u][a] = r[F];
                    dv[u][a] = d[F];
                    qv[u][a] = q[F];
                }
            }
#pragma unroll
            for (int u = 0; u < kZBatchA; ++u) {
                const bool in = k0 + u < c.k1;
                const int X = c.X0 + (in ? k0 + u : c.k0) * s.N2;
                const int sc[3] = {sx_of(cd[u]), sy_of(cd[u]), sz_of(cd[u])};
                T xn[3], rn[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    xn[a] = xv[u][a] + alpha * dv[u][a];
                    rn[a] = rv[u][a] - alpha * qv[u][a];
                    const T z = rn[a] * inv_diag_A_t<T>(sc[a]);
                    acc[0] += in ? (double)rn[a] * (double)z : 0.0;
                    acc[1] += in ? (double)z * (double)z : 0.0;
                }
                if (in)
                    for (int a = 0; a < 3; ++a) {
                        x[(size_t)a * s.n3 + X] = xn[a];
                        r[(size_t)a * s.n3 + X] = rn[a];
                    }
            }
        }
    }
    write_partials<2>(acc, part, kRZ, c.lb);
}

// ---- SIMPLE matrix (cells), Jacobi with the precomputed inverse diagonal ----
template <class T>
__global__ void k_cgS_init(Sweep s, const T* __restrict__ invd, const double* b, T* __restrict__ x, T* r,
                           CgState* st, double* part, double eps, int maxit) {
    shift_nn((size_t)blockIdx.y * s.bstride, invd, b, x, r, st, part);
    if (!member_active(s.active)) {
        // this member sits the solve out: it is done before its first iteration
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->it = 0;
            st->status = 0;
            st->done = 1;
        }
        return;
    }
    const Column c = sweep_column(s);
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const int X = c.X0 + k * s.N2;
            const T bv = (T)b[X];
            const T z = bv * invd[X];
            x[X] = T(0);
            r[X] = bv;
            acc[0] += (double)bv * (double)z;
            acc[1] += (double)z * (double)z;
        }
    }
    write_partials<2>(acc, part, kRZ, c.lb);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->eps = eps;
        st->maxit = maxit;
        st->it = 0;
        st->status = 0;
        st->done = 0;
        st->alpha = st->beta = st->dq = 0.0;
    }
}

// zpre == nullptr: Jacobi, z = D^-1 r; otherwise z is read from zpre (the
// multigrid-preconditioned residual)
template <class T>
__global__ void k_cgS_dir(Sweep s, const T* __restrict__ invd, const T* __restrict__ r, T* __restrict__ d,
                          CgState* st, double* part, const T* __restrict__ zpre) {
    shift_nn((size_t)blockIdx.y * s.bstride, invd, r, d, st, part);
    shift_all((size_t)blockIdx.y * s.bstride, zpre);
    if (st->done) return;
    double beta_d;
    int j;
    if (cg_dir_scalars(st, part, s.nblk, &beta_d, &j)) return;
    const T beta = (T)beta_d;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const bool first = j == 0;
    for (int k0 = c.k0; k0 < c.k1; k0 += kZBatch) {
        T rv[kZBatch], iv[kZBatch], dv[kZBatch];
#pragma unroll
        for (int u = 0; u < kZBatch; ++u) {
            const int X = c.X0 + (k0 + u < c.k1 ? k0 + u : c.k0) * s.N2;
            if (zpre) {
                rv[u] = zpre[X];
                iv[u] = T(1);
            } else {
                rv[u] = r[X];
                iv[u] = invd[X];
            }
            dv[u] = d[X];
        }
#pragma unroll
        for (int u = 0; u < kZBatch; ++u) {
            const T z = rv[u] * iv[u];
            const T dn = first ? z : z + beta * dv[u];
            if (k0 + u < c.k1) d[c.X0 + (k0 + u) * s.N2] = dn;
        }
    }
}

// ---- LDS-tiled stencils -------------------------------------------------------
// A block marches its BX x BY column through z; a thread keeps its own
// column's values at k-1, k, k+1 in registers, and plane k of the tile plus a
// one-voxel ring (loaded by the first 2 (BX + BY) threads) goes through LDS
// (double-buffered: one barrier per plane) for the in-plane neighbours, so each
// value is loaded from memory about once instead of seven times.  Lanes past
// the box edge load their wrapped position, the periodic neighbour of the last
// voxel inside.
constexpr int kTileMax = 396;   // (BX + 2)(BY + 2): 64 x 4 -> 396, 32 x 8 -> 340

struct Tile {
    int lb, N, W;
    int gi, gj, wi, wj;      // own column (global, wrapped)
    bool valid;
    int k0, k1;
    int own;                 // LDS slot of the own column
    bool ring;               // this thread loads a ring point
    int hi, hj, hslot;       // its wrapped position and LDS slot
};

__device__ __forceinline__ Tile tile_of(const Sweep& s) {
    Tile t;
    t.N = s.N;
    t.lb = xcd_remap((int)blockIdx.x, s.nblk);
    const int BX = 1 << s.bxlog, BY = kBlock >> s.bxlog;
    t.W = BX + 2;
    const int bx = t.lb % s.gx, r = t.lb / s.gx, by = r % s.gy, bz = r / s.gy;
    const int tx = (int)threadIdx.x & (BX - 1), ty = (int)threadIdx.x >> s.bxlog;
    t.gi = bx * BX + tx;
    t.gj = by * BY + ty;
    t.valid = t.gi < s.N && t.gj < s.N;
    t.wi = t.gi % s.N;
    t.wj = t.gj % s.N;
    t.k0 = bz * s.lz;
    t.k1 = min(s.N, t.k0 + s.lz);
    t.own = (ty + 1) * t.W + (tx + 1);
    const int h = (int)threadIdx.x;
    int hx, hy;
    if (h < BY) { hx = -1; hy = h; }
    else if (h < 2 * BY) { hx = BX; hy = h - BY; }
    else if (h < 2 * BY + BX) { hx = h - 2 * BY; hy = -1; }
    else { hx = h - 2 * BY - BX; hy = BY; }
    t.ring = h < 2 * (BX + BY);
    t.hi = ((bx * BX + hx) % s.N + s.N) % s.N;
    t.hj = ((by * BY + hy) % s.N + s.N) % s.N;
    t.hslot = (hy + 1) * t.W + (hx + 1);
    return t;
}

__device__ __forceinline__ int tile_zw(int k, int N) { return k < 0 ? k + N : (k >= N ? k - N : k); }

// q = Shat d on the cells and the partial (d, q), LDS-tiled
template <class T>
__global__ void __launch_bounds__(kBlock) k_cgS_stencil_tiled(Sweep s, const uint8_t* __restrict__ code,
                                                              const T* __restrict__ d, T* __restrict__ q,
                                                              CgState* st, double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, d, q, st, part);
    if (st->done) return;
    __shared__ T tl[2][kTileMax];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    const Tile t = tile_of(s);
    const int N = t.N, N2 = N * N, W = t.W;
    const int col = t.wi + N * t.wj;
    const int hcol = t.hi + N * t.hj;
    const int xp = t.wi == N - 1 ? col - (N - 1) : col + 1;
    const int yp = t.wj == N - 1 ? col - (N - 1) * N : col + N;
    T dprev = d[col + tile_zw(t.k0 - 1, N) * N2], dcur = d[col + t.k0 * N2];
    int ccur = code[col + t.k0 * N2];
    double acc[1] = {0.0};
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k) {
        const int kn = tile_zw(k + 1, N);
        const T dnext = d[col + kn * N2];
        const int cnext = code[col + kn * N2];
        const int cxp = code[xp + k * N2], cyp = code[yp + k * N2];
        if (t.ring) tl[buf][t.hslot] = d[hcol + k * N2];
        tl[buf][t.own] = dcur;
        __syncthreads();
        const T* w = tl[buf];
        const T qv = ((ft.inv[0][ccur] * (dcur - w[t.own - 1]) + ft.inv[0][cxp] * (dcur - w[t.own + 1])) +
                      (ft.inv[1][ccur] * (dcur - w[t.own - W]) + ft.inv[1][cyp] * (dcur - w[t.own + W]))) +
                     (ft.inv[2][ccur] * (dcur - dprev) + ft.inv[2][cnext] * (dcur - dnext));
        if (t.valid) {
            q[col + k * N2] = qv;
            acc[0] += (double)dcur * (double)qv;
        }
        dprev = dcur;
        dcur = dnext;
        ccur = cnext;
        buf ^= 1;
    }
    write_partials<1>(acc, part, kDQ, t.lb);
}

// q = A d on the faces (three planes) and the partial (d, q), LDS-tiled
template <class T>
__global__ void __launch_bounds__(kBlock) k_cgA_stencil_tiled(Sweep s, const uint8_t* __restrict__ code,
                                                              const T* __restrict__ d, T* __restrict__ q,
                                                              CgState* st, double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, d, q, st, part);
    if (st->done) return;
    __shared__ T tl[2][3][kTileMax];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    const Tile t = tile_of(s);
    const int N = t.N, N2 = N * N, W = t.W;
    const size_t n3 = (size_t)s.n3;
    const int col = t.wi + N * t.wj;
    const int hcol = t.hi + N * t.hj;
    T dprev[3], dcur[3];
    {
        const int Xp = col + tile_zw(t.k0 - 1, N) * N2, Xc = col + t.k0 * N2;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dprev[a] = d[a * n3 + Xp];
            dcur[a] = d[a * n3 + Xc];
        }
    }
    double acc[1] = {0.0};
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k) {
        const int Xn = col + tile_zw(k + 1, N) * N2, X = col + k * N2;
        T dnext[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) dnext[a] = d[a * n3 + Xn];
        const int cd = code[X];
        if (t.ring) {
            const int Xh = hcol + k * N2;
#pragma unroll
            for (int a = 0; a < 3; ++a) tl[buf][a][t.hslot] = d[a * n3 + Xh];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) tl[buf][a][t.own] = dcur[a];
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T* w = tl[buf][a];
            const T nbs = ((w[t.own - 1] + w[t.own + 1]) + (w[t.own - W] + w[t.own + W])) + (dprev[a] + dnext[a]);
            const T dg = ft.dg[a][cd];
            const T qv = dg > T(0) ? dg * dcur[a] - nbs : T(0);
            if (t.valid) {
                q[a * n3 + X] = qv;
                acc[0] += (double)dcur[a] * (double)qv;
            }
            dprev[a] = dcur[a];
            dcur[a] = dnext[a];
        }
        buf ^= 1;
    }
    write_partials<1>(acc, part, kDQ, t.lb);
}

// Direction update fused with the stencil, for the multigrid-preconditioned
// solves: beta and the convergence test from the previous partials (as the
// direction kernel), then dout = z + beta din (din ignored when j = 0) formed at
// every tile and ring point, written at the own voxel, and q = M dout with the
// partial (dout, q).  din and dout are different buffers: blocks read din at
// their ring points while neighbouring blocks write their own points.
template <class T>
__global__ void __launch_bounds__(kBlock) k_cgS_dirstencil_tiled(Sweep s, const uint8_t* __restrict__ code,
                                                                 const T* __restrict__ z, const T* __restrict__ din,
                                                                 T* __restrict__ dout, T* __restrict__ q, CgState* st,
                                                                 double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, z, din, dout, q, st, part);
    if (st->done) return;
    double beta_d;
    int j;
    if (cg_dir_scalars(st, part, s.nblk, &beta_d, &j)) return;
    const T beta = (T)beta_d;
    const bool first = j == 0;
    __shared__ T tl[2][kTileMax];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    const Tile t = tile_of(s);
    const int N = t.N, N2 = N * N, W = t.W;
    const int col = t.wi + N * t.wj;
    const int hcol = t.hi + N * t.hj;
    const int xp = t.wi == N - 1 ? col - (N - 1) : col + 1;
    const int yp = t.wj == N - 1 ? col - (N - 1) * N : col + N;
    auto dn = [&](int X) -> T { return first ? z[X] : z[X] + beta * din[X]; };
    T dprev = dn(col + tile_zw(t.k0 - 1, N) * N2), dcur = dn(col + t.k0 * N2);
    int ccur = code[col + t.k0 * N2];
    double acc[1] = {0.0};
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k) {
        const int kn = tile_zw(k + 1, N);
        const T dnext = dn(col + kn * N2);
        const int cnext = code[col + kn * N2];
        const int cxp = code[xp + k * N2], cyp = code[yp + k * N2];
        if (t.ring) tl[buf][t.hslot] = dn(hcol + k * N2);
        tl[buf][t.own] = dcur;
        __syncthreads();
        const T* w = tl[buf];
        const T qv = ((ft.inv[0][ccur] * (dcur - w[t.own - 1]) + ft.inv[0][cxp] * (dcur - w[t.own + 1])) +
                      (ft.inv[1][ccur] * (dcur - w[t.own - W]) + ft.inv[1][cyp] * (dcur - w[t.own + W]))) +
                     (ft.inv[2][ccur] * (dcur - dprev) + ft.inv[2][cnext] * (dcur - dnext));
        if (t.valid) {
            dout[col + k * N2] = dcur;
            q[col + k * N2] = qv;
            acc[0] += (double)dcur * (double)qv;
        }
        dprev = dcur;
        dcur = dnext;
        ccur = cnext;
        buf ^= 1;
    }
    write_partials<1>(acc, part, kDQ, t.lb);
}

// k_cgS_dirstencil_tiled with its loads software-pipelined over the z-march:
// at plane k a thread issues the loads of its own column at k + 2 (16-bit
// code, z, din) and of its ring point at k + 1 (z, din), and forms the
// direction from the values loaded one plane earlier, so the loads have a
// whole plane to arrive; the own 16-bit code (k_code2) gives the weights of
// all six faces.  Same arithmetic as the unpipelined kernel, point by point.
template <class T>
struct CgsRaw {
    int cd;
    T z, di;
};

template <class T>
__global__ void __launch_bounds__(kBlock) k_cgS_dirstencil_pipe(Sweep s, const uint16_t* __restrict__ code2,
                                                                const T* __restrict__ z, const T* __restrict__ din,
                                                                T* __restrict__ dout, T* __restrict__ q, CgState* st,
                                                                double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code2, z, din, dout, q, st, part);
    if (st->done) return;
    double beta_d;
    int j;
    if (cg_dir_scalars(st, part, s.nblk, &beta_d, &j)) return;
    const T beta = (T)beta_d;
    const bool first = j == 0;
    __shared__ T tl[2][kTileMax];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    const Tile t = tile_of(s);
    const int N = t.N, N2 = N * N, W = t.W, own = t.own, hslot = t.hslot;
    const bool ring = t.ring;
    const int col = t.wi + N * t.wj;
    const int hcol = t.hi + N * t.hj;
    // din is read also when the first iteration ignores it (an allocated
    // vector), so no branch on the iteration sits between the loads.  The own
    // column's 16-bit code gives all six face weights; ring points need none.
    auto load = [&](CgsRaw<T>& w, int X) {
        w.cd = code2[X];
        w.z = z[X];
        w.di = din[X];
    };
    auto loadh = [&](CgsRaw<T>& w, int X) {
        w.z = z[X];
        w.di = din[X];
    };
    auto dn = [&](const CgsRaw<T>& w) -> T { return first ? w.z : w.z + beta * w.di; };
    CgsRaw<T> ra, rb, ha, hb;
    load(ra, col + tile_zw(t.k0 - 1, N) * N2);
    load(rb, col + t.k0 * N2);
    T dprev = dn(ra), dcur = dn(rb);
    int ccur = rb.cd;
    load(ra, col + tile_zw(t.k0 + 1, N) * N2);
    if (ring) loadh(ha, hcol + t.k0 * N2);
    double acc[1] = {0.0};
    int buf = 0;
    auto plane = [&](int k, const CgsRaw<T>& rfin, CgsRaw<T>& rload, const CgsRaw<T>& hfin, CgsRaw<T>& hload) {
        load(rload, col + tile_zw(k + 2, N) * N2);
        if (ring) loadh(hload, hcol + tile_zw(k + 1, N) * N2);
        const T dnext = dn(rfin);
        const int cnext = rfin.cd;
        if (ring) tl[buf][hslot] = dn(hfin);
        tl[buf][own] = dcur;
        __syncthreads();
        const T* w = tl[buf];
        const int lo = ccur & 255, up = ccur >> 8;
        const T qv = ((ft.inv[0][lo] * (dcur - w[own - 1]) + ft.inv[0][up] * (dcur - w[own + 1])) +
                      (ft.inv[1][lo] * (dcur - w[own - W]) + ft.inv[1][up] * (dcur - w[own + W]))) +
                     (ft.inv[2][lo] * (dcur - dprev) + ft.inv[2][up] * (dcur - dnext));
        if (t.valid) {
            dout[col + k * N2] = dcur;
            q[col + k * N2] = qv;
            acc[0] += (double)dcur * (double)qv;
        }
        dprev = dcur;
        dcur = dnext;
        ccur = cnext;
        buf ^= 1;
    };
    int k = t.k0;
    for (; k + 1 < t.k1; k += 2) {
        plane(k, ra, rb, ha, hb);
        plane(k + 1, rb, ra, hb, ha);
    }
    if (k < t.k1) plane(k, ra, rb, ha, hb);
    write_partials<1>(acc, part, kDQ, t.lb);
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_cgA_dirstencil_tiled(Sweep s, const uint8_t* __restrict__ code,
                                                                 const T* __restrict__ z, const T* __restrict__ din,
                                                                 T* __restrict__ dout, T* __restrict__ q, CgState* st,
                                                                 double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, z, din, dout, q, st, part);
    if (st->done) return;
    double beta_d;
    int j;
    if (cg_dir_scalars(st, part, s.nblk, &beta_d, &j)) return;
    const T beta = (T)beta_d;
    const bool first = j == 0;
    __shared__ T tl[2][3][kTileMax];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    const Tile t = tile_of(s);
    const int N = t.N, N2 = N * N, W = t.W;
    const size_t n3 = (size_t)s.n3;
    const int col = t.wi + N * t.wj;
    const int hcol = t.hi + N * t.hj;
    auto dn = [&](size_t F) -> T { return first ? z[F] : z[F] + beta * din[F]; };
    T dprev[3], dcur[3];
    {
        const int Xp = col + tile_zw(t.k0 - 1, N) * N2, Xc = col + t.k0 * N2;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dprev[a] = dn(a * n3 + Xp);
            dcur[a] = dn(a * n3 + Xc);
        }
    }
    double acc[1] = {0.0};
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k) {
        const int Xn = col + tile_zw(k + 1, N) * N2, X = col + k * N2;
        T dnext[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) dnext[a] = dn(a * n3 + Xn);
        const int cd = code[X];
        if (t.ring) {
            const int Xh = hcol + k * N2;
#pragma unroll
            for (int a = 0; a < 3; ++a) tl[buf][a][t.hslot] = dn(a * n3 + Xh);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) tl[buf][a][t.own] = dcur[a];
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T* w = tl[buf][a];
            const T nbs = ((w[t.own - 1] + w[t.own + 1]) + (w[t.own - W] + w[t.own + W])) + (dprev[a] + dnext[a]);
            const T dg = ft.dg[a][cd];
            const T qv = dg > T(0) ? dg * dcur[a] - nbs : T(0);
            if (t.valid) {
                dout[a * n3 + X] = dcur[a];
                q[a * n3 + X] = qv;
                acc[0] += (double)dcur[a] * (double)qv;
            }
            dprev[a] = dcur[a];
            dcur[a] = dnext[a];
        }
        buf ^= 1;
    }
    write_partials<1>(acc, part, kDQ, t.lb);
}

template <class T>
__global__ void k_cgS_update(Sweep s, const T* __restrict__ invd, T* __restrict__ x, T* __restrict__ r,
                             const T* __restrict__ d, const T* __restrict__ q, CgState* st, double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, invd, x, r, d, q, st, part);
    if (st->done) return;
    double alpha_d;
    if (cg_update_scalars(st, part, s.nblk, &alpha_d)) return;
    const T alpha = (T)alpha_d;
    const Column c = sweep_column(s);
    double acc[2] = {0.0, 0.0};
    if (c.valid) {
        for (int k0 = c.k0; k0 < c.k1; k0 += kZBatch) {
            T xv[kZBatch], rv[kZBatch], dv[kZBatch], qv[kZBatch], iv[kZBatch];
#pragma unroll
            for (int u = 0; u < kZBatch; ++u) {
                const int X = c.X0 + (k0 + u < c.k1 ? k0 + u : c.k0) * s.N2;
                xv[u] = x[X];
                rv[u] = r[X];
                dv[u] = d[X];
                qv[u] = q[X];
                iv[u] = invd[X];
            }
#pragma unroll
            for (int u = 0; u < kZBatch; ++u) {
                const bool in = k0 + u < c.k1;
                const T xn = xv[u] + alpha * dv[u];
                const T rn = rv[u] - alpha * qv[u];
                const T z = rn * iv[u];
                acc[0] += in ? (double)rn * (double)z : 0.0;
                acc[1] += in ? (double)z * (double)z : 0.0;
                if (in) {
                    const int X = c.X0 + (k0 + u) * s.N2;
                    x[X] = xn;
                    r[X] = rn;
                }
            }
        }
    }
    write_partials<2>(acc, part, kRZ, c.lb);
}

// ---- mixed-precision helpers -------------------------------------------------
// out = in converted to FP64 (cells)
__global__ void k_widen_cells(Sweep s, const float* __restrict__ in, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, in, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        out[X] = (double)in[X];
    }
}

__global__ void k_narrow_cells(Sweep s, const double* __restrict__ in, float* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, in, out);
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        out[X] = (float)in[X];
    }
}

// res = rhs - A u in FP64 on active faces (residual of the velocity refinement);
// partials of (res, res) and (rhs, rhs) to out[3*b + 0..1]
__global__ void k_residual_A(Sweep s, const uint8_t* __restrict__ code, const double* __restrict__ rhs,
                             const double* __restrict__ u, double* __restrict__ res, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, rhs, u, res, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    double acc[3] = {0.0, 0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const Nbr n = neighbours(s, c, k);
            const int cd = code[n.X];
            const int sc[3] = {sx_of(cd), sy_of(cd), sz_of(cd)};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t off = (size_t)a * s.n3;
                const double bv = rhs[off + n.X];
                const double v = sc[a] ? bv - apply_A_face(u + off, n, sc[a]) : 0.0;
                res[off + n.X] = v;
                acc[0] += v * v;
                acc[1] += sc[a] ? bv * bv : 0.0;
            }
        }
    }
    block_sum_all<3>(acc);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[3 * c.lb + q] = acc[q];
}

// u += a v with v in FP32 (faces)
__global__ void k_axpy_faces_f32(Sweep s, double* __restrict__ u, const float* __restrict__ v, MemberScalars am) {
    shift_nn((size_t)blockIdx.y * s.bstride, u, v);
    if (!member_active(s.active)) return;
    const double a = am.v[blockIdx.y];
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        for (int q = 0; q < 3; ++q) u[(size_t)q * s.n3 + X] += a * (double)v[(size_t)q * s.n3 + X];
    }
}

// (B v)_X with v in FP32, result in FP64
__global__ void k_apply_B_f32(Sweep s, const float* __restrict__ u, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, u, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const float* ux = u;
    const float* uy = u + (size_t)s.n3;
    const float* uz = u + 2 * (size_t)s.n3;
    for (int k = c.k0; k < c.k1; ++k) {
        const Nbr n = neighbours(s, c, k);
        out[n.X] = (((double)ux[n.X] - (double)ux[n.xp]) + ((double)uy[n.X] - (double)uy[n.yp])) +
                   ((double)uz[n.X] - (double)uz[n.zp]);
    }
}

// ---------------------------------------------------------------------------
// Outer-loop vector work (scalars from the host)
// ---------------------------------------------------------------------------
// up to three dot products of cell vectors; per-block partials to out[3*b + q]
__global__ void k_dots(Sweep s, const double* a0, const double* b0, const double* a1, const double* b1,
                       const double* a2, const double* b2, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, a0, b0, out);
    shift_all((size_t)blockIdx.y * s.bstride, a1, b1, a2, b2);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    double acc[3] = {0.0, 0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const int X = c.X0 + k * s.N2;
            acc[0] += a0[X] * b0[X];
            if (a1) acc[1] += a1[X] * b1[X];
            if (a2) acc[2] += a2[X] * b2[X];
        }
    }
    block_sum_all<3>(acc);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[3 * c.lb + q] = acc[q];
}

// sums of the three velocity planes; per-block partials to out[3*b + c]
__global__ void k_face_sums(Sweep s, const double* __restrict__ u, double* __restrict__ out) {
    shift_nn((size_t)blockIdx.y * s.bstride, u, out);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    double acc[3] = {0.0, 0.0, 0.0};
    if (c.valid) {
        for (int k = c.k0; k < c.k1; ++k) {
            const int X = c.X0 + k * s.N2;
            acc[0] += u[X];
            acc[1] += u[(size_t)s.n3 + X];
            acc[2] += u[2 * (size_t)s.n3 + X];
        }
    }
    block_sum_all<3>(acc);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[3 * c.lb + q] = acc[q];
}

// p += alpha d, r -= alpha q
__global__ void k_outer_update(Sweep s, double* __restrict__ p, double* __restrict__ r, const double* __restrict__ d,
                               const double* __restrict__ q, MemberScalars am) {
    shift_nn((size_t)blockIdx.y * s.bstride, p, r, d, q);
    if (!member_active(s.active)) return;
    const double alpha = am.v[blockIdx.y];
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        p[X] += alpha * d[X];
        r[X] -= alpha * q[X];
    }
}

// u += a v on all three planes
__global__ void k_axpy_faces(Sweep s, double* __restrict__ u, const double* __restrict__ v, MemberScalars am) {
    shift_nn((size_t)blockIdx.y * s.bstride, u, v);
    if (!member_active(s.active)) return;
    const double a = am.v[blockIdx.y];
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        u[X] += a * v[X];
        u[(size_t)s.n3 + X] += a * v[(size_t)s.n3 + X];
        u[2 * (size_t)s.n3 + X] += a * v[2 * (size_t)s.n3 + X];
    }
}

// dst = src (cells), for the members in s.active
__global__ void k_copy_cells(Sweep s, double* __restrict__ dst, const double* __restrict__ src) {
    shift_nn((size_t)blockIdx.y * s.bstride, dst, src);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        dst[X] = src[X];
    }
}

// d = z + beta d
__global__ void k_dir_cells(Sweep s, double* __restrict__ d, const double* __restrict__ z, MemberScalars bm) {
    shift_nn((size_t)blockIdx.y * s.bstride, d, z);
    if (!member_active(s.active)) return;
    const double beta = bm.v[blockIdx.y];
    const Column c = sweep_column(s);
    if (!c.valid) return;
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
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
                           double* __restrict__ part, size_t bstride, unsigned active) {
    shift_nn((size_t)blockIdx.y * bstride, x, bits, part);
    shift_all((size_t)blockIdx.y * bstride, label);
    if (!member_active(active)) return;
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
                            double* __restrict__ mean, size_t bstride, unsigned active) {
    shift_nn((size_t)blockIdx.y * bstride, part, count, mean);
    if (!member_active(active)) return;
    const int L = blockIdx.x * kBlock + threadIdx.x;
    if (L >= K) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += part[(int64_t)b * K + L];
    mean[L] = a / count[L];
}

__global__ void k_comp_sub(double* __restrict__ x, const uint16_t* __restrict__ label,
                           const uint32_t* __restrict__ bits, int N, int wpr, int64_t n3,
                           const double* __restrict__ mean, size_t bstride, unsigned active) {
    shift_nn((size_t)blockIdx.y * bstride, x, bits, mean);
    shift_all((size_t)blockIdx.y * bstride, label);
    if (!member_active(active)) return;
    for (int64_t X = (int64_t)blockIdx.x * kBlock + threadIdx.x; X < n3; X += (int64_t)gridDim.x * kBlock) {
        const int l = label_at(label, bits, N, wpr, X);
        if (l >= 0) x[X] -= mean[l];
    }
}

// One conducting component (the common case): its mean is the box mean over the
// fluid cells, and cells outside it hold 0, so the sum runs over every cell.
// Per-block partials of the sum, then a kernel whose every block re-adds them
// in block order (bit-identical mean in every block) and subtracts the mean at
// the fluid cells: two sweeps instead of three latency-bound kernels.
__global__ void k_sum1(Sweep s, const double* __restrict__ x, double* __restrict__ part) {
    shift_nn((size_t)blockIdx.y * s.bstride, x, part);
    if (!member_active(s.active)) return;
    const Column c = sweep_column(s);
    double acc[1] = {0.0};
    if (c.valid)
        for (int k = c.k0; k < c.k1; ++k) acc[0] += x[c.X0 + k * s.N2];
    write_partials<1>(acc, part, 0, c.lb);
}

__global__ void k_sub_mean1(Sweep s, double* __restrict__ x, const uint32_t* __restrict__ bits, int wpr,
                            const double* __restrict__ part, double inv_count) {
    shift_nn((size_t)blockIdx.y * s.bstride, x, bits, part);
    if (!member_active(s.active)) return;
    const int slots[1] = {0};
    double tot[1];
    read_totals<1>(part, slots, s.nblk, tot);
    const double mean = tot[0] * inv_count;
    const Column c = sweep_column(s);
    if (!c.valid) return;
    const uint32_t bit = 1u << (c.i & 31);
    for (int k = c.k0; k < c.k1; ++k) {
        const int X = c.X0 + k * s.N2;
        if (bits[((int64_t)k * s.N + c.j) * wpr + (c.i >> 5)] & bit) x[X] -= mean;
    }
}

}  // namespace stokes
