// Geometric multigrid V-cycles used as preconditioners of the inner CG solves
// (the paper preconditions its inner solves with algebraic multigrid, Sec. 3.2):
//   - the SIMPLE matrix Shat = B diag(A)^-1 B^T on the cells (one plane), and
//   - the velocity Laplacian A, which is block-diagonal over the three
//     velocity components: each component is a scalar 7-point operator on its
//     own face lattice, so the cycle runs on a batch of three planes.
//
// Hierarchy: level 0 is the voxel grid, applied matrix-free from the face
// codes; level l+1 aggregates 2x2x2 blocks of level l (piecewise-constant
// prolongation P, restriction P^T) and holds the Galerkin operator P^T A_l P.
// For a 7-point operator that operator is again 7-point, stored per node as its
// diagonal D and the couplings W^x, W^y, W^z to the -x, -y, -z neighbours
// (matrix entries -W):
//   D_I   = sum of the children's diagonals - 2 * (couplings inside the block)
//   W^c_I = sum of the couplings of the four children on the block's -c face
// to the neighbouring block.
//
// V-cycle (symmetric, hence a valid CG preconditioner): on each level one
// smoothing step from zero, residual restricted to the next level, coarse
// correction prolonged and scaled, one smoothing step; the smoothing step is a
// damped-Jacobi sweep on level 0 and on the tiled coarse levels, and a
// red-black Gauss-Seidel sweep (red then black going down, black then red
// going up) on the smaller coarse levels; the coarsest level runs a fixed
// number of Jacobi sweeps inside one workgroup.  Scaling the coarse correction
// (by less than 2) keeps the cycle SPD and offsets the weak coarse operators
// of piecewise-constant aggregation.  Nodes that are not unknowns (diagonal 0)
// are held at 0.
#pragma once

#include "kernels.h"

namespace stokes {

// Level geometry: nb planes of n^3 nodes; node I = p * n3 + (i + n (j + n k)).
struct MgGrid {
    int n, n2, n3, nb;
    size_t bstride;   // batched contexts: bytes between members' buffers (0: one member)
};

enum { kMgFineShat = 0, kMgFineA = 1 };

__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int mg_idx(const MgGrid& g, int i, int j, int k) {
    return wrapc(i, g.n) + g.n * (wrapc(j, g.n) + g.n * wrapc(k, g.n));
}

// ---------------------------------------------------------------------------
// Level-0 coefficients from the face codes.
//   SIMPLE matrix: W^c(X) = 1 / diag(A) of face (c, X) (0 if not an unknown),
//                  D(X) = sum of the six face weights of X.
//   A, plane p:    node = face (p, X), D = 5 + s_p(X) if it is an unknown,
//                  W^c(X) = 1 if faces (p, X) and (p, X - e_c) are both unknowns.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int s_plane(int cd, int p) { return p == 0 ? sx_of(cd) : (p == 1 ? sy_of(cd) : sz_of(cd)); }

__device__ __forceinline__ double fine_shat_w(const uint8_t* __restrict__ code, const MgGrid& g, int i, int j, int k,
                                              int c) {
    return inv_diag_A(s_plane(code[mg_idx(g, i, j, k)], c));
}

__device__ __forceinline__ void fine_coeffs(const uint8_t* __restrict__ code, const MgGrid& g, int kind, int p, int i,
                                            int j, int k, double* D, double w[3]) {
    if (kind == kMgFineShat) {
        for (int c = 0; c < 3; ++c) w[c] = fine_shat_w(code, g, i, j, k, c);
        *D = (w[0] + fine_shat_w(code, g, i + 1, j, k, 0)) + (w[1] + fine_shat_w(code, g, i, j + 1, k, 1)) +
             (w[2] + fine_shat_w(code, g, i, j, k + 1, 2));
        return;
    }
    const int s = s_plane(code[mg_idx(g, i, j, k)], p);
    *D = s ? (double)(5 + s) : 0.0;
    const int sm[3] = {s_plane(code[mg_idx(g, i - 1, j, k)], p), s_plane(code[mg_idx(g, i, j - 1, k)], p),
                       s_plane(code[mg_idx(g, i, j, k - 1)], p)};
    for (int c = 0; c < 3; ++c) w[c] = (s && sm[c]) ? 1.0 : 0.0;
}

// Build level 1 from the codes.  One thread per coarse node (setup only).
template <class T>
__global__ void k_mg_coarsen_fine(MgGrid fg, MgGrid cg, int kind, const uint8_t* __restrict__ code,
                                  T* __restrict__ D, T* __restrict__ Wx, T* __restrict__ Wy, T* __restrict__ Wz) {
    shift_nn((size_t)blockIdx.y * fg.bstride, code, D, Wx, Wy, Wz);
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= cg.nb * cg.n3) return;
    const int p = I / cg.n3, L = I - p * cg.n3;
    const int ci = L % cg.n, cj = (L / cg.n) % cg.n, ck = L / cg.n2;
    double diag = 0.0, inner = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double d, w[3];
                fine_coeffs(code, fg, kind, p, 2 * ci + a, 2 * cj + b, 2 * ck + c, &d, w);
                diag += d;
                if (a == 1) inner += w[0]; else wx += w[0];
                if (b == 1) inner += w[1]; else wy += w[1];
                if (c == 1) inner += w[2]; else wz += w[2];
            }
    D[I] = (T)(diag - 2.0 * inner);
    Wx[I] = (T)wx;
    Wy[I] = (T)wy;
    Wz[I] = (T)wz;
}

// Build level l+1 from level l (l >= 1).
template <class T>
__global__ void k_mg_coarsen(MgGrid fg, MgGrid cg, const T* __restrict__ Df, const T* __restrict__ Wxf,
                             const T* __restrict__ Wyf, const T* __restrict__ Wzf, T* __restrict__ D,
                             T* __restrict__ Wx, T* __restrict__ Wy, T* __restrict__ Wz) {
    shift_nn((size_t)blockIdx.y * fg.bstride, Df, Wxf, Wyf, Wzf, D, Wx, Wy, Wz);
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= cg.nb * cg.n3) return;
    const int p = I / cg.n3, L = I - p * cg.n3;
    const int ci = L % cg.n, cj = (L / cg.n) % cg.n, ck = L / cg.n2;
    double diag = 0.0, inner = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const int f = p * fg.n3 + mg_idx(fg, 2 * ci + a, 2 * cj + b, 2 * ck + c);
                diag += (double)Df[f];
                if (a == 1) inner += (double)Wxf[f]; else wx += (double)Wxf[f];
                if (b == 1) inner += (double)Wyf[f]; else wy += (double)Wyf[f];
                if (c == 1) inner += (double)Wzf[f]; else wz += (double)Wzf[f];
            }
    D[I] = (T)(diag - 2.0 * inner);
    Wx[I] = (T)wx;
    Wy[I] = (T)wy;
    Wz[I] = (T)wz;
}

// Operator of one level.  Level 0 (code != nullptr) is matrix-free.
struct MgOp {
    const uint8_t* code;
    int kind;           // level 0: kMgFineShat or kMgFineA
    const void* invd;   // level 0, SIMPLE matrix: inverse diagonal (T)
    // levels >= 1: the Galerkin operator's diagonal and couplings, stored in
    // FP32 for both precisions (the cycle is a preconditioner; its vectors and
    // arithmetic keep the precision of the solve)
    const void* D;
    const void* Wx;
    const void* Wy;
    const void* Wz;
};

__device__ __forceinline__ void shift_op(MgOp& op, size_t o) {
    shift_all(o, op.code, op.invd, op.D, op.Wx, op.Wy, op.Wz);
}

// ---------------------------------------------------------------------------
// Level 0 (the voxel grid), column sweeps.  The first Jacobi sweep from zero,
// x0 = omega D^-1 b, is never stored: both kernels recompute it at the seven
// points of a stencil from b and the diagonal.
// ---------------------------------------------------------------------------

// Level-0 operator of plane a at voxel X, given x at the seven points
// (centre, -x, +x, -y, +y, -z, +z).  KIND A: (5 + s) x - sum of neighbours on
// an active face (s = face state from the voxel's code), 0 otherwise.
// KIND Shat: sum over the six faces of w (x_X - x_nbr), w = 1 / diag(A) of
// the face (0 on an inactive face).
template <class T, int KIND>
__device__ __forceinline__ T mgf_apply(const T (&v)[7], int cX, int cxp, int cyp, int czp, int a,
                                       const FaceTab<T>& ft) {
    if (KIND == kMgFineA) {
        const T dg = ft.dg[a][cX];
        const T nb = ((v[1] + v[2]) + (v[3] + v[4])) + (v[5] + v[6]);
        return dg > T(0) ? dg * v[0] - nb : T(0);
    }
    const T wxl = ft.inv[0][cX], wyl = ft.inv[1][cX], wzl = ft.inv[2][cX];
    const T wxh = ft.inv[0][cxp], wyh = ft.inv[1][cyp], wzh = ft.inv[2][czp];
    return ((wxl * (v[0] - v[1]) + wxh * (v[0] - v[2])) + (wyl * (v[0] - v[3]) + wyh * (v[0] - v[4]))) +
           (wzl * (v[0] - v[5]) + wzh * (v[0] - v[6]));
}

// Parents (level-1 nodes) of a voxel and of its neighbours across x, y and z:
// of the two x-neighbours one shares the voxel's parent, the other lies in
// the block across; likewise for y and z.
struct MgParents {
    int c;          // parent of the voxel
    int x, y, z;    // parent of the block across x, y, z
    bool xlo, ylo, zlo;  // voxel is the lower one of its pair (so -x lies across)
};

__device__ __forceinline__ MgParents mg_parents(int N, int cn, int i, int j, int k) {
    MgParents q;
    q.xlo = !(i & 1);
    q.ylo = !(j & 1);
    q.zlo = !(k & 1);
    const int ci = i >> 1, cj = j >> 1, ck = k >> 1;
    const int ai = q.xlo ? (i == 0 ? N - 1 : i - 1) >> 1 : (i == N - 1 ? 0 : i + 1) >> 1;
    const int aj = q.ylo ? (j == 0 ? N - 1 : j - 1) >> 1 : (j == N - 1 ? 0 : j + 1) >> 1;
    const int ak = q.zlo ? (k == 0 ? N - 1 : k - 1) >> 1 : (k == N - 1 ? 0 : k + 1) >> 1;
    q.c = ci + cn * (cj + cn * ck);
    q.x = ai + cn * (cj + cn * ck);
    q.y = ci + cn * (aj + cn * ck);
    q.z = ci + cn * (cj + cn * ak);
    return q;
}

// scale * (P xc) at the seven points (centre, -x, +x, -y, +y, -z, +z)
template <class T>
__device__ __forceinline__ void mg_prolong7(const MgParents& q, const T (&xp)[4], T scale, T (&e)[7]) {
    const T own = scale * xp[0], ax = scale * xp[1], ay = scale * xp[2], az = scale * xp[3];
    e[0] = own;
    e[1] = q.xlo ? ax : own;
    e[2] = q.xlo ? own : ax;
    e[3] = q.ylo ? ay : own;
    e[4] = q.ylo ? own : ay;
    e[5] = q.zlo ? az : own;
    e[6] = q.zlo ? own : az;
}

// ---------------------------------------------------------------------------
// Level 0, LDS-tiled: each block marches its BX x BY column through z.  The
// smoothed iterate (x0 = omega D^-1 b for the restriction, x' = x0 + scale P xc
// for the post-smoothing, 0 where D = 0) is computed once per point: a thread keeps its own
// column's values at k-1, k, k+1 in registers, and plane k of the tile plus
// a one-voxel ring (computed by the first 2 (BX + BY) threads) goes through
// LDS (double-buffered, one barrier per plane) for the in-plane neighbours.
// Lanes past the box edge compute the value at their wrapped position, which
// is exactly the periodic neighbour of the last voxel inside.
// ---------------------------------------------------------------------------

// Sum of v over the 2 x 2 in-plane blocks of voxels: the i pair by shuffle
// (lane i^1); the j pair by shuffle (lane^32) when columns are 32 wide, else
// through LDS (64-wide columns put the two rows in different waves).  Every
// thread of the block must call it (it may synchronise); the sums are valid in
// the lanes of even j.  lds: NB * kBlock / 2 values.
template <class T, int NB>
__device__ __forceinline__ void mg_pair_sum(T (&v)[NB], int bxlog, T* lds) {
#pragma unroll
    for (int a = 0; a < NB; ++a) v[a] += __shfl_xor(v[a], 1, 64);
    if (bxlog == 5) {
#pragma unroll
        for (int a = 0; a < NB; ++a) v[a] += __shfl_xor(v[a], 32, 64);
        return;
    }
    const int tx = (int)threadIdx.x & 63, ty = (int)threadIdx.x >> 6;
    const int slot = (ty >> 1) * 64 + tx;
    if (ty & 1) {
#pragma unroll
        for (int a = 0; a < NB; ++a) lds[a * (kBlock / 2) + slot] = v[a];
    }
    __syncthreads();
    if (!(ty & 1)) {
#pragma unroll
        for (int a = 0; a < NB; ++a) v[a] += lds[a * (kBlock / 2) + slot];
    }
    __syncthreads();
}

// Per-point data of the level-0 smoothed iterate.
template <class T, int KIND>
struct MgfPt {
    static constexpr int NB = KIND == kMgFineA ? 3 : 1;
    int cd;          // code of the voxel
    T b[NB];         // b of each plane
    T inv[NB];       // 1 / D of each plane
    T x[NB];         // smoothed iterate
};

template <class T, int KIND, bool POST>
__device__ __forceinline__ void mgf_point(MgfPt<T, KIND>& q, int N, int cn, int i, int j, int k,
                                          const uint8_t* __restrict__ code, const T* __restrict__ invd,
                                          const T* __restrict__ b, const T* __restrict__ xc, T scale, T omega,
                                          const FaceTab<T>& ft) {
    constexpr int NB = MgfPt<T, KIND>::NB;
    const int X = i + N * (j + N * k);
    const size_t n3 = (size_t)N * N * N;
    q.cd = code[X];
    T e[NB];
    if (POST) {
        const size_t cn3 = (size_t)cn * cn * cn;
        const int C = (i >> 1) + cn * ((j >> 1) + cn * (k >> 1));
#pragma unroll
        for (int a = 0; a < NB; ++a) e[a] = xc[a * cn3 + C];
    }
    if (KIND == kMgFineShat) q.inv[0] = invd[X];
#pragma unroll
    for (int a = 0; a < NB; ++a) q.b[a] = b[a * n3 + X];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        if (KIND == kMgFineA) q.inv[a] = ft.inv[a][q.cd];
        q.x[a] = omega * q.inv[a] * q.b[a];
        // the prolonged correction is held at 0 on nodes that are not unknowns:
        // A's stencil sums all six neighbours, and a wall must read as zero
        if (POST && q.inv[a] > T(0)) q.x[a] += scale * e[a];
    }
}

// POST = false: bc = P^T (b - A x0) into level 1 (Sweep with even z-runs; the
// 2 x 2 x 2 sum adds two consecutive planes, then the 2 x 2 in-plane block).
// POST = true: y = x' + omega D^-1 (b - A x'), nodes with 1/D = 0 held at 0,
// and the block's partial of (b, y) into part[slot][block] (Sweep: the CG's).
template <class T, int KIND, bool POST>
__global__ void __launch_bounds__(kBlock) k_mgf_tiled(Sweep s, int cn, const uint8_t* __restrict__ code,
                                                      const T* __restrict__ invd, const T* __restrict__ b,
                                                      const T* __restrict__ xc, T scale, T omega, T* __restrict__ out,
                                                      double* part, int slot, const CgState* st) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, b, out);
    shift_all((size_t)blockIdx.y * s.bstride, invd, xc, part, st);
    constexpr int NB = MgfPt<T, KIND>::NB;
    __shared__ T tile[2][NB][kTileMax];
    __shared__ T pair_lds[POST ? 1 : NB * kBlock / 2];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    __syncthreads();
    const Tile tt = tile_of(s);
    const int N = tt.N, W = tt.W, lb = tt.lb;
    const int gi = tt.gi, gj = tt.gj, wi = tt.wi, wj = tt.wj, k0 = tt.k0, k1 = tt.k1;
    const bool valid = tt.valid;
    const int hi = tt.hi, hj = tt.hj, hslot = tt.hslot, own = tt.own;
    auto zw = [N](int k) { return k < 0 ? k + N : (k >= N ? k - N : k); };

    MgfPt<T, KIND> cur, nxt;
    T xprev[NB];
    {
        MgfPt<T, KIND> pv;
        mgf_point<T, KIND, POST>(pv, N, cn, wi, wj, zw(k0 - 1), code, invd, b, xc, scale, omega, ft);
#pragma unroll
        for (int a = 0; a < NB; ++a) xprev[a] = pv.x[a];
    }
    mgf_point<T, KIND, POST>(cur, N, cn, wi, wj, k0, code, invd, b, xc, scale, omega, ft);
    // a finished solve is checked after the first loads (in bounds either way)
    if (st && st->done) return;
    double acc = 0.0;       // POST: partial of (b, y)
    T rsum[NB];             // restriction: residual summed over the plane pair
#pragma unroll
    for (int a = 0; a < NB; ++a) rsum[a] = T(0);
    int buf = 0;
    for (int k = k0; k < k1; ++k) {
        mgf_point<T, KIND, POST>(nxt, N, cn, wi, wj, zw(k + 1), code, invd, b, xc, scale, omega, ft);
        if (tt.ring) {
            MgfPt<T, KIND> hp;
            mgf_point<T, KIND, POST>(hp, N, cn, hi, hj, k, code, invd, b, xc, scale, omega, ft);
#pragma unroll
            for (int a = 0; a < NB; ++a) tile[buf][a][hslot] = hp.x[a];
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) tile[buf][a][own] = cur.x[a];
        // KIND Shat: the +x and +y faces' codes
        int cxp = 0, cyp = 0;
        if (KIND == kMgFineShat) {
            const int X = wi + N * (wj + N * k);
            cxp = code[X - wi + (wi == N - 1 ? 0 : wi + 1)];
            cyp = code[X + (wj == N - 1 ? -(N - 1) * N : N)];
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const T* tl = tile[buf][a];
            const T v[7] = {cur.x[a], tl[own - 1], tl[own + 1], tl[own - W], tl[own + W], xprev[a], nxt.x[a]};
            const T ax = mgf_apply<T, KIND>(v, cur.cd, cxp, cyp, nxt.cd, a, ft);
            if (POST) {
                const T yv = cur.inv[a] > T(0) ? v[0] + omega * cur.inv[a] * (cur.b[a] - ax) : T(0);
                if (valid) {
                    out[(size_t)a * s.n3 + wi + N * (wj + N * k)] = yv;
                    acc += (double)cur.b[a] * (double)yv;
                }
            } else {
                rsum[a] += cur.b[a] - ax;
            }
        }
        if (!POST && (k & 1)) {
            // pair complete: 2 x 2 in-plane sum and store
            const int cN = N >> 1;
            mg_pair_sum<T, NB>(rsum, s.bxlog, pair_lds);
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                if (valid && !(gi & 1) && !(gj & 1))
                    out[(size_t)a * cN * cN * cN + (gi >> 1) + cN * ((gj >> 1) + cN * (k >> 1))] = rsum[a];
                rsum[a] = T(0);
            }
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) xprev[a] = cur.x[a];
        cur = nxt;
        buf ^= 1;
    }
    if (POST) {
        double v1[1] = {acc};
        write_partials<1>(v1, part, slot, lb);
    }
}

// The SIMPLE matrix's level-0 post-smoothing (k_mgf_tiled<T, kMgFineShat,
// true>) with its loads software-pipelined over the z-march: at plane k a
// thread issues the raw loads of its own column at k + 2 and of its ring point
// at k + 1, and finishes the values loaded one plane earlier, so every load has
// a whole plane (barrier and stencil) to arrive instead of being waited for in
// the plane that issued it.  A point's six face states come from its 16-bit
// code (k_code2), so it needs neither the stored 1/D nor its neighbours'
// codes: 1/D is recomputed with the arithmetic of k_inv_diag_Shat (bitwise the
// stored value), and the six face weights it needs are kept for the point's
// stencil.  Same arithmetic as the unpipelined kernel, point by point.
// The six face weights of a voxel (lower x, y, z, then upper x, y, z) from its
// 16-bit code, and its inverse diagonal.
template <class T>
__device__ __forceinline__ T weights_S2(int c2, const FaceTab<T>& ft, T (&w)[6]) {
    const int lo = c2 & 255, up = c2 >> 8;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w[a] = ft.inv[a][lo];
        w[3 + a] = ft.inv[a][up];
    }
    const T dS = ((w[0] + w[3]) + (w[1] + w[4])) + (w[2] + w[5]);
    return dS > T(0) ? T(1) / dS : T(0);
}

// the SIMPLE matrix at level 0 from a voxel's six face weights (the sums of
// mgf_apply<T, kMgFineShat> in the same order)
template <class T>
__device__ __forceinline__ T apply_S_w(const T (&v)[7], const T (&w)[6]) {
    return ((w[0] * (v[0] - v[1]) + w[3] * (v[0] - v[2])) + (w[1] * (v[0] - v[3]) + w[4] * (v[0] - v[4]))) +
           (w[2] * (v[0] - v[5]) + w[5] * (v[0] - v[6]));
}

template <class T>
struct MgfRawS {
    int cd;
    T b, e;
};

template <class T>
__device__ __forceinline__ void mgfs_load(MgfRawS<T>& q, int N, int cn, int i, int j, int k,
                                          const uint16_t* __restrict__ code2, const T* __restrict__ b,
                                          const T* __restrict__ xc) {
    const int X = i + N * (j + N * k);
    q.cd = code2[X];
    q.b = b[X];
    q.e = xc[(i >> 1) + cn * ((j >> 1) + cn * (k >> 1))];
}

template <class T>
struct MgfPtS {
    T w[6];         // face weights (weights_S2)
    T inv, b, x;
};

template <class T>
__global__ void __launch_bounds__(kBlock) k_mgf_smooth_S_pipe(Sweep s, int cn, const uint16_t* __restrict__ code2,
                                                              const T* __restrict__ b, const T* __restrict__ xc,
                                                              T scale, T omega, T* __restrict__ out, double* part,
                                                              int slot, const CgState* st) {
    shift_nn((size_t)blockIdx.y * s.bstride, code2, b, xc, out, part);
    shift_all((size_t)blockIdx.y * s.bstride, st);
    __shared__ T tile[2][kTileMax];
    __shared__ FaceTab<T> ft;
    face_tab_fill<T>(ft);
    __syncthreads();
    const Tile tt = tile_of(s);
    const int N = tt.N, W = tt.W, lb = tt.lb;
    const int wi = tt.wi, wj = tt.wj, k0 = tt.k0, k1 = tt.k1;
    const int hi = tt.hi, hj = tt.hj, hslot = tt.hslot, own = tt.own;
    auto zw = [N](int k) { return k < 0 ? k + N : (k >= N ? k - N : k); };
    const FaceTab<T>& ftr = ft;
    auto finish = [scale, omega, &ftr](const MgfRawS<T>& q) {
        MgfPtS<T> p;
        p.inv = weights_S2<T>(q.cd, ftr, p.w);
        p.b = q.b;
        p.x = omega * p.inv * q.b;
        if (p.inv > T(0)) p.x += scale * q.e;
        return p;
    };

    // two sets of raw loads alternate between the planes of an unrolled pair,
    // so no register that a load is still filling is copied at the loop's end
    MgfRawS<T> ra, rb, ha, hb;
    mgfs_load<T>(ra, N, cn, wi, wj, zw(k0 - 1), code2, b, xc);
    mgfs_load<T>(rb, N, cn, wi, wj, k0, code2, b, xc);
    const T x_first = finish(ra).x;
    mgfs_load<T>(ra, N, cn, wi, wj, zw(k0 + 1), code2, b, xc);
    if (tt.ring) mgfs_load<T>(ha, N, cn, hi, hj, k0, code2, b, xc);
    // a finished solve is checked after the first loads (in bounds either way)
    if (st && st->done) return;
    T xprev = x_first;
    MgfPtS<T> cur = finish(rb);
    double acc = 0.0;
    int buf = 0;
    // plane k: issue the loads of k + 2 (own) and k + 1 (ring), finish k + 1
    // (own) and k (ring) from the loads issued one plane earlier
    auto plane = [&](int k, const MgfRawS<T>& rfin, MgfRawS<T>& rload, const MgfRawS<T>& hfin, MgfRawS<T>& hload) {
        mgfs_load<T>(rload, N, cn, wi, wj, zw(k + 2), code2, b, xc);
        if (tt.ring) mgfs_load<T>(hload, N, cn, hi, hj, zw(k + 1), code2, b, xc);
        const MgfPtS<T> nxt = finish(rfin);
        if (tt.ring) tile[buf][hslot] = finish(hfin).x;
        tile[buf][own] = cur.x;
        __syncthreads();
        const T* tl = tile[buf];
        const T v[7] = {cur.x, tl[own - 1], tl[own + 1], tl[own - W], tl[own + W], xprev, nxt.x};
        const T ax = apply_S_w<T>(v, cur.w);
        const T yv = cur.inv > T(0) ? v[0] + omega * cur.inv * (cur.b - ax) : T(0);
        if (tt.valid) {
            out[wi + N * (wj + N * k)] = yv;
            acc += (double)cur.b * (double)yv;
        }
        xprev = cur.x;
        cur = nxt;
        buf ^= 1;
    };
    int k = k0;
    for (; k + 1 < k1; k += 2) {
        plane(k, ra, rb, ha, hb);
        plane(k + 1, rb, ra, hb, ha);
    }
    if (k < k1) plane(k, ra, rb, ha, hb);
    double v1[1] = {acc};
    write_partials<1>(v1, part, slot, lb);
}

// The inner CG update fused with the level-0 restriction that follows it:
// alpha from the stencil's partials, x += alpha d, rout = rin - alpha q, and
// bc = P^T (rout - A x0), x0 = omega D^-1 rout, in one LDS-tiled sweep (the
// updated residual is formed at every tile and ring point from rin and q).
// rin and rout are different buffers: blocks read rin at their ring points
// while neighbouring blocks write their own points.
// Partials of (r, D^-1 r) and (D^-1 r, D^-1 r) go to the RZ and ZZ slots as the
// plain update's do.  Sweep: even z-runs and the stencil's block count (its
// partials are re-added here).
// The loads of a point (code, the SIMPLE matrix's 1/D, r and q of each plane),
// apart from the arithmetic that needs alpha, so a kernel can issue its first
// points' loads before it reduces alpha.
template <class T, int KIND>
struct MgfRaw {
    static constexpr int NB = MgfPt<T, KIND>::NB;
    int cd;
    T inv0;
    T r[NB], q[NB];
};

template <class T, int KIND>
__device__ __forceinline__ void mgf_load_upd(MgfRaw<T, KIND>& w, int N, int i, int j, int k,
                                             const uint8_t* __restrict__ code, const T* __restrict__ invd,
                                             const T* __restrict__ r, const T* __restrict__ qv) {
    constexpr int NB = MgfPt<T, KIND>::NB;
    const int X = i + N * (j + N * k);
    const size_t n3 = (size_t)N * N * N;
    w.cd = code[X];
    w.inv0 = KIND == kMgFineShat ? invd[X] : T(0);
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        w.r[a] = r[a * n3 + X];
        w.q[a] = qv[a * n3 + X];
    }
}

template <class T, int KIND>
__device__ __forceinline__ void mgf_finish_upd(MgfPt<T, KIND>& q, const MgfRaw<T, KIND>& w, T alpha, T omega,
                                               const FaceTab<T>& ft) {
    constexpr int NB = MgfPt<T, KIND>::NB;
    q.cd = w.cd;
    if (KIND == kMgFineShat) q.inv[0] = w.inv0;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        if (KIND == kMgFineA) q.inv[a] = ft.inv[a][q.cd];
        q.b[a] = w.r[a] - alpha * w.q[a];
        q.x[a] = omega * q.inv[a] * q.b[a];
    }
}

template <class T, int KIND>
__device__ __forceinline__ void mgf_point_upd(MgfPt<T, KIND>& q, int N, int i, int j, int k,
                                              const uint8_t* __restrict__ code, const T* __restrict__ invd,
                                              const T* __restrict__ r, const T* __restrict__ qv, T alpha, T omega,
                                              const FaceTab<T>& ft) {
    MgfRaw<T, KIND> w;
    mgf_load_upd<T, KIND>(w, N, i, j, k, code, invd, r, qv);
    mgf_finish_upd<T, KIND>(q, w, alpha, omega, ft);
}

template <class T, int KIND>
__global__ void __launch_bounds__(kBlock) k_mgf_update_restrict(Sweep s, const uint8_t* __restrict__ code,
                                                                const T* __restrict__ invd, T* __restrict__ x,
                                                                const T* __restrict__ r, T* __restrict__ rout,
                                                                const T* __restrict__ d, const T* __restrict__ q,
                                                                T* __restrict__ bc, T omega, CgState* st,
                                                                double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code, x, r, rout, d, q, bc, st, part);
    shift_all((size_t)blockIdx.y * s.bstride, invd);
    constexpr int NB = MgfPt<T, KIND>::NB;
    __shared__ T tile[2][NB][kTileMax];
    __shared__ T pair_lds[NB * kBlock / 2];
    __shared__ FaceTab<T> ft;
    const size_t n3 = (size_t)s.n3;
    const Tile tt = tile_of(s);
    const int N = tt.N, W = tt.W, lb = tt.lb;
    const int gi = tt.gi, gj = tt.gj, wi = tt.wi, wj = tt.wj, k0 = tt.k0, k1 = tt.k1;
    const bool valid = tt.valid;
    const int hi = tt.hi, hj = tt.hj, hslot = tt.hslot, own = tt.own;
    auto zw = [N](int k) { return k < 0 ? k + N : (k >= N ? k - N : k); };
    // the first two planes' loads go out before alpha is reduced (in bounds
    // whether or not the solve has finished)
    MgfRaw<T, KIND> wprev, wcur;
    mgf_load_upd<T, KIND>(wprev, N, wi, wj, zw(k0 - 1), code, invd, r, q);
    mgf_load_upd<T, KIND>(wcur, N, wi, wj, k0, code, invd, r, q);
    if (st->done) return;
    double alpha_d;
    if (cg_update_scalars(st, part, s.nblk, &alpha_d)) return;
    const T alpha = (T)alpha_d;
    face_tab_fill<T>(ft);
    __syncthreads();

    MgfPt<T, KIND> cur, nxt;
    T xprev[NB];
    {
        MgfPt<T, KIND> pv;
        mgf_finish_upd<T, KIND>(pv, wprev, alpha, omega, ft);
#pragma unroll
        for (int a = 0; a < NB; ++a) xprev[a] = pv.x[a];
    }
    mgf_finish_upd<T, KIND>(cur, wcur, alpha, omega, ft);
    double acc[2] = {0.0, 0.0};
    T rsum[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) rsum[a] = T(0);
    int buf = 0;
    for (int k = k0; k < k1; ++k) {
        mgf_point_upd<T, KIND>(nxt, N, wi, wj, zw(k + 1), code, invd, r, q, alpha, omega, ft);
        if (tt.ring) {
            MgfPt<T, KIND> hp;
            mgf_point_upd<T, KIND>(hp, N, hi, hj, k, code, invd, r, q, alpha, omega, ft);
#pragma unroll
            for (int a = 0; a < NB; ++a) tile[buf][a][hslot] = hp.x[a];
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) tile[buf][a][own] = cur.x[a];
        int cxp = 0, cyp = 0;
        if (KIND == kMgFineShat) {
            const int X = wi + N * (wj + N * k);
            cxp = code[X - wi + (wi == N - 1 ? 0 : wi + 1)];
            cyp = code[X + (wj == N - 1 ? -(N - 1) * N : N)];
        }
        // own point: the CG update proper
        if (valid) {
            const size_t X = (size_t)wi + (size_t)N * (wj + (size_t)N * k);
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                const size_t F = a * n3 + X;
                x[F] = x[F] + alpha * d[F];
                rout[F] = cur.b[a];
                const T z = cur.b[a] * cur.inv[a];
                acc[0] += (double)cur.b[a] * (double)z;
                acc[1] += (double)z * (double)z;
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const T* tl = tile[buf][a];
            const T v[7] = {cur.x[a], tl[own - 1], tl[own + 1], tl[own - W], tl[own + W], xprev[a], nxt.x[a]};
            rsum[a] += cur.b[a] - mgf_apply<T, KIND>(v, cur.cd, cxp, cyp, nxt.cd, a, ft);
        }
        if (k & 1) {
            const int cN = N >> 1;
            mg_pair_sum<T, NB>(rsum, s.bxlog, pair_lds);
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                if (valid && !(gi & 1) && !(gj & 1))
                    bc[(size_t)a * cN * cN * cN + (gi >> 1) + cN * ((gj >> 1) + cN * (k >> 1))] = rsum[a];
                rsum[a] = T(0);
            }
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) xprev[a] = cur.x[a];
        cur = nxt;
        buf ^= 1;
    }
    write_partials<2>(acc, part, kRZ, lb);
}

// The SIMPLE matrix's fused CG update and level-0 restriction
// (k_mgf_update_restrict<T, kMgFineShat>) with its stencil loads
// software-pipelined as in k_mgf_smooth_S_pipe: at plane k a thread issues the
// loads of its own column at k + 2 (code, 1/D, r, q) and of its ring point at
// k + 1, and finishes the values loaded one plane earlier.  x and d are read
// where the update uses them
// (measured at 256^3: x and d two planes ahead made this sweep slower).  Same arithmetic as the unpipelined
// kernel, point by point.
template <class T>
struct MgfRawU {
    int cd;
    T r, q;
};

template <class T>
__device__ __forceinline__ void mgfu_load(MgfRawU<T>& w, int X, const uint16_t* __restrict__ code2,
                                          const T* __restrict__ r, const T* __restrict__ q) {
    w.cd = code2[X];
    w.r = r[X];
    w.q = q[X];
}

template <class T>
__device__ __forceinline__ MgfPtS<T> mgfu_finish(const MgfRawU<T>& w, T alpha, T omega, const FaceTab<T>& ft) {
    MgfPtS<T> p;
    p.inv = weights_S2<T>(w.cd, ft, p.w);
    p.b = w.r - alpha * w.q;
    p.x = omega * p.inv * p.b;
    return p;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_mgf_update_restrict_S_pipe(Sweep s, const uint16_t* __restrict__ code2,
                                                                       T* __restrict__ x, const T* __restrict__ r,
                                                                       T* __restrict__ rout, const T* __restrict__ d,
                                                                       const T* __restrict__ q, T* __restrict__ bc,
                                                                       T omega, CgState* st, double* part) {
    shift_nn((size_t)blockIdx.y * s.bstride, code2, x, r, rout, d, q, bc, st, part);
    __shared__ T tile[2][kTileMax];
    __shared__ T pair_lds[kBlock / 2];
    __shared__ FaceTab<T> ft;
    const Tile tt = tile_of(s);
    const int N = tt.N, W = tt.W, lb = tt.lb;
    const int gi = tt.gi, gj = tt.gj, wi = tt.wi, wj = tt.wj, k0 = tt.k0, k1 = tt.k1;
    const bool valid = tt.valid, ring = tt.ring;
    const int hslot = tt.hslot, own = tt.own;
    const int N2 = N * N;
    const int col = wi + N * wj, hcol = tt.hi + N * tt.hj;
    auto zw = [N](int k) { return k < 0 ? k + N : (k >= N ? k - N : k); };
    // the first planes' loads go out before alpha is reduced (in bounds
    // whether or not the solve has finished)
    MgfRawU<T> ra, rb, ha, hb;
    mgfu_load<T>(ra, col + zw(k0 - 1) * N2, code2, r, q);
    mgfu_load<T>(rb, col + k0 * N2, code2, r, q);
    if (st->done) return;
    double alpha_d;
    if (cg_update_scalars(st, part, s.nblk, &alpha_d)) return;
    const T alpha = (T)alpha_d;
    face_tab_fill<T>(ft);
    __syncthreads();
    T xprev = mgfu_finish<T>(ra, alpha, omega, ft).x;
    MgfPtS<T> cur = mgfu_finish<T>(rb, alpha, omega, ft);
    mgfu_load<T>(ra, col + zw(k0 + 1) * N2, code2, r, q);
    if (ring) mgfu_load<T>(ha, hcol + k0 * N2, code2, r, q);
    double acc[2] = {0.0, 0.0};
    T rsum = T(0);
    int buf = 0;
    // plane k: issue the loads of k + 2 (own) and k + 1 (ring), finish k + 1
    // (own) and k (ring) from the loads issued one plane earlier
    auto plane = [&](int k, const MgfRawU<T>& rfin, MgfRawU<T>& rload, const MgfRawU<T>& hfin, MgfRawU<T>& hload) {
        mgfu_load<T>(rload, col + zw(k + 2) * N2, code2, r, q);
        if (ring) mgfu_load<T>(hload, hcol + zw(k + 1) * N2, code2, r, q);
        const MgfPtS<T> nxt = mgfu_finish<T>(rfin, alpha, omega, ft);
        if (ring) tile[buf][hslot] = mgfu_finish<T>(hfin, alpha, omega, ft).x;
        tile[buf][own] = cur.x;
        // own point: the CG update proper
        if (valid) {
            const int X = col + k * N2;
            x[X] = x[X] + alpha * d[X];
            rout[X] = cur.b;
            const T z = cur.b * cur.inv;
            acc[0] += (double)cur.b * (double)z;
            acc[1] += (double)z * (double)z;
        }
        __syncthreads();
        const T* tl = tile[buf];
        const T v[7] = {cur.x, tl[own - 1], tl[own + 1], tl[own - W], tl[own + W], xprev, nxt.x};
        rsum += cur.b - apply_S_w<T>(v, cur.w);
        if (k & 1) {
            const int cN = N >> 1;
            T rs[1] = {rsum};
            mg_pair_sum<T, 1>(rs, s.bxlog, pair_lds);
            if (valid && !(gi & 1) && !(gj & 1)) bc[(gi >> 1) + cN * ((gj >> 1) + cN * (k >> 1))] = rs[0];
            rsum = T(0);
        }
        xprev = cur.x;
        cur = nxt;
        buf ^= 1;
    };
    int k = k0;
    for (; k + 1 < k1; k += 2) {
        plane(k, ra, rb, ha, hb);
        plane(k + 1, rb, ra, hb, ha);
    }
    if (k < k1) plane(k, ra, rb, ha, hb);
    write_partials<2>(acc, part, kRZ, lb);
}

// ---------------------------------------------------------------------------
// Levels >= 1 (assembled 7-point operators), one thread per node
// ---------------------------------------------------------------------------

// Coefficients, b and 1/D at the seven points of node (p; i, j, k)
template <class T>
struct MgcPoint {
    T b[7], inv[7];
    T d;            // diagonal at the node
    T w[6];         // couplings to -x, +x, -y, +y, -z, +z
};

template <class T>
__device__ __forceinline__ void mgc_load(MgcPoint<T>& m, const MgGrid& g, const MgOp& op, const T* __restrict__ b,
                                         int p, int i, int j, int k) {
    const size_t o = (size_t)p * g.n3;
    const float* D = (const float*)op.D + o;
    const float* Wx = (const float*)op.Wx + o;
    const float* Wy = (const float*)op.Wy + o;
    const float* Wz = (const float*)op.Wz + o;
    const T* bp = b + o;
    const int idx[7] = {mg_idx(g, i, j, k),     mg_idx(g, i - 1, j, k), mg_idx(g, i + 1, j, k), mg_idx(g, i, j - 1, k),
                        mg_idx(g, i, j + 1, k), mg_idx(g, i, j, k - 1), mg_idx(g, i, j, k + 1)};
    T dd[7];
#pragma unroll
    for (int t = 0; t < 7; ++t) {
        m.b[t] = bp[idx[t]];
        dd[t] = D[idx[t]];
    }
    m.w[0] = Wx[idx[0]];
    m.w[1] = Wx[idx[2]];
    m.w[2] = Wy[idx[0]];
    m.w[3] = Wy[idx[4]];
    m.w[4] = Wz[idx[0]];
    m.w[5] = Wz[idx[6]];
    m.d = dd[0];
#pragma unroll
    for (int t = 0; t < 7; ++t) m.inv[t] = dd[t] > T(0) ? T(1) / dd[t] : T(0);
}

template <class T>
__device__ __forceinline__ T mgc_apply(const MgcPoint<T>& m, const T (&v)[7]) {
    return m.d * v[0] - (((m.w[0] * v[1] + m.w[1] * v[2]) + (m.w[2] * v[3] + m.w[3] * v[4])) +
                         (m.w[4] * v[5] + m.w[5] * v[6]));
}

// bc = P^T (b - A x0), x0 = omega D^-1 b, from level l to level l+1.  The
// eight children of a coarse node sit in eight consecutive lanes (thread t:
// coarse node t / 8, child t % 8) and are summed with shuffles.
template <class T>
__global__ void k_mgc_restrict(MgGrid g, MgGrid cg, MgOp op, const T* __restrict__ b, T* __restrict__ bc, T omega,
                               const CgState* st) {
    shift_nn((size_t)blockIdx.y * g.bstride, b, bc);
    shift_all((size_t)blockIdx.y * g.bstride, st);
    shift_op(op, (size_t)blockIdx.y * g.bstride);
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int I = t >> 3, ch = t & 7;
    T r = T(0);
    if (I < cg.nb * cg.n3) {
        const int p = I / cg.n3, L = I - p * cg.n3;
        const int i = 2 * (L % cg.n) + (ch & 1), j = 2 * ((L / cg.n) % cg.n) + ((ch >> 1) & 1),
                  k = 2 * (L / cg.n2) + (ch >> 2);
        MgcPoint<T> m;
        mgc_load<T>(m, g, op, b, p, i, j, k);
        T x0[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) x0[q] = omega * m.inv[q] * m.b[q];
        r = m.b[0] - mgc_apply<T>(m, x0);
    }
    r += __shfl_xor(r, 1, 64);
    r += __shfl_xor(r, 2, 64);
    r += __shfl_xor(r, 4, 64);
    // a finished solve is checked after the loads (in bounds either way), so
    // its latency overlaps theirs; nothing is written then
    if (st && st->done) return;
    if (ch == 0 && I < cg.nb * cg.n3) bc[I] = r;
}

// y = x' + omega D^-1 (b - A x'), x' = x0 + scale * P xc, x0 = omega D^-1 b,
// on a level >= 1; nodes with D = 0 are held at 0.
template <class T>
__global__ void k_mgc_postsmooth(MgGrid g, MgOp op, const T* __restrict__ b, const T* __restrict__ xc, int cn,
                                 T scale, T omega, T* __restrict__ y, const CgState* st) {
    shift_nn((size_t)blockIdx.y * g.bstride, b, xc, y);
    shift_all((size_t)blockIdx.y * g.bstride, st);
    shift_op(op, (size_t)blockIdx.y * g.bstride);
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= g.nb * g.n3) return;
    const int p = I / g.n3, X = I - p * g.n3;
    const int i = X % g.n, j = (X / g.n) % g.n, k = X / g.n2;
    MgcPoint<T> m;
    mgc_load<T>(m, g, op, b, p, i, j, k);
    const MgParents q = mg_parents(g.n, cn, i, j, k);
    const T* xa = xc + (size_t)p * cn * cn * cn;
    const T xp[4] = {xa[q.c], xa[q.x], xa[q.y], xa[q.z]};
    T e[7], v[7];
    mg_prolong7<T>(q, xp, scale, e);
#pragma unroll
    for (int t = 0; t < 7; ++t) v[t] = omega * m.inv[t] * m.b[t] + e[t];
    const T ax = mgc_apply<T>(m, v);
    if (st && st->done) return;
    y[I] = m.inv[0] > T(0) ? v[0] + omega * m.inv[0] * (m.b[0] - ax) : T(0);
}

// ---------------------------------------------------------------------------
// Levels >= 1 below the tiled size, red-black Gauss-Seidel smoothing.  Colour
// of node (i, j, k): (i + j + k) & 1, red = 0 (such levels have an even side,
// so the colouring is periodic and a 7-point row couples only opposite
// colours).  A relaxation solves the node's row for its own value,
// x = (b + sum of W x over the six neighbours) / D, and keeps 0 where D = 0.
// Down: red, then black, from zero; up: black, then red (the adjoint order,
// so the cycle stays symmetric for CG).
// One workgroup per brick of kGsB^3 nodes of one plane.  The brick's window
// with two halo layers sits in LDS: red values from zero depend only on b, so
// they are formed over the whole window; black values then over the first
// halo layer, which is all the brick's own rows read.  Nothing crosses a
// workgroup.
// ---------------------------------------------------------------------------
constexpr int kGsB = 8;                               // brick side (even: a coarse node's children stay together)
constexpr int kGsW = kGsB + 4;                        // window side
constexpr int kGsThreads = kGsB * kGsB * kGsB;        // one interior node per thread
constexpr int kGsWin = kGsW * kGsW * kGsW;
constexpr int kGsBlack1 = (kGsB + 2) * (kGsB + 2) * (kGsB + 2) / 2;   // black nodes of brick + first layer
static_assert(kGsBlack1 <= kGsThreads, "one black node of the first layer per thread");

struct GsBrick {
    int p;          // plane
    int o[3];       // origin (global coordinates of the brick's first node)
};

__device__ __forceinline__ GsBrick gs_brick(const MgGrid& g) {
    const int nbk = (g.n + kGsB - 1) / kGsB;
    int b = blockIdx.x;
    GsBrick r;
    r.p = b / (nbk * nbk * nbk);
    b -= r.p * nbk * nbk * nbk;
    r.o[0] = (b % nbk) * kGsB;
    r.o[1] = ((b / nbk) % nbk) * kGsB;
    r.o[2] = (b / (nbk * nbk)) * kGsB;
    return r;
}

// Row of one node: b, D, 1/D and the couplings to -x, +x, -y, +y, -z, +z
template <class T>
struct GsRow {
    T b, d, inv, w[6];
};

// the row of window point (wx, wy, wz), which is global node o + w - 2, wrapped
// (the side is at least 10, so one wrap suffices)
template <class T>
__device__ __forceinline__ void gs_row(GsRow<T>& r, const MgGrid& g, const MgOp& op, const T* __restrict__ b,
                                       const GsBrick& k, int wx, int wy, int wz) {
    const size_t o = (size_t)k.p * g.n3;
    const int i = wrapc(k.o[0] + wx - 2, g.n), j = wrapc(k.o[1] + wy - 2, g.n), kk = wrapc(k.o[2] + wz - 2, g.n);
    const int X = i + g.n * (j + g.n * kk);
    const float* D = (const float*)op.D + o;
    const float* Wx = (const float*)op.Wx + o;
    const float* Wy = (const float*)op.Wy + o;
    const float* Wz = (const float*)op.Wz + o;
    r.b = b[o + X];
    r.d = D[X];
    r.w[0] = Wx[X];
    r.w[1] = Wx[mg_idx(g, i + 1, j, kk)];
    r.w[2] = Wy[X];
    r.w[3] = Wy[mg_idx(g, i, j + 1, kk)];
    r.w[4] = Wz[X];
    r.w[5] = Wz[mg_idx(g, i, j, kk + 1)];
    r.inv = r.d > T(0) ? T(1) / r.d : T(0);
}

// sum of W x over the six neighbours of window point w
template <class T>
__device__ __forceinline__ T gs_nbsum(const GsRow<T>& r, const T* x, int w) {
    constexpr int sy = kGsW, sz = kGsW * kGsW;
    return ((r.w[0] * x[w - 1] + r.w[1] * x[w + 1]) + (r.w[2] * x[w - sy] + r.w[3] * x[w + sy])) +
           (r.w[4] * x[w - sz] + r.w[5] * x[w + sz]);
}

// Interior node of thread t: the eight children of a coarse node in eight
// consecutive lanes (bit 0: x, 1: y, 2: z), coarse nodes of the brick 4 x 4 x 4.
__device__ __forceinline__ void gs_interior(int t, int& lx, int& ly, int& lz) {
    const int ch = t & 7, cb = t >> 3;
    lx = 2 * (cb & 3) + (ch & 1);
    ly = 2 * ((cb >> 2) & 3) + ((ch >> 1) & 1);
    lz = 2 * (cb >> 4) + (ch >> 2);
}

// Black node q < kGsBlack1 of the brick plus its first halo layer (window
// coordinates 1 .. kGsB + 2): five per row of ten, x chosen by row parity.
__device__ __forceinline__ void gs_black1(int q, int& wx, int& wy, int& wz) {
    constexpr int half = (kGsB + 2) / 2;
    wz = 1 + q / (half * (kGsB + 2));
    wy = 1 + (q / half) % (kGsB + 2);
    wx = 1 + 2 * (q % half) + ((wy + wz) & 1);
}

constexpr int kGsPer = (kGsWin + kGsThreads - 1) / kGsThreads;   // window points per thread

__device__ __forceinline__ bool gs_red(int w) {
    return (((w % kGsW) + ((w / kGsW) % kGsW) + w / (kGsW * kGsW)) & 1) == 0;
}

// b and D (and, for the post-smoothing, the parent's coarse correction) at the
// red window points w = threadIdx.x + q * kGsThreads; black points and points
// past the window load nothing.
template <class T, bool POST>
__device__ __forceinline__ void gs_window_loads(const MgGrid& g, const GsBrick& k, const MgOp& op,
                                                const T* __restrict__ b, const T* __restrict__ xc, int cn,
                                                T (&bv)[kGsPer], T (&dv)[kGsPer], T* ev) {
    const float* D = (const float*)op.D + (size_t)k.p * g.n3;
    const T* bp = b + (size_t)k.p * g.n3;
    const T* xa = POST ? xc + (size_t)k.p * cn * cn * cn : nullptr;
#pragma unroll
    for (int q = 0; q < kGsPer; ++q) {
        const int w = (int)threadIdx.x + q * kGsThreads;
        bv[q] = T(0);
        dv[q] = T(0);
        if (POST) ev[q] = T(0);
        if (w < kGsWin && gs_red(w)) {
            const int wx = w % kGsW, wy = (w / kGsW) % kGsW, wz = w / (kGsW * kGsW);
            const int i = wrapc(k.o[0] + wx - 2, g.n), j = wrapc(k.o[1] + wy - 2, g.n),
                      kk = wrapc(k.o[2] + wz - 2, g.n);
            const int X = i + g.n * (j + g.n * kk);
            bv[q] = bp[X];
            dv[q] = D[X];
            if (POST) ev[q] = xa[(i >> 1) + cn * ((j >> 1) + cn * (kk >> 1))];
        }
    }
}

// bc = P^T (b - A x), x = the red-then-black relaxation of A x = b from zero.
template <class T>
__global__ void __launch_bounds__(kGsThreads) k_mgc_gs_restrict(MgGrid g, MgGrid cg, MgOp op,
                                                                const T* __restrict__ b, T* __restrict__ bc,
                                                                const CgState* st) {
    shift_nn((size_t)blockIdx.y * g.bstride, b, bc);
    shift_all((size_t)blockIdx.y * g.bstride, st);
    shift_op(op, (size_t)blockIdx.y * g.bstride);
    __shared__ T sx[kGsWin];
    const GsBrick k = gs_brick(g);
    const int t = threadIdx.x;
    // every load is issued before the first store: the window's red points
    // first (the first phase needs them), then the rows of this thread's nodes
    T bv[kGsPer], dv[kGsPer];
    gs_window_loads<T, false>(g, k, op, b, nullptr, 0, bv, dv, nullptr);
    int lx, ly, lz;
    gs_interior(t, lx, ly, lz);
    const bool inside = k.o[0] + lx < g.n && k.o[1] + ly < g.n && k.o[2] + lz < g.n;
    const bool has_black = t < kGsBlack1;
    int bx = 1, by = 1, bz = 1;
    if (has_black) gs_black1(t, bx, by, bz);
    GsRow<T> ri, rb;
    if (inside) gs_row(ri, g, op, b, k, lx + 2, ly + 2, lz + 2);
    if (has_black) gs_row(rb, g, op, b, k, bx, by, bz);
    // a finished solve is checked after the loads (in bounds either way)
    if (st && st->done) return;
    // red values over the window (black ones are written below where read)
#pragma unroll
    for (int q = 0; q < kGsPer; ++q) {
        const int w = t + q * kGsThreads;
        if (w < kGsWin) sx[w] = gs_red(w) ? (dv[q] > T(0) ? T(1) / dv[q] : T(0)) * bv[q] : T(0);
    }
    __syncthreads();
    if (has_black) {
        const int w = bx + kGsW * (by + kGsW * bz);
        sx[w] = rb.inv * (rb.b + gs_nbsum(rb, sx, w));
    }
    __syncthreads();
    T r = T(0);
    if (inside) {
        const int w = (lx + 2) + kGsW * ((ly + 2) + kGsW * (lz + 2));
        r = ri.b - (ri.d * sx[w] - gs_nbsum(ri, sx, w));
    }
    r += __shfl_xor(r, 1, 64);
    r += __shfl_xor(r, 2, 64);
    r += __shfl_xor(r, 4, 64);
    if ((t & 7) == 0 && inside) {
        const int ci = (k.o[0] >> 1) + (lx >> 1), cj = (k.o[1] >> 1) + (ly >> 1), ck = (k.o[2] >> 1) + (lz >> 1);
        bc[(size_t)k.p * cg.n3 + ci + cg.n * (cj + cg.n * ck)] = r;
    }
}

// y = the black-then-red relaxation of A y = b starting from x' = x + scale P xc,
// x = the red-then-black relaxation from zero (its black values are not
// needed: a black relaxation overwrites them).
template <class T>
__global__ void __launch_bounds__(kGsThreads) k_mgc_gs_postsmooth(MgGrid g, MgOp op, const T* __restrict__ b,
                                                                  const T* __restrict__ xc, int cn, T scale,
                                                                  T* __restrict__ y, const CgState* st) {
    shift_nn((size_t)blockIdx.y * g.bstride, b, xc, y);
    shift_all((size_t)blockIdx.y * g.bstride, st);
    shift_op(op, (size_t)blockIdx.y * g.bstride);
    __shared__ T sx[kGsWin];
    const GsBrick k = gs_brick(g);
    const int t = threadIdx.x;
    T bv[kGsPer], dv[kGsPer], ev[kGsPer];
    gs_window_loads<T, true>(g, k, op, b, xc, cn, bv, dv, ev);
    int lx, ly, lz;
    gs_interior(t, lx, ly, lz);
    const bool inside = k.o[0] + lx < g.n && k.o[1] + ly < g.n && k.o[2] + lz < g.n;
    const bool has_black = t < kGsBlack1;
    int bx = 1, by = 1, bz = 1;
    if (has_black) gs_black1(t, bx, by, bz);
    GsRow<T> ri, rb;
    if (inside) gs_row(ri, g, op, b, k, lx + 2, ly + 2, lz + 2);
    if (has_black) gs_row(rb, g, op, b, k, bx, by, bz);
    if (st && st->done) return;
#pragma unroll
    for (int q = 0; q < kGsPer; ++q) {
        const int w = t + q * kGsThreads;
        if (w < kGsWin)
            sx[w] = gs_red(w) ? (dv[q] > T(0) ? T(1) / dv[q] : T(0)) * bv[q] + scale * ev[q] : T(0);
    }
    __syncthreads();
    if (has_black) {
        const int w = bx + kGsW * (by + kGsW * bz);
        sx[w] = rb.inv * (rb.b + gs_nbsum(rb, sx, w));
    }
    __syncthreads();
    if (inside) {
        const int w = (lx + 2) + kGsW * ((ly + 2) + kGsW * (lz + 2));
        const T v = ((lx + ly + lz) & 1) ? sx[w] : ri.inv * (ri.b + gs_nbsum(ri, sx, w));
        y[(size_t)k.p * g.n3 + (k.o[0] + lx) + g.n * ((k.o[1] + ly) + g.n * (k.o[2] + lz))] = v;
    }
}

// Levels >= 1 with a side of at least 64, LDS-tiled like level 0: the
// iterate x once per point, own column k-1, k, k+1 in registers, plane k plus a
// ring in LDS.  The couplings to +x and +y are read from the neighbour's W^x,
// W^y; the one to +z is the next plane's own W^z.  s: a sweep over this level
// (even z-runs).  MODE:
//   kMgcPre      x = omega D^-1 b; the residual b - A x summed over 2x2x2 into out (level + 1)
//   kMgcPost     x = omega D^-1 b + scale P xc; out = x + omega D^-1 (b - A x)
//   kMgcPostAcc  as kMgcPost, added to what out holds (the second of two visits)
//   kMgcResid    x = xc (an iterate of this level); out = b - A x
// Nodes that are not unknowns (D = 0) get 0 in the post and residual forms.
constexpr int kMgcPre = 0, kMgcPost = 1, kMgcPostAcc = 2, kMgcResid = 3;

template <class T, int NB>
struct MgcPt {
    T d[NB], b[NB], x[NB], wz[NB];
};

template <class T, int NB, int MODE>
__device__ __forceinline__ void mgc_point(MgcPt<T, NB>& q, int n, int cn, int i, int j, int k, const MgOp& op,
                                          const T* __restrict__ b, const T* __restrict__ xc, T scale, T omega) {
    constexpr bool POST = MODE == kMgcPost || MODE == kMgcPostAcc;
    const size_t n3 = (size_t)n * n * n;
    const int X = i + n * (j + n * k);
    const float* D = (const float*)op.D;
    const float* Wz = (const float*)op.Wz;
    T e[NB];
    if (POST) {
        const size_t cn3 = (size_t)cn * cn * cn;
        const int C = (i >> 1) + cn * ((j >> 1) + cn * (k >> 1));
#pragma unroll
        for (int a = 0; a < NB; ++a) e[a] = xc[a * cn3 + C];
    }
    if (MODE == kMgcResid) {
#pragma unroll
        for (int a = 0; a < NB; ++a) e[a] = xc[a * n3 + X];
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        q.d[a] = D[a * n3 + X];
        q.b[a] = b[a * n3 + X];
        q.wz[a] = Wz[a * n3 + X];
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        if (MODE == kMgcResid) {
            q.x[a] = e[a];
        } else {
            const T inv = q.d[a] > T(0) ? T(1) / q.d[a] : T(0);
            q.x[a] = omega * inv * q.b[a];
            if (POST) q.x[a] += scale * e[a];
        }
    }
}

template <class T, int NB, int MODE>
__global__ void __launch_bounds__(kBlock) k_mgc_tiled(Sweep s, int cn, MgOp op, const T* __restrict__ b,
                                                      const T* __restrict__ xc, T scale, T omega, T* __restrict__ out,
                                                      const CgState* st) {
    constexpr bool PRE = MODE == kMgcPre;
    shift_nn((size_t)blockIdx.y * s.bstride, b, out);
    shift_all((size_t)blockIdx.y * s.bstride, xc, st);
    shift_op(op, (size_t)blockIdx.y * s.bstride);
    __shared__ T tile[2][NB][kTileMax];
    __shared__ T pair_lds[PRE ? NB * kBlock / 2 : 1];
    const Tile t = tile_of(s);
    const int n = t.N, W = t.W;
    const size_t n3 = (size_t)s.n3;
    const float* Wx = (const float*)op.Wx;
    const float* Wy = (const float*)op.Wy;
    auto zw = [n](int k) { return k < 0 ? k + n : (k >= n ? k - n : k); };
    MgcPt<T, NB> cur, nxt;
    T xprev[NB];
    {
        MgcPt<T, NB> pv;
        mgc_point<T, NB, MODE>(pv, n, cn, t.wi, t.wj, zw(t.k0 - 1), op, b, xc, scale, omega);
#pragma unroll
        for (int a = 0; a < NB; ++a) xprev[a] = pv.x[a];
    }
    mgc_point<T, NB, MODE>(cur, n, cn, t.wi, t.wj, t.k0, op, b, xc, scale, omega);
    // a finished solve is checked after the first loads (in bounds either way)
    if (st && st->done) return;
    T rsum[NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) rsum[a] = T(0);
    const int xp = t.wi == n - 1 ? 0 : t.wi + 1, yp = t.wj == n - 1 ? 0 : t.wj + 1;
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k) {
        mgc_point<T, NB, MODE>(nxt, n, cn, t.wi, t.wj, zw(k + 1), op, b, xc, scale, omega);
        if (t.ring) {
            MgcPt<T, NB> hp;
            mgc_point<T, NB, MODE>(hp, n, cn, t.hi, t.hj, k, op, b, xc, scale, omega);
#pragma unroll
            for (int a = 0; a < NB; ++a) tile[buf][a][t.hslot] = hp.x[a];
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) tile[buf][a][t.own] = cur.x[a];
        const int X = t.wi + n * (t.wj + n * k);
        const int Xxp = xp + n * (t.wj + n * k), Xyp = t.wi + n * (yp + n * k);
        T wx[NB], wxp[NB], wy[NB], wyp[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            wx[a] = Wx[a * n3 + X];
            wxp[a] = Wx[a * n3 + Xxp];
            wy[a] = Wy[a * n3 + X];
            wyp[a] = Wy[a * n3 + Xyp];
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NB; ++a) {
            const T* tl = tile[buf][a];
            const T ax = cur.d[a] * cur.x[a] - (((wx[a] * tl[t.own - 1] + wxp[a] * tl[t.own + 1]) +
                                                 (wy[a] * tl[t.own - W] + wyp[a] * tl[t.own + W])) +
                                                (cur.wz[a] * xprev[a] + nxt.wz[a] * nxt.x[a]));
            if (MODE == kMgcPost || MODE == kMgcPostAcc) {
                const T inv = cur.d[a] > T(0) ? T(1) / cur.d[a] : T(0);
                if (t.valid) {
                    const T y = inv > T(0) ? cur.x[a] + omega * inv * (cur.b[a] - ax) : T(0);
                    out[a * n3 + X] = MODE == kMgcPostAcc ? out[a * n3 + X] + y : y;
                }
            } else if (MODE == kMgcResid) {
                if (t.valid) out[a * n3 + X] = cur.d[a] > T(0) ? cur.b[a] - ax : T(0);
            } else {
                rsum[a] += cur.b[a] - ax;
            }
        }
        if (PRE && (k & 1)) {
            mg_pair_sum<T, NB>(rsum, s.bxlog, pair_lds);
            const size_t cn3 = (size_t)cn * cn * cn;
#pragma unroll
            for (int a = 0; a < NB; ++a) {
                if (t.valid && !(t.gi & 1) && !(t.gj & 1))
                    out[a * cn3 + (t.gi >> 1) + cn * ((t.gj >> 1) + cn * (k >> 1))] = rsum[a];
                rsum[a] = T(0);
            }
        }
#pragma unroll
        for (int a = 0; a < NB; ++a) xprev[a] = cur.x[a];
        cur = nxt;
        buf ^= 1;
    }
}

// Coarsest level: `sweeps` damped-Jacobi sweeps from zero inside one workgroup
// (x in LDS, double-buffered).  Each thread keeps the coefficients and
// neighbour indices of its nodes in registers, so a sweep touches only LDS.
// nb * n3 <= kMgCoarsestMax, at most kMgCoarsestPer nodes per thread.
constexpr int kMgCoarsestMax = 2048;
constexpr int kMgCoarsestThreads = 1024;
constexpr int kMgCoarsestPer = kMgCoarsestMax / kMgCoarsestThreads;

template <class T>
__global__ void k_mg_coarsest(MgGrid g, MgOp op, const T* __restrict__ b, T* __restrict__ xout, T omega, int sweeps,
                              const CgState* st) {
    shift_nn((size_t)blockIdx.y * g.bstride, b, xout);
    shift_all((size_t)blockIdx.y * g.bstride, st);
    shift_op(op, (size_t)blockIdx.y * g.bstride);
    __shared__ T xs[2][kMgCoarsestMax];
    const int n = g.nb * g.n3;
    // per node: omega/D, b, the six couplings and the six neighbour slots
    T wd[kMgCoarsestPer], bb[kMgCoarsestPer], w[kMgCoarsestPer][6], dg[kMgCoarsestPer];
    int nbr[kMgCoarsestPer][6];
#pragma unroll
    for (int q = 0; q < kMgCoarsestPer; ++q) {
        const int I = threadIdx.x + q * kMgCoarsestThreads;
        const int Ic = I < n ? I : 0;
        const int p = Ic / g.n3, X = Ic - p * g.n3;
        const int i = X % g.n, j = (X / g.n) % g.n, k = X / g.n2;
        const int base = p * g.n3;
        nbr[q][0] = base + mg_idx(g, i - 1, j, k);
        nbr[q][1] = base + mg_idx(g, i + 1, j, k);
        nbr[q][2] = base + mg_idx(g, i, j - 1, k);
        nbr[q][3] = base + mg_idx(g, i, j + 1, k);
        nbr[q][4] = base + mg_idx(g, i, j, k - 1);
        nbr[q][5] = base + mg_idx(g, i, j, k + 1);
        // the coarsest level is always an assembled (coarse) level
        const float* D = (const float*)op.D;
        const float* Wx = (const float*)op.Wx;
        const float* Wy = (const float*)op.Wy;
        const float* Wz = (const float*)op.Wz;
        dg[q] = D[Ic];
        w[q][0] = Wx[Ic];
        w[q][1] = Wx[nbr[q][1]];
        w[q][2] = Wy[Ic];
        w[q][3] = Wy[nbr[q][3]];
        w[q][4] = Wz[Ic];
        w[q][5] = Wz[nbr[q][5]];
        wd[q] = dg[q] > T(0) ? omega / dg[q] : T(0);
        bb[q] = b[Ic];
    }
    // a finished solve is checked after the loads (in bounds either way)
    if (st && st->done) return;
#pragma unroll
    for (int q = 0; q < kMgCoarsestPer; ++q) {
        const int I = threadIdx.x + q * kMgCoarsestThreads;
        if (I < n) xs[0][I] = wd[q] * bb[q];
    }
    __syncthreads();
    int cur = 0;
    for (int it = 1; it < sweeps; ++it) {
#pragma unroll
        for (int q = 0; q < kMgCoarsestPer; ++q) {
            const int I = threadIdx.x + q * kMgCoarsestThreads;
            if (I >= n) continue;
            const T* x = xs[cur];
            const T ax = dg[q] * x[I] - (((w[q][0] * x[nbr[q][0]] + w[q][1] * x[nbr[q][1]]) +
                                          (w[q][2] * x[nbr[q][2]] + w[q][3] * x[nbr[q][3]])) +
                                         (w[q][4] * x[nbr[q][4]] + w[q][5] * x[nbr[q][5]]));
            xs[cur ^ 1][I] = x[I] + wd[q] * (bb[q] - ax);
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int I = threadIdx.x; I < n; I += kMgCoarsestThreads) xout[I] = xs[cur][I];
}

// Per-block partials of (a, b), (a, c), (b, b) over n values, written as
// part[3 * block + q] (the power iteration of the two-visit estimate; plain
// contexts only)
__global__ void __launch_bounds__(kBlock) k_dots3_flat(int n, const double* __restrict__ a,
                                                       const double* __restrict__ b, const double* __restrict__ c,
                                                       double* __restrict__ part) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < n; X += gridDim.x * blockDim.x) {
        const double av = a[X], bv = b[X];
        v[0] += av * bv;
        v[1] += av * c[X];
        v[2] += bv * bv;
    }
    block_sum_all<3>(v);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[3 * blockIdx.x + q] = v[q];
}

// out = s * in, flat
__global__ void k_scale_flat(int n, const double* __restrict__ in, double s, double* __restrict__ out) {
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < n; X += gridDim.x * blockDim.x) out[X] = s * in[X];
}

// out = (float) in, flat
__global__ void k_narrow_flat(int n, const double* __restrict__ in, float* __restrict__ out, size_t bstride) {
    shift_nn((size_t)blockIdx.y * bstride, in, out);
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < n; X += gridDim.x * blockDim.x) out[X] = (float)in[X];
}

}  // namespace stokes
