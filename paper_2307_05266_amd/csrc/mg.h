// Geometric multigrid V-cycle for the SIMPLE matrix Shat = B diag(A)^-1 B^T,
// used as the preconditioner of the inner CG solve (the paper preconditions its
// inner solves with algebraic multigrid, Sec. 3.2).
//
// Hierarchy: level 0 is the voxel grid, applied matrix-free from the face
// codes; level l+1 aggregates 2x2x2 blocks of level l (piecewise-constant
// prolongation P, restriction P^T) and holds the Galerkin operator P^T A_l P.
// For a 7-point operator that operator is again 7-point, stored per node as its
// diagonal D and the couplings W^x, W^y, W^z to the -x, -y, -z neighbours
// (entries of the matrix are -W):
//   D_I   = sum of the children's diagonals - 2 * (couplings inside the block)
//   W^c_I = sum of the couplings of the four children on the block's -c face
// to the neighbouring block.
//
// V-cycle (symmetric, hence a valid CG preconditioner): on each level one
// damped-Jacobi sweep from zero, residual restricted to the next level,
// coarse correction prolonged and scaled, one damped-Jacobi sweep; the
// coarsest level runs a fixed number of Jacobi sweeps inside one workgroup.
#pragma once

#include "kernels.h"

namespace stokes {

// Level geometry: n nodes per side; flat index i + n (j + n k), periodic.
struct MgGrid {
    int n, n2, n3;
};

__device__ __forceinline__ int wrapc(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int mg_idx(const MgGrid& g, int i, int j, int k) {
    return wrapc(i, g.n) + g.n * (wrapc(j, g.n) + g.n * wrapc(k, g.n));
}

// ---------------------------------------------------------------------------
// Level-0 couplings from the face codes: W^c(X) = 1 / diag(A) of the face
// (c, X) between X - e_c and X when it is an unknown, else 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fine_w(const uint8_t* __restrict__ code, const MgGrid& g, int i, int j, int k, int c) {
    const int cd = code[mg_idx(g, i, j, k)];
    return inv_diag_A(c == 0 ? sx_of(cd) : (c == 1 ? sy_of(cd) : sz_of(cd)));
}

// Build level 1 from the codes.  One thread per coarse node.  (Setup only.)
template <class T>
__global__ void k_mg_coarsen_fine(MgGrid fg, MgGrid cg, const uint8_t* __restrict__ code, T* __restrict__ D,
                                  T* __restrict__ Wx, T* __restrict__ Wy, T* __restrict__ Wz) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= cg.n3) return;
    const int ci = I % cg.n, cj = (I / cg.n) % cg.n, ck = I / cg.n2;
    double diag = 0.0, inner = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const int i = 2 * ci + a, j = 2 * cj + b, k = 2 * ck + c;
                const double w0 = fine_w(code, fg, i, j, k, 0), w1 = fine_w(code, fg, i, j, k, 1),
                             w2 = fine_w(code, fg, i, j, k, 2);
                diag += (w0 + fine_w(code, fg, i + 1, j, k, 0)) + (w1 + fine_w(code, fg, i, j + 1, k, 1)) +
                        (w2 + fine_w(code, fg, i, j, k + 1, 2));
                if (a == 1) inner += w0; else wx += w0;
                if (b == 1) inner += w1; else wy += w1;
                if (c == 1) inner += w2; else wz += w2;
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
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= cg.n3) return;
    const int ci = I % cg.n, cj = (I / cg.n) % cg.n, ck = I / cg.n2;
    double diag = 0.0, inner = 0.0, wx = 0.0, wy = 0.0, wz = 0.0;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                const int f = mg_idx(fg, 2 * ci + a, 2 * cj + b, 2 * ck + c);
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

// Operator pieces at a node.
struct MgOp {
    // level 0 (matrix-free from codes) when code != nullptr
    const uint8_t* code;
    const void* invd;   // level 0: inverse diagonal (T)
    const void* D;      // levels >= 1
    const void* Wx;
    const void* Wy;
    const void* Wz;
};

// (A x)_node and 1/D at node (i, j, k) of a level.
template <class T>
__device__ __forceinline__ T mg_apply(const MgGrid& g, const MgOp& op, const T* __restrict__ x, int i, int j, int k,
                                      T* inv_diag) {
    const int X = mg_idx(g, i, j, k);
    const int xm = mg_idx(g, i - 1, j, k), xp = mg_idx(g, i + 1, j, k);
    const int ym = mg_idx(g, i, j - 1, k), yp = mg_idx(g, i, j + 1, k);
    const int zm = mg_idx(g, i, j, k - 1), zp = mg_idx(g, i, j, k + 1);
    const T xX = x[X];
    if (op.code) {
        const int cX = op.code[X];
        const T wxl = inv_diag_A_t<T>(sx_of(cX)), wyl = inv_diag_A_t<T>(sy_of(cX)), wzl = inv_diag_A_t<T>(sz_of(cX));
        const T wxh = inv_diag_A_t<T>(sx_of(op.code[xp])), wyh = inv_diag_A_t<T>(sy_of(op.code[yp])),
                wzh = inv_diag_A_t<T>(sz_of(op.code[zp]));
        *inv_diag = ((const T*)op.invd)[X];
        return ((wxl * (xX - x[xm]) + wxh * (xX - x[xp])) + (wyl * (xX - x[ym]) + wyh * (xX - x[yp]))) +
               (wzl * (xX - x[zm]) + wzh * (xX - x[zp]));
    }
    const T* D = (const T*)op.D;
    const T* Wx = (const T*)op.Wx;
    const T* Wy = (const T*)op.Wy;
    const T* Wz = (const T*)op.Wz;
    const T d = D[X];
    *inv_diag = d > T(0) ? T(1) / d : T(0);
    return d * xX - (((Wx[X] * x[xm] + Wx[xp] * x[xp]) + (Wy[X] * x[ym] + Wy[yp] * x[yp])) +
                     (Wz[X] * x[zm] + Wz[zp] * x[zp]));
}

template <class T>
__device__ __forceinline__ T mg_inv_diag(const MgGrid& g, const MgOp& op, int X) {
    if (op.code) return ((const T*)op.invd)[X];
    const T d = ((const T*)op.D)[X];
    return d > T(0) ? T(1) / d : T(0);
}

// x = omega D^-1 b (a first Jacobi sweep from zero)
template <class T>
__global__ void k_mg_presmooth(MgGrid g, MgOp op, const T* __restrict__ b, T* __restrict__ x, T omega,
                               const CgState* st) {
    if (st && st->done) return;
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < g.n3; X += gridDim.x * blockDim.x)
        x[X] = omega * mg_inv_diag<T>(g, op, X) * b[X];
}

// bc[I] = sum over the 8 children of (b - A x) (residual restricted to the next level)
template <class T>
__global__ void k_mg_restrict(MgGrid g, MgGrid cg, MgOp op, const T* __restrict__ b, const T* __restrict__ x,
                              T* __restrict__ bc, const CgState* st) {
    if (st && st->done) return;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < cg.n3; I += gridDim.x * blockDim.x) {
        const int ci = I % cg.n, cj = (I / cg.n) % cg.n, ck = I / cg.n2;
        T acc = T(0);
        for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
                for (int a = 0; a < 2; ++a) {
                    const int i = 2 * ci + a, j = 2 * cj + bb, k = 2 * ck + c;
                    T inv;
                    const T ax = mg_apply<T>(g, op, x, i, j, k, &inv);
                    acc += b[mg_idx(g, i, j, k)] - ax;
                }
        bc[I] = acc;
    }
}

// y = x' + omega D^-1 (b - A x') with x' = x + scale * P xc (the coarse
// correction added on the fly at the node and its neighbours).  With part !=
// nullptr the block also writes its partial of (b, y) into part[slot][lb].
template <class T>
__global__ void k_mg_postsmooth(MgGrid g, MgOp op, const T* __restrict__ b, const T* __restrict__ x,
                                const T* __restrict__ xc, int cn, T scale, T omega, T* __restrict__ y, double* part,
                                int slot, const CgState* st) {
    if (st && st->done) return;
    double acc[1] = {0.0};
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < g.n3; X += gridDim.x * blockDim.x) {
        const int i = X % g.n, j = (X / g.n) % g.n, k = X / g.n2;
        // corrected iterate at the seven points
        auto corr = [=](int ii, int jj, int kk) -> T {
            const int f = mg_idx(g, ii, jj, kk);
            const int fi = wrapc(ii, g.n), fj = wrapc(jj, g.n), fk = wrapc(kk, g.n);
            const int C = (fi >> 1) + cn * ((fj >> 1) + cn * (fk >> 1));
            return x[f] + scale * xc[C];
        };
        const T xX = corr(i, j, k);
        const T xxm = corr(i - 1, j, k), xxp = corr(i + 1, j, k);
        const T xym = corr(i, j - 1, k), xyp = corr(i, j + 1, k);
        const T xzm = corr(i, j, k - 1), xzp = corr(i, j, k + 1);
        T ax, inv;
        if (op.code) {
            const int cX = op.code[X];
            const int xp = mg_idx(g, i + 1, j, k), yp = mg_idx(g, i, j + 1, k), zp = mg_idx(g, i, j, k + 1);
            const T wxl = inv_diag_A_t<T>(sx_of(cX)), wyl = inv_diag_A_t<T>(sy_of(cX)),
                    wzl = inv_diag_A_t<T>(sz_of(cX));
            const T wxh = inv_diag_A_t<T>(sx_of(op.code[xp])), wyh = inv_diag_A_t<T>(sy_of(op.code[yp])),
                    wzh = inv_diag_A_t<T>(sz_of(op.code[zp]));
            inv = ((const T*)op.invd)[X];
            ax = ((wxl * (xX - xxm) + wxh * (xX - xxp)) + (wyl * (xX - xym) + wyh * (xX - xyp))) +
                 (wzl * (xX - xzm) + wzh * (xX - xzp));
        } else {
            const T* D = (const T*)op.D;
            const T* Wx = (const T*)op.Wx;
            const T* Wy = (const T*)op.Wy;
            const T* Wz = (const T*)op.Wz;
            const T d = D[X];
            inv = d > T(0) ? T(1) / d : T(0);
            ax = d * xX - (((Wx[X] * xxm + Wx[mg_idx(g, i + 1, j, k)] * xxp) +
                            (Wy[X] * xym + Wy[mg_idx(g, i, j + 1, k)] * xyp)) +
                           (Wz[X] * xzm + Wz[mg_idx(g, i, j, k + 1)] * xzp));
        }
        // a coarse correction also reaches solid voxels that share an aggregate
        // with fluid; nodes that are not unknowns (1/D = 0) are held at 0
        const T yv = inv > T(0) ? xX + omega * inv * (b[X] - ax) : T(0);
        y[X] = yv;
        acc[0] += (double)b[X] * (double)yv;
    }
    // the grid then has exactly as many blocks as the CG sweeps, whose next
    // kernel re-adds these partials
    if (part) write_partials<1>(acc, part, slot, blockIdx.x);
}

// Coarsest level: `sweeps` damped-Jacobi sweeps from zero inside one workgroup
// (x in LDS, double-buffered).  n3 <= kMgCoarsestMax.
constexpr int kMgCoarsestMax = 2048;

template <class T>
__global__ void k_mg_coarsest(MgGrid g, MgOp op, const T* __restrict__ b, T* __restrict__ xout, T omega, int sweeps,
                              const CgState* st) {
    if (st && st->done) return;
    __shared__ T xs[2][kMgCoarsestMax];
    for (int X = threadIdx.x; X < g.n3; X += blockDim.x) xs[0][X] = omega * mg_inv_diag<T>(g, op, X) * b[X];
    __syncthreads();
    int cur = 0;
    for (int it = 1; it < sweeps; ++it) {
        for (int X = threadIdx.x; X < g.n3; X += blockDim.x) {
            const int i = X % g.n, j = (X / g.n) % g.n, k = X / g.n2;
            T inv;
            const T ax = mg_apply<T>(g, op, xs[cur], i, j, k, &inv);
            xs[cur ^ 1][X] = xs[cur][X] + omega * inv * (b[X] - ax);
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int X = threadIdx.x; X < g.n3; X += blockDim.x) xout[X] = xs[cur][X];
}

// out = (float) in, flat
__global__ void k_narrow_flat(int n, const double* __restrict__ in, float* __restrict__ out) {
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < n; X += gridDim.x * blockDim.x) out[X] = (float)in[X];
}

}  // namespace stokes
