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
// damped-Jacobi sweep from zero, residual restricted to the next level,
// coarse correction prolonged and scaled, one damped-Jacobi sweep; the
// coarsest level runs a fixed number of Jacobi sweeps inside one workgroup.
// Nodes that are not unknowns (diagonal 0) are held at 0.
#pragma once

#include "kernels.h"

namespace stokes {

// Level geometry: nb planes of n^3 nodes; node I = p * n3 + (i + n (j + n k)).
struct MgGrid {
    int n, n2, n3, nb;
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
    const void* D;      // levels >= 1
    const void* Wx;
    const void* Wy;
    const void* Wz;
};

// Seven values of a plane's vector around node (i, j, k).
template <class T>
struct Seven {
    T c, xm, xp, ym, yp, zm, zp;
};

template <class T>
__device__ __forceinline__ Seven<T> mg_load7(const MgGrid& g, const T* __restrict__ x, int p, int i, int j, int k) {
    const T* xpl = x + (size_t)p * g.n3;
    return {xpl[mg_idx(g, i, j, k)],     xpl[mg_idx(g, i - 1, j, k)], xpl[mg_idx(g, i + 1, j, k)],
            xpl[mg_idx(g, i, j - 1, k)], xpl[mg_idx(g, i, j + 1, k)], xpl[mg_idx(g, i, j, k - 1)],
            xpl[mg_idx(g, i, j, k + 1)]};
}

// (A v)_node and 1/D at node (p; i, j, k), given the seven values v.
template <class T>
__device__ __forceinline__ T mg_apply7(const MgGrid& g, const MgOp& op, const Seven<T>& v, int p, int i, int j, int k,
                                       T* inv_diag) {
    const int X = mg_idx(g, i, j, k);
    if (op.code) {
        const int cX = op.code[X];
        if (op.kind == kMgFineShat) {
            const T wxl = inv_diag_A_t<T>(sx_of(cX)), wyl = inv_diag_A_t<T>(sy_of(cX)),
                    wzl = inv_diag_A_t<T>(sz_of(cX));
            const T wxh = inv_diag_A_t<T>(sx_of(op.code[mg_idx(g, i + 1, j, k)])),
                    wyh = inv_diag_A_t<T>(sy_of(op.code[mg_idx(g, i, j + 1, k)])),
                    wzh = inv_diag_A_t<T>(sz_of(op.code[mg_idx(g, i, j, k + 1)]));
            *inv_diag = ((const T*)op.invd)[X];
            return ((wxl * (v.c - v.xm) + wxh * (v.c - v.xp)) + (wyl * (v.c - v.ym) + wyh * (v.c - v.yp))) +
                   (wzl * (v.c - v.zm) + wzh * (v.c - v.zp));
        }
        const int s = s_plane(cX, p);
        *inv_diag = inv_diag_A_t<T>(s);
        const T nb = ((v.xm + v.xp) + (v.ym + v.yp)) + (v.zm + v.zp);
        return s ? (T)(5 + s) * v.c - nb : T(0);
    }
    const size_t o = (size_t)p * g.n3;
    const T* D = (const T*)op.D + o;
    const T* Wx = (const T*)op.Wx + o;
    const T* Wy = (const T*)op.Wy + o;
    const T* Wz = (const T*)op.Wz + o;
    const T d = D[X];
    *inv_diag = d > T(0) ? T(1) / d : T(0);
    return d * v.c - (((Wx[X] * v.xm + Wx[mg_idx(g, i + 1, j, k)] * v.xp) +
                       (Wy[X] * v.ym + Wy[mg_idx(g, i, j + 1, k)] * v.yp)) +
                      (Wz[X] * v.zm + Wz[mg_idx(g, i, j, k + 1)] * v.zp));
}

template <class T>
__device__ __forceinline__ T mg_inv_diag(const MgGrid& g, const MgOp& op, int p, int X) {
    if (op.code) {
        if (op.kind == kMgFineShat) return ((const T*)op.invd)[X];
        return inv_diag_A_t<T>(s_plane(op.code[X], p));
    }
    const T d = ((const T*)op.D)[(size_t)p * g.n3 + X];
    return d > T(0) ? T(1) / d : T(0);
}

// x = omega D^-1 b (a first Jacobi sweep from zero)
template <class T>
__global__ void k_mg_presmooth(MgGrid g, MgOp op, const T* __restrict__ b, T* __restrict__ x, T omega,
                               const CgState* st) {
    if (st && st->done) return;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < g.nb * g.n3; I += gridDim.x * blockDim.x) {
        const int p = I / g.n3;
        x[I] = omega * mg_inv_diag<T>(g, op, p, I - p * g.n3) * b[I];
    }
}

// bc[I] = sum over the 8 children of (b - A x) (residual restricted to the next level)
template <class T>
__global__ void k_mg_restrict(MgGrid g, MgGrid cg, MgOp op, const T* __restrict__ b, const T* __restrict__ x,
                              T* __restrict__ bc, const CgState* st) {
    if (st && st->done) return;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < cg.nb * cg.n3; I += gridDim.x * blockDim.x) {
        const int p = I / cg.n3, L = I - p * cg.n3;
        const int ci = L % cg.n, cj = (L / cg.n) % cg.n, ck = L / cg.n2;
        T acc = T(0);
        for (int c = 0; c < 2; ++c)
            for (int bb = 0; bb < 2; ++bb)
                for (int a = 0; a < 2; ++a) {
                    const int i = 2 * ci + a, j = 2 * cj + bb, k = 2 * ck + c;
                    T inv;
                    const Seven<T> v = mg_load7<T>(g, x, p, i, j, k);
                    const T ax = mg_apply7<T>(g, op, v, p, i, j, k, &inv);
                    acc += b[(size_t)p * g.n3 + mg_idx(g, i, j, k)] - ax;
                }
        bc[I] = acc;
    }
}

// y = x' + omega D^-1 (b - A x') with x' = x + scale * P xc (the coarse
// correction added on the fly at the node and its neighbours).  With part !=
// nullptr the block writes its partial of (b, y) into part[slot][blockIdx.x];
// the grid then has exactly as many blocks as the CG sweeps, whose next kernel
// re-adds these partials.
template <class T>
__global__ void k_mg_postsmooth(MgGrid g, MgOp op, const T* __restrict__ b, const T* __restrict__ x,
                                const T* __restrict__ xc, int cn, T scale, T omega, T* __restrict__ y, double* part,
                                int slot, const CgState* st) {
    if (st && st->done) return;
    double acc[1] = {0.0};
    const int cn3 = cn * cn * cn;
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < g.nb * g.n3; I += gridDim.x * blockDim.x) {
        const int p = I / g.n3, X = I - p * g.n3;
        const int i = X % g.n, j = (X / g.n) % g.n, k = X / g.n2;
        const T* xpl = x + (size_t)p * g.n3;
        const T* cpl = xc + (size_t)p * cn3;
        // corrected iterate at the seven points
        auto corr = [=](int ii, int jj, int kk) -> T {
            const int fi = wrapc(ii, g.n), fj = wrapc(jj, g.n), fk = wrapc(kk, g.n);
            return xpl[fi + g.n * (fj + g.n * fk)] + scale * cpl[(fi >> 1) + cn * ((fj >> 1) + cn * (fk >> 1))];
        };
        const Seven<T> v = {corr(i, j, k),     corr(i - 1, j, k), corr(i + 1, j, k), corr(i, j - 1, k),
                            corr(i, j + 1, k), corr(i, j, k - 1), corr(i, j, k + 1)};
        T inv;
        const T ax = mg_apply7<T>(g, op, v, p, i, j, k, &inv);
        // a coarse correction also reaches nodes that share an aggregate with
        // unknowns; nodes that are not unknowns (1/D = 0) are held at 0
        const T yv = inv > T(0) ? v.c + omega * inv * (b[I] - ax) : T(0);
        y[I] = yv;
        acc[0] += (double)b[I] * (double)yv;
    }
    if (part) write_partials<1>(acc, part, slot, blockIdx.x);
}

// Coarsest level: `sweeps` damped-Jacobi sweeps from zero inside one workgroup
// (x in LDS, double-buffered).  nb * n3 <= kMgCoarsestMax.
constexpr int kMgCoarsestMax = 2048;

template <class T>
__global__ void k_mg_coarsest(MgGrid g, MgOp op, const T* __restrict__ b, T* __restrict__ xout, T omega, int sweeps,
                              const CgState* st) {
    if (st && st->done) return;
    __shared__ T xs[2][kMgCoarsestMax];
    const int n = g.nb * g.n3;
    for (int I = threadIdx.x; I < n; I += blockDim.x) {
        const int p = I / g.n3;
        xs[0][I] = omega * mg_inv_diag<T>(g, op, p, I - p * g.n3) * b[I];
    }
    __syncthreads();
    int cur = 0;
    for (int it = 1; it < sweeps; ++it) {
        for (int I = threadIdx.x; I < n; I += blockDim.x) {
            const int p = I / g.n3, X = I - p * g.n3;
            const int i = X % g.n, j = (X / g.n) % g.n, k = X / g.n2;
            const Seven<T> v = mg_load7<T>(g, xs[cur], p, i, j, k);
            T inv;
            const T ax = mg_apply7<T>(g, op, v, p, i, j, k, &inv);
            xs[cur ^ 1][I] = v.c + omega * inv * (b[I] - ax);
        }
        __syncthreads();
        cur ^= 1;
    }
    for (int I = threadIdx.x; I < n; I += blockDim.x) xout[I] = xs[cur][I];
}

// out = (float) in, flat
__global__ void k_narrow_flat(int n, const double* __restrict__ in, float* __restrict__ out) {
    for (int X = blockIdx.x * blockDim.x + threadIdx.x; X < n; X += gridDim.x * blockDim.x) out[X] = (float)in[X];
}

}  // namespace stokes
