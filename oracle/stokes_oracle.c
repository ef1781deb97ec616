/*
 * stokes_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU reference, in FP64, for the pressure Schur-complement
 * method of Pimanov, Iliev, Oseledets, Muravleva, "On the efficient
 * preconditioning of the Stokes equations in tight geometries"
 * (arXiv 2307.05266).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * does, and this file shares no code with it.
 *
 * What it computes:
 *  - the voxel geometry and its periodic fluid components (Sec. 2.1, 2.2);
 *  - the staggered (MAC) operators as explicit sparse matrices over the
 *    active unknowns only: the negative velocity Laplacian A with no-slip
 *    walls, the negative divergence B and the gradient B^T, each assembled
 *    from its own rule (Sec. 1, eq. coupled_matrix; Sec. 2.1);
 *  - S = B A^{-1} B^T and g = B A^{-1} f applied through inner solves
 *    (eqs. schur_system, schur_rhs);
 *  - the outer preconditioned CG of Algorithm 1 with the Uzawa (identity)
 *    or SIMPLE (B diag(A)^{-1} B^T) preconditioner (eq. schur_uzawa_prec),
 *    with the sign convention of standard PCG (r = g - S p);
 *  - inner Jacobi-preconditioned CG solves with A and with the SIMPLE
 *    matrix, stopped on the relative preconditioned residual (Sec. 3.2);
 *  - the permeability as the mean velocity along the force (Sec. 2.3).
 *
 * Conventions (voxel units, h = 1):
 *   cell X = (i,j,k), flat index i + N*(j + N*k), periodic.
 *   face (c,X) = lower face of X in direction c, between X - e_c and X.
 *   A face is an unknown ("active") when both of its cells are fluid.
 *   Dense face arrays hold component c at offset c*N^3; inactive entries 0.
 *   Wall convention for A: the row of an active face F=(c,X) has
 *     diagonal 6 + t(F) and -1 for every active neighbour face (c, X +- e_d),
 *   where t(F) counts the tangential neighbour faces (d != c) whose two
 *   cells are both solid (a wall half a voxel away, mirrored ghost value);
 *   inactive neighbours with a fluid cell lie on the wall and contribute 0.
 *   Parity unpinned: nothing here is compared with the paper's own numbers,
 *   whose inputs (CT images, 2D seeds) are not available.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    long n;         /* rows */
    long *ptr;      /* n+1 */
    long *col;
    double *val;
} csr_t;

typedef struct {
    int N;
    long n3;
    double force[3];
    uint8_t *fluid_in;     /* mask as given */
    uint8_t *fluid;        /* after removing non-conducting components */
    int32_t *comp;         /* kept-component id per cell, -1 elsewhere */
    int ncomp_all, ncomp_kept;
    long nfluid_in, nfluid, nsurf;
    long *comp_size;       /* [ncomp_kept] */
    long nf;               /* active faces */
    long *face_id;         /* [3*n3] -> unknown or -1 */
    long *face_pos;        /* [nf] -> c*n3 + X */
    long nc;               /* fluid cells */
    long *cell_id;         /* [n3] */
    long *cell_pos;        /* [nc] */
    csr_t A, B, BT;
    double *diagA;         /* [nf] */
    double *diagS;         /* [nc] */
} osys_t;

static inline long cidx(int N, int i, int j, int k)
{
    i %= N; if (i < 0) i += N;
    j %= N; if (j < 0) j += N;
    k %= N; if (k < 0) k += N;
    return (long)i + (long)N * ((long)j + (long)N * (long)k);
}

static inline void coords(int N, long X, int *i, int *j, int *k)
{
    *i = (int)(X % N);
    *j = (int)((X / N) % N);
    *k = (int)(X / ((long)N * N));
}

/* neighbour of X shifted by s (+1/-1) along axis d */
static inline long shift(int N, long X, int d, int s)
{
    int c[3];
    coords(N, X, &c[0], &c[1], &c[2]);
    c[d] += s;
    return cidx(N, c[0], c[1], c[2]);
}

/* ---------------------------------------------------------------------- */
/* Components and their windings (Sec. 2.2: connected flow domain; the    */
/* pressure is fixed up to one constant per component).                   */
/*                                                                        */
/* Breadth-first search from each unlabelled fluid cell, carrying an      */
/* unwrapped position for every reached cell.  An edge that closes a      */
/* cycle returns to an already placed cell; the difference of positions,  */
/* divided by N, is that cycle's winding vector w.  A component conducts  */
/* flow under the force f when some winding has f.w != 0; otherwise the   */
/* pressure p = f . (unwrapped position) balances the force exactly and   */
/* the velocity is identically zero there, so such components are turned  */
/* into solid without changing the solution anywhere.                     */
/* ---------------------------------------------------------------------- */
static void label_components(osys_t *s)
{
    const int N = s->N;
    const long n3 = s->n3;
    int32_t *lab = (int32_t *)malloc(n3 * sizeof(int32_t));
    int32_t *pos = (int32_t *)malloc(3 * n3 * sizeof(int32_t));
    long *queue = (long *)malloc(n3 * sizeof(long));
    uint8_t *conducts = NULL;
    int ncomp = 0, cap = 0;
    for (long X = 0; X < n3; ++X) lab[X] = -1;

    for (long seed = 0; seed < n3; ++seed) {
        if (!s->fluid_in[seed] || lab[seed] >= 0) continue;
        if (ncomp == cap) {
            cap = cap ? 2 * cap : 64;
            conducts = (uint8_t *)realloc(conducts, cap);
        }
        int id = ncomp++;
        conducts[id] = 0;
        long head = 0, tail = 0;
        queue[tail++] = seed;
        lab[seed] = id;
        coords(N, seed, &pos[3 * seed], &pos[3 * seed + 1], &pos[3 * seed + 2]);
        while (head < tail) {
            long a = queue[head++];
            for (int d = 0; d < 3; ++d) {
                for (int sg = -1; sg <= 1; sg += 2) {
                    long b = shift(N, a, d, sg);
                    if (!s->fluid_in[b]) continue;
                    int want[3] = {pos[3 * a], pos[3 * a + 1], pos[3 * a + 2]};
                    want[d] += sg;
                    if (lab[b] < 0) {
                        lab[b] = id;
                        pos[3 * b] = want[0];
                        pos[3 * b + 1] = want[1];
                        pos[3 * b + 2] = want[2];
                        queue[tail++] = b;
                    } else {
                        double fw = 0.0;
                        for (int e = 0; e < 3; ++e) {
                            int w = (want[e] - pos[3 * b + e]) / N;   /* exact multiple of N */
                            fw += s->force[e] * (double)w;
                        }
                        if (fw != 0.0) conducts[id] = 1;
                    }
                }
            }
        }
    }

    /* renumber the conducting components 0..ncomp_kept-1 */
    int32_t *newid = (int32_t *)malloc((ncomp > 0 ? ncomp : 1) * sizeof(int32_t));
    int kept = 0;
    for (int c = 0; c < ncomp; ++c) newid[c] = conducts[c] ? kept++ : -1;
    s->ncomp_all = ncomp;
    s->ncomp_kept = kept;
    s->comp_size = (long *)calloc(kept > 0 ? kept : 1, sizeof(long));
    s->nfluid = 0;
    for (long X = 0; X < n3; ++X) {
        int c = lab[X] >= 0 ? newid[lab[X]] : -1;
        s->comp[X] = c;
        s->fluid[X] = (uint8_t)(c >= 0);
        if (c >= 0) { s->comp_size[c]++; s->nfluid++; }
    }
    free(newid);
    free(conducts);
    free(queue);
    free(pos);
    free(lab);
}

/* Label every fluid component, conducting or not (used when nothing is
 * removed: then each component keeps its own pressure constant). */
static void keep_all_components(osys_t *s)
{
    const int N = s->N;
    const long n3 = s->n3;
    long *queue = (long *)malloc(n3 * sizeof(long));
    long *sizes = NULL;
    int id = 0;
    for (long X = 0; X < n3; ++X) s->comp[X] = -1;
    for (long seed = 0; seed < n3; ++seed) {
        if (!s->fluid_in[seed] || s->comp[seed] >= 0) continue;
        sizes = (long *)realloc(sizes, (id + 1) * sizeof(long));
        sizes[id] = 0;
        long head = 0, tail = 0;
        queue[tail++] = seed;
        s->comp[seed] = id;
        while (head < tail) {
            long a = queue[head++];
            sizes[id]++;
            for (int d = 0; d < 3; ++d)
                for (int sg = -1; sg <= 1; sg += 2) {
                    long b = shift(N, a, d, sg);
                    if (s->fluid_in[b] && s->comp[b] < 0) { s->comp[b] = id; queue[tail++] = b; }
                }
        }
        ++id;
    }
    free(queue);
    free(s->comp_size);
    s->comp_size = sizes ? sizes : (long *)calloc(1, sizeof(long));
    s->ncomp_kept = id;
    s->nfluid = s->nfluid_in;
    memcpy(s->fluid, s->fluid_in, n3);
}

/* solid voxels sharing a face with a fluid voxel (eq. surface_area) */
static void count_surface(osys_t *s)
{
    long ns = 0, nfl = 0;
    for (long X = 0; X < s->n3; ++X) {
        if (s->fluid_in[X]) { nfl++; continue; }
        int touch = 0;
        for (int d = 0; d < 3 && !touch; ++d)
            for (int sg = -1; sg <= 1; sg += 2)
                if (s->fluid_in[shift(s->N, X, d, sg)]) touch = 1;
        ns += touch;
    }
    s->nsurf = ns;
    s->nfluid_in = nfl;
}

/* ---------------------------------------------------------------------- */
/* Sparse assembly.  Rows are built one at a time from a short list of    */
/* (column, value) pairs; repeated columns (possible when N = 2 and the   */
/* +e_d and -e_d neighbours coincide) are summed.                         */
/* ---------------------------------------------------------------------- */
typedef struct { long col[16]; double val[16]; int n; } rowbuf_t;

static void row_add(rowbuf_t *r, long col, double v)
{
    for (int q = 0; q < r->n; ++q)
        if (r->col[q] == col) { r->val[q] += v; return; }
    r->col[r->n] = col;
    r->val[r->n] = v;
    r->n++;
}

static void csr_alloc(csr_t *m, long n, long nnz_max)
{
    m->n = n;
    m->ptr = (long *)calloc(n + 1, sizeof(long));
    m->col = (long *)malloc((nnz_max > 0 ? nnz_max : 1) * sizeof(long));
    m->val = (double *)malloc((nnz_max > 0 ? nnz_max : 1) * sizeof(double));
}

static void csr_free(csr_t *m)
{
    free(m->ptr); free(m->col); free(m->val);
    memset(m, 0, sizeof(*m));
}

static void csr_push_row(csr_t *m, long row, const rowbuf_t *r)
{
    long at = m->ptr[row];
    for (int q = 0; q < r->n; ++q) {
        m->col[at + q] = r->col[q];
        m->val[at + q] = r->val[q];
    }
    m->ptr[row + 1] = at + r->n;
}

static inline int is_fluid(const osys_t *s, long X) { return s->fluid[X] != 0; }

/* face (c, X) is an unknown when both of its cells are fluid */
static inline int is_active(const osys_t *s, int c, long X)
{
    return is_fluid(s, X) && is_fluid(s, shift(s->N, X, c, -1));
}

/* Row of A at the active face F = c*n3 + X as (dense face position, value)
 * pairs, the diagonal first: diagonal 6 + t, -1 for each active neighbour
 * face (c, X +- e_d); a tangential neighbour with both cells solid is a wall
 * half a voxel away (mirrored ghost value, +1 on the diagonal); an inactive
 * neighbour touching fluid lies on the wall, where u = 0.  Returns the count. */
static int a_row(const osys_t *s, long F, long *pos, double *val)
{
    const int N = s->N;
    const long n3 = s->n3;
    const int c = (int)(F / n3);
    const long X = F % n3;
    const long Xm = shift(N, X, c, -1);        /* the other cell of this face */
    int n = 1;
    double diag = 6.0;
    for (int d = 0; d < 3; ++d) {
        for (int sg = -1; sg <= 1; sg += 2) {
            long Y = shift(N, X, d, sg);         /* neighbour face (c, Y) */
            if (is_active(s, c, Y)) {
                pos[n] = c * n3 + Y;
                val[n++] = -1.0;
            } else if (d != c) {
                long Ym = shift(N, Xm, d, sg);   /* its other cell */
                if (!is_fluid(s, Y) && !is_fluid(s, Ym)) diag += 1.0;
            }
        }
    }
    pos[0] = F;
    val[0] = diag;
    return n;
}

static void assemble(osys_t *s)
{
    const int N = s->N;
    const long n3 = s->n3;

    /* unknowns: active faces (both cells fluid) and fluid cells */
    s->nf = 0;
    for (int c = 0; c < 3; ++c)
        for (long X = 0; X < n3; ++X) {
            long F = c * n3 + X;
            if (is_fluid(s, X) && is_fluid(s, shift(N, X, c, -1))) s->face_id[F] = s->nf++;
            else s->face_id[F] = -1;
        }
    s->face_pos = (long *)malloc((s->nf > 0 ? s->nf : 1) * sizeof(long));
    for (long F = 0; F < 3 * n3; ++F)
        if (s->face_id[F] >= 0) s->face_pos[s->face_id[F]] = F;
    s->nc = 0;
    for (long X = 0; X < n3; ++X) s->cell_id[X] = is_fluid(s, X) ? s->nc++ : -1;
    s->cell_pos = (long *)malloc((s->nc > 0 ? s->nc : 1) * sizeof(long));
    for (long X = 0; X < n3; ++X)
        if (s->cell_id[X] >= 0) s->cell_pos[s->cell_id[X]] = X;

    /* A: negative vector Laplacian with no-slip on the voxel walls */
    csr_alloc(&s->A, s->nf, 7 * s->nf);
    s->diagA = (double *)malloc((s->nf > 0 ? s->nf : 1) * sizeof(double));
    for (long r = 0; r < s->nf; ++r) {
        long pos[7];
        double val[7];
        const int n = a_row(s, s->face_pos[r], pos, val);
        rowbuf_t row;
        row.n = 0;
        for (int q = 1; q < n; ++q) row_add(&row, s->face_id[pos[q]], val[q]);
        row_add(&row, r, val[0]);
        s->diagA[r] = val[0];
        csr_push_row(&s->A, r, &row);
    }

    /* B: negative divergence, (B u)_X = -sum_c [u(c, X + e_c) - u(c, X)] */
    csr_alloc(&s->B, s->nc, 6 * s->nc);
    for (long r = 0; r < s->nc; ++r) {
        long X = s->cell_pos[r];
        rowbuf_t row;
        row.n = 0;
        for (int c = 0; c < 3; ++c) {
            long lo = c * n3 + X;
            long hi = c * n3 + shift(N, X, c, +1);
            if (s->face_id[lo] >= 0) row_add(&row, s->face_id[lo], +1.0);
            if (s->face_id[hi] >= 0) row_add(&row, s->face_id[hi], -1.0);
        }
        csr_push_row(&s->B, r, &row);
    }

    /* B^T: the gradient, (B^T p)(c, X) = p_X - p_{X - e_c}, built from its own rule */
    csr_alloc(&s->BT, s->nf, 2 * s->nf);
    for (long r = 0; r < s->nf; ++r) {
        long F = s->face_pos[r];
        int c = (int)(F / n3);
        long X = F % n3;
        rowbuf_t row;
        row.n = 0;
        row_add(&row, s->cell_id[X], +1.0);
        row_add(&row, s->cell_id[shift(N, X, c, -1)], -1.0);
        csr_push_row(&s->BT, r, &row);
    }

    /* diagonal of the SIMPLE matrix B diag(A)^{-1} B^T */
    s->diagS = (double *)malloc((s->nc > 0 ? s->nc : 1) * sizeof(double));
    for (long r = 0; r < s->nc; ++r) {
        double acc = 0.0;
        for (long q = s->B.ptr[r]; q < s->B.ptr[r + 1]; ++q)
            acc += s->B.val[q] * s->B.val[q] / s->diagA[s->B.col[q]];
        s->diagS[r] = acc;
    }
}

/* ---------------------------------------------------------------------- */
/* Plain vector kernels                                                   */
/* ---------------------------------------------------------------------- */
static void spmv(const csr_t *m, const double *x, double *y)
{
    long r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < m->n; ++r) {
        double acc = 0.0;
        for (long q = m->ptr[r]; q < m->ptr[r + 1]; ++q) acc += m->val[q] * x[m->col[q]];
        y[r] = acc;
    }
}

static double dot(long n, const double *a, const double *b)
{
    double acc = 0.0;
    long q;
#pragma omp parallel for schedule(static) reduction(+ : acc)
    for (q = 0; q < n; ++q) acc += a[q] * b[q];
    return acc;
}

static double nrm2(long n, const double *a) { return sqrt(dot(n, a, a)); }

/* subtract each kept component's mean (the constant pressure nullspace) */
static void project(const osys_t *s, double *x)
{
    int K = s->ncomp_kept;
    double *sum = (double *)calloc(K > 0 ? K : 1, sizeof(double));
    for (long r = 0; r < s->nc; ++r) sum[s->comp[s->cell_pos[r]]] += x[r];
    for (int c = 0; c < K; ++c) sum[c] /= (double)s->comp_size[c];
    for (long r = 0; r < s->nc; ++r) x[r] -= sum[s->comp[s->cell_pos[r]]];
    free(sum);
}

/* S-hat = B diag(A)^{-1} B^T applied as three steps */
static void apply_shat(const osys_t *s, const double *p, double *out, double *face_tmp)
{
    spmv(&s->BT, p, face_tmp);
    for (long r = 0; r < s->nf; ++r) face_tmp[r] /= s->diagA[r];
    spmv(&s->B, face_tmp, out);
}

/* ---------------------------------------------------------------------- */
/* Inner Jacobi-preconditioned CG (Saad, Alg. 9.1), x0 = 0, stopped when  */
/* ||D^{-1} r_j|| / ||D^{-1} r_0|| < eps (Sec. 3.2).  Returns the number  */
/* of operator applications, or -1 on breakdown.                          */
/* ---------------------------------------------------------------------- */
typedef struct { const osys_t *s; int which; double *tmp; } opctx_t;

static void opctx_apply(const opctx_t *o, const double *in, double *out)
{
    if (o->which == 0) spmv(&o->s->A, in, out);
    else apply_shat(o->s, in, out, o->tmp);
}

static int pcg(const opctx_t *o, long n, const double *diag,
               const double *b, double *x, double eps, int maxit, int *status)
{
    double *r = (double *)malloc((n > 0 ? n : 1) * sizeof(double));
    double *z = (double *)malloc((n > 0 ? n : 1) * sizeof(double));
    double *d = (double *)malloc((n > 0 ? n : 1) * sizeof(double));
    double *q = (double *)malloc((n > 0 ? n : 1) * sizeof(double));
    int it = 0;
    for (long i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        z[i] = r[i] / diag[i];
        d[i] = z[i];
    }
    double rho = dot(n, r, z);
    double z0 = nrm2(n, z);
    if (z0 == 0.0) goto done;
    for (;;) {
        if (it >= maxit) { *status = 1; break; }
        opctx_apply(o, d, q);
        ++it;
        double dq = dot(n, d, q);
        if (!(dq > 0.0)) { *status = -4; break; }
        double alpha = rho / dq;
        for (long i = 0; i < n; ++i) {
            x[i] += alpha * d[i];
            r[i] -= alpha * q[i];
            z[i] = r[i] / diag[i];
        }
        if (nrm2(n, z) / z0 < eps) break;
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (long i = 0; i < n; ++i) d[i] = z[i] + beta * d[i];
    }
done:
    free(r); free(z); free(d); free(q);
    return it;
}

/* ---------------------------------------------------------------------- */
/* Public entry points (ctypes)                                           */
/* ---------------------------------------------------------------------- */
void oracle_destroy(osys_t *s)
{
    if (!s) return;
    free(s->fluid_in); free(s->fluid); free(s->comp); free(s->comp_size);
    free(s->face_id); free(s->face_pos); free(s->cell_id); free(s->cell_pos);
    csr_free(&s->A); csr_free(&s->B); csr_free(&s->BT);
    free(s->diagA); free(s->diagS);
    free(s);
}

/* strip = 0 keeps every fluid component (each one then carries its own
 * pressure constant); strip = 1 removes the ones that cannot conduct.
 * assemble = 0 stops after the components (for oracle_sample_residuals on
 * boxes too large to assemble); every other entry point needs assemble = 1. */
osys_t *oracle_create_ex(int N, const uint8_t *mask, const double *force, int strip, int assemble_it)
{
    if (N < 2) return NULL;
    osys_t *s = (osys_t *)calloc(1, sizeof(osys_t));
    s->N = N;
    s->n3 = (long)N * N * N;
    for (int c = 0; c < 3; ++c) s->force[c] = force[c];
    s->fluid_in = (uint8_t *)malloc(s->n3);
    s->fluid = (uint8_t *)malloc(s->n3);
    s->comp = (int32_t *)malloc(s->n3 * sizeof(int32_t));
    if (assemble_it) {
        s->face_id = (long *)malloc(3 * s->n3 * sizeof(long));
        s->cell_id = (long *)malloc(s->n3 * sizeof(long));
    }
    for (long X = 0; X < s->n3; ++X) s->fluid_in[X] = mask[X] ? 1 : 0;
    count_surface(s);
    label_components(s);
    if (!strip) keep_all_components(s);
    if (assemble_it) assemble(s);
    return s;
}

osys_t *oracle_create(int N, const uint8_t *mask, const double *force, int strip)
{
    return oracle_create_ex(N, mask, force, strip, 1);
}

/* Residuals of the discrete Stokes system (Sec. 2.2) at sampled unknowns,
 * row by row, without assembling: for the face position F = c*n3 + X,
 *   rf = (A u)_F + p_X - p_{X-e_c} - f_c        (momentum, eq. for u)
 * and for the cell X,
 *   rc = -sum_c [u(c, X+e_c) - u(c, X)] over active faces   (B u, continuity).
 * u: dense faces (3 n3), p: dense cells.  Positions that are not unknowns get
 * NAN.  Works on a context created with or without assembly. */
void oracle_sample_residuals(const osys_t *s, const double *u, const double *p, long nfs, const long *fpos,
                             double *rf, long ncs, const long *cpos, double *rc)
{
    const int N = s->N;
    const long n3 = s->n3;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < nfs; ++q) {
        const long F = fpos[q];
        const int c = (int)(F / n3);
        const long X = F % n3;
        if (F < 0 || F >= 3 * n3 || !is_active(s, c, X)) { rf[q] = NAN; continue; }
        long pos[7];
        double val[7];
        const int n = a_row(s, F, pos, val);
        double acc = 0.0;
        for (int t = 0; t < n; ++t) acc += val[t] * u[pos[t]];
        rf[q] = acc + (p[X] - p[shift(N, X, c, -1)]) - s->force[c];
    }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < ncs; ++q) {
        const long X = cpos[q];
        if (X < 0 || X >= n3 || !is_fluid(s, X)) { rc[q] = NAN; continue; }
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) {
            const long hi = shift(N, X, c, +1);
            if (is_active(s, c, X)) acc += u[c * n3 + X];
            if (is_active(s, c, hi)) acc -= u[c * n3 + hi];
        }
        rc[q] = acc;
    }
}

/* info[0..9] = N, nfluid_in, nfluid(kept), nsurf, ncomp_all, ncomp_kept,
 *              nf (active faces), nc (fluid cells), nnz(A), nnz(B) */
void oracle_info(const osys_t *s, long *info)
{
    info[0] = s->N;
    info[1] = s->nfluid_in;
    info[2] = s->nfluid;
    info[3] = s->nsurf;
    info[4] = s->ncomp_all;
    info[5] = s->ncomp_kept;
    info[6] = s->nf;
    info[7] = s->nc;
    info[8] = s->A.ptr ? s->A.ptr[s->A.n] : 0;
    info[9] = s->B.ptr ? s->B.ptr[s->B.n] : 0;
}

/* kept fluid mask (after stripping) and kept-component labels (-1 solid) */
void oracle_masks(const osys_t *s, uint8_t *fluid, int32_t *comp)
{
    if (fluid) memcpy(fluid, s->fluid, s->n3);
    if (comp) memcpy(comp, s->comp, s->n3 * sizeof(int32_t));
}

/* which: 0 = A, 1 = B, 2 = B^T.  Writes CSR arrays of the matrix over the
 * active unknowns and the unknown -> dense position maps. */
void oracle_csr(const osys_t *s, int which, long *ptr, long *col, double *val)
{
    const csr_t *m = which == 0 ? &s->A : which == 1 ? &s->B : &s->BT;
    long nnz = m->ptr[m->n];
    memcpy(ptr, m->ptr, (m->n + 1) * sizeof(long));
    memcpy(col, m->col, nnz * sizeof(long));
    memcpy(val, m->val, nnz * sizeof(double));
}

void oracle_unknowns(const osys_t *s, long *face_pos, long *cell_pos)
{
    if (face_pos) memcpy(face_pos, s->face_pos, s->nf * sizeof(long));
    if (cell_pos) memcpy(cell_pos, s->cell_pos, s->nc * sizeof(long));
}

static void gather_faces(const osys_t *s, const double *dense, double *v)
{
    for (long r = 0; r < s->nf; ++r) v[r] = dense[s->face_pos[r]];
}
static void scatter_faces(const osys_t *s, const double *v, double *dense)
{
    memset(dense, 0, 3 * s->n3 * sizeof(double));
    for (long r = 0; r < s->nf; ++r) dense[s->face_pos[r]] = v[r];
}
static void gather_cells(const osys_t *s, const double *dense, double *v)
{
    for (long r = 0; r < s->nc; ++r) v[r] = dense[s->cell_pos[r]];
}
static void scatter_cells(const osys_t *s, const double *v, double *dense)
{
    memset(dense, 0, s->n3 * sizeof(double));
    for (long r = 0; r < s->nc; ++r) dense[s->cell_pos[r]] = v[r];
}

/* Apply one operator to a dense field.  op: 0 = A (faces->faces),
 * 1 = B (faces->cells), 2 = B^T (cells->faces), 3 = SIMPLE matrix
 * (cells->cells), 4 = diag(A) (faces), 5 = diag(SIMPLE) (cells),
 * 6 = per-component mean removal (cells->cells).
 * Entries of `in` at inactive positions are ignored. */
int oracle_apply(const osys_t *s, int op, const double *in, double *out)
{
    long nf = s->nf > 0 ? s->nf : 1, nc = s->nc > 0 ? s->nc : 1;
    double *fa = (double *)calloc(nf, sizeof(double));
    double *fb = (double *)calloc(nf, sizeof(double));
    double *ca = (double *)calloc(nc, sizeof(double));
    double *cb = (double *)calloc(nc, sizeof(double));
    int rc = 0;
    switch (op) {
    case 0: gather_faces(s, in, fa); spmv(&s->A, fa, fb); scatter_faces(s, fb, out); break;
    case 1: gather_faces(s, in, fa); spmv(&s->B, fa, ca); scatter_cells(s, ca, out); break;
    case 2: gather_cells(s, in, ca); spmv(&s->BT, ca, fa); scatter_faces(s, fa, out); break;
    case 3: gather_cells(s, in, ca); apply_shat(s, ca, cb, fa); scatter_cells(s, cb, out); break;
    case 4: scatter_faces(s, s->diagA, out); break;
    case 5: scatter_cells(s, s->diagS, out); break;
    case 6: gather_cells(s, in, ca); project(s, ca); scatter_cells(s, ca, out); break;
    default: rc = -1;
    }
    free(fa); free(fb); free(ca); free(cb);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* The outer solve (Algorithm 1 as standard PCG on S p = g).              */
/*                                                                        */
/* params[0] tol        outer tolerance                                   */
/* params[1] eps_A      inner tolerance for A                             */
/* params[2] eps_S      inner tolerance for the SIMPLE matrix             */
/* params[3] max_outer                                                    */
/* params[4] max_inner                                                    */
/* params[5] stop_prec  0: ||r||/||r0|| < tol; 1: ||z||/||z0|| < tol      */
/* params[6] true_u     1: also recompute u = A^{-1}(f - B^T p)           */
/* params[7] zero_rhs_factor  g = B u0 counts as zero when ||g|| <=       */
/*           zero_rhs_factor * eps_A * sqrt(f . u0): since S has no       */
/*           eigenvalue above 1 (Sec. 4.2.2), an exact g obeys            */
/*           ||g||^2 <= f . A^{-1} f, and an inner residual r_A moves g   */
/*           by at most ||A^{-1/2} r_A||; below the floor g is the inner  */
/*           solve's error (channels along the force, exact g = 0)        */
/*                                                                        */
/* stats (double[24]):                                                    */
/*  0 k_hat  1 k_vox  2 outer  3 inner_A  4 inner_S  5 rel_res            */
/*  6 rel_res_prec  7 ||B u|| (recursive u)  8 status  9 ||r0||  10 ||z0||*/
/*  11 k_hat (true u)  12 ||B u_true||  13..15 mean velocity (voxel units)*/
/*  16 seconds  17 threads  18 1 when g counted as zero  19 f . u0      */
/* hist (double[hist_cap][8]) per outer iteration k = 1..:                */
/*  ||r_k||/||r_0||, ||z_k||/||z_0||, k_hat(u_k), inner A, inner S,       */
/*  alpha_{k-1}, beta_{k-1} (0 when the loop stopped first), unused       */
/* ---------------------------------------------------------------------- */
static double khat_of(const osys_t *s, const double *u, double mean_out[3])
{
    double m[3] = {0, 0, 0};
    for (long r = 0; r < s->nf; ++r) {
        int c = (int)(s->face_pos[r] / s->n3);
        m[c] += u[r];
    }
    double f2 = 0.0, fu = 0.0;
    for (int c = 0; c < 3; ++c) {
        m[c] /= (double)s->n3;            /* voxel-unit mean velocity over the box */
        f2 += s->force[c] * s->force[c];
        fu += s->force[c] * m[c];
        if (mean_out) mean_out[c] = m[c];
    }
    return fu / f2;                       /* permeability in voxel units */
}

/* As oracle_solve, with a given right-hand side: g_dense (N^3 doubles, read on
 * the fluid cells) replaces g = B A^{-1} f, the loop starts from p0 = 0 and
 * u0 = 0 (the recursive velocity is then -A^{-1} B^T p), and only an exactly
 * zero g skips the loop.  g_dense == NULL is oracle_solve itself. */
int oracle_solve_g(const osys_t *s, int precond, const double *params, const double *g_dense,
                   double *p_dense, double *u_dense, double *stats, double *hist, int hist_cap);

int oracle_solve(const osys_t *s, int precond, const double *params,
                 double *p_dense, double *u_dense, double *stats, double *hist, int hist_cap)
{
    return oracle_solve_g(s, precond, params, NULL, p_dense, u_dense, stats, hist, hist_cap);
}

int oracle_solve_g(const osys_t *s, int precond, const double *params, const double *g_dense,
                   double *p_dense, double *u_dense, double *stats, double *hist, int hist_cap)
{
    const long nf = s->nf, nc = s->nc;
    const double tol = params[0], epsA = params[1], epsS = params[2];
    const int max_outer = (int)params[3], max_inner = (int)params[4];
    const int stop_prec = (int)params[5], true_u = (int)params[6];
    const double zero_rhs_factor = params[7];
    const double N2 = (double)s->N * (double)s->N;
    int status = 0, inner_st = 0;
    long innerA = 0, innerS = 0;
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    memset(stats, 0, 24 * sizeof(double));

    long nfa = nf > 0 ? nf : 1, nca = nc > 0 ? nc : 1;
    double *f = (double *)calloc(nfa, sizeof(double));
    double *u = (double *)calloc(nfa, sizeof(double));
    double *w = (double *)calloc(nfa, sizeof(double));
    double *v = (double *)calloc(nfa, sizeof(double));
    double *ftmp = (double *)calloc(nfa, sizeof(double));
    double *p = (double *)calloc(nca, sizeof(double));
    double *r = (double *)calloc(nca, sizeof(double));
    double *z = (double *)calloc(nca, sizeof(double));
    double *d = (double *)calloc(nca, sizeof(double));
    double *q = (double *)calloc(nca, sizeof(double));
    opctx_t opA = {s, 0, NULL}, opS = {s, 1, ftmp};

    for (long i = 0; i < nf; ++i) f[i] = s->force[s->face_pos[i] / s->n3];

    if (g_dense) {
        /* p0 = 0, u0 = 0: r0 = g */
        gather_cells(s, g_dense, r);
    } else {
        /* p0 = 0: u0 = A^{-1} f, r0 = g - S p0 = B u0 */
        innerA += pcg(&opA, nf, s->diagA, f, u, epsA, max_inner, &inner_st);
        spmv(&s->B, u, r);
    }
    project(s, r);

#define PRECOND(rr, zz)                                                         \
    do {                                                                        \
        if (precond == 0) memcpy(zz, rr, nca * sizeof(double));                 \
        else {                                                                  \
            innerS += pcg(&opS, nc, s->diagS, rr, zz, epsS, max_inner, &inner_st); \
            project(s, zz);                                                     \
        }                                                                       \
    } while (0)

    PRECOND(r, z);
    memcpy(d, z, nca * sizeof(double));
    double rz = dot(nc, r, z);
    double r0 = nrm2(nc, r), z0 = nrm2(nc, z);
    double rel = 0.0, relz = 0.0;
    double fu0 = dot(nf, f, u);
    double g_floor = (fu0 > 0.0 && !g_dense) ? zero_rhs_factor * epsA * sqrt(fu0) : 0.0;
    int k = 0;
    if (r0 > g_floor) {
        for (k = 0; k < max_outer;) {
            long ia0 = innerA, is0 = innerS;
            spmv(&s->BT, d, w);                                 /* w = B^T d */
            innerA += pcg(&opA, nf, s->diagA, w, v, epsA, max_inner, &inner_st);
            spmv(&s->B, v, q);                                  /* q = S d   */
            double dq = dot(nc, d, q);
            if (!(dq > 0.0)) { status = -4; break; }
            double alpha = rz / dq;
            for (long i = 0; i < nc; ++i) { p[i] += alpha * d[i]; r[i] -= alpha * q[i]; }
            for (long i = 0; i < nf; ++i) u[i] -= alpha * v[i];
            project(s, r);
            PRECOND(r, z);
            ++k;
            rel = nrm2(nc, r) / r0;
            relz = nrm2(nc, z) / z0;
            double beta = 0.0;
            int stop = stop_prec ? (relz < tol) : (rel < tol);
            if (!stop) {
                double rz_new = dot(nc, r, z);
                beta = rz_new / rz;
                rz = rz_new;
                for (long i = 0; i < nc; ++i) d[i] = z[i] + beta * d[i];
            }
            if (hist && k <= hist_cap) {
                double *h = hist + 8 * (k - 1);
                h[0] = rel; h[1] = relz;
                h[2] = khat_of(s, u, NULL) / N2;
                h[3] = (double)(innerA - ia0);
                h[4] = (double)(innerS - is0);
                h[5] = alpha; h[6] = beta; h[7] = 0.0;
            }
            if (stop) break;
        }
        if (status == 0 && k >= max_outer && !(stop_prec ? (relz < tol) : (rel < tol))) status = 1;
    }
    project(s, p);
    if (inner_st == -4 && status == 0) status = -4;

    double mean[3];
    double kvox = khat_of(s, u, mean);
    spmv(&s->B, u, q);
    stats[0] = kvox / N2;
    stats[1] = kvox;
    stats[2] = k;
    stats[3] = (double)innerA;
    stats[4] = (double)innerS;
    stats[5] = rel;
    stats[6] = relz;
    stats[7] = nrm2(nc, q);
    stats[8] = status;
    stats[9] = r0;
    stats[10] = z0;
    stats[18] = r0 > g_floor ? 0.0 : 1.0;
    stats[19] = fu0;
    stats[13] = mean[0]; stats[14] = mean[1]; stats[15] = mean[2];
    if (true_u) {
        /* u_true = A^{-1}(f - B^T p) */
        spmv(&s->BT, p, w);
        for (long i = 0; i < nf; ++i) w[i] = f[i] - w[i];
        int st2 = 0;
        pcg(&opA, nf, s->diagA, w, v, epsA, max_inner, &st2);
        stats[11] = khat_of(s, v, NULL) / N2;
        spmv(&s->B, v, q);
        stats[12] = nrm2(nc, q);
    }
    if (p_dense) scatter_cells(s, p, p_dense);
    if (u_dense) scatter_faces(s, u, u_dense);
    clock_gettime(CLOCK_MONOTONIC, &t1);
    stats[16] = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
#ifdef _OPENMP
    stats[17] = omp_get_max_threads();
#else
    stats[17] = 1;
#endif
#undef PRECOND
    free(f); free(u); free(w); free(v); free(ftmp);
    free(p); free(r); free(z); free(d); free(q);
    return status;
}

/* One inner solve on its own, for tests: which = 0 solves A x = b (faces),
 * which = 1 solves the SIMPLE system (cells; b is projected first and x
 * after).  Returns the iteration count (negative on breakdown). */
int oracle_inner_solve(const osys_t *s, int which, const double *b_dense, double *x_dense,
                       double eps, int maxit)
{
    int st = 0, it;
    if (which == 0) {
        long n = s->nf > 0 ? s->nf : 1;
        double *b = (double *)calloc(n, sizeof(double)), *x = (double *)calloc(n, sizeof(double));
        gather_faces(s, b_dense, b);
        opctx_t o = {s, 0, NULL};
        it = pcg(&o, s->nf, s->diagA, b, x, eps, maxit, &st);
        scatter_faces(s, x, x_dense);
        free(b); free(x);
    } else {
        long n = s->nc > 0 ? s->nc : 1;
        double *b = (double *)calloc(n, sizeof(double)), *x = (double *)calloc(n, sizeof(double));
        double *tmp = (double *)calloc(s->nf > 0 ? s->nf : 1, sizeof(double));
        gather_cells(s, b_dense, b);
        project(s, b);
        opctx_t o = {s, 1, tmp};
        it = pcg(&o, s->nc, s->diagS, b, x, eps, maxit, &st);
        project(s, x);
        scatter_cells(s, x, x_dense);
        free(b); free(x); free(tmp);
    }
    return st < 0 ? -it - 1 : it;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
