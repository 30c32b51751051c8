/*
 * mmoc_oracle.c -- CPU reference ("oracle") for the particle-based modified
 * method of characteristics (Kohl, Mohr, Eibl, Ruede, arXiv 2103.02388).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  The GPU library never links,
 * includes or calls it, and it shares no code with the GPU library.
 *
 * Plain, single-threaded, IEEE double; built with -O2 -ffp-contract=off so
 * that every product and sum is rounded as written.  Speed is not a goal.
 *
 * What it computes (one MMOC advection step, Alg. 1 departure-point and
 * advection lines; Sec. 2.3.1 steps (i)-(iii); Sec. 2.3.2 field evaluation):
 *
 *   (i)   one particle per P2 degree of freedom x_i (vertices and edge
 *         midpoints of the uniformly refined mesh, Sec. 2.3.1 and 2.2);
 *   (ii)  X_i = x_i - int_{t_n}^{t_{n+1}} u(X(x_i,t_{n+1},t),t) dt  (eq.
 *         departure-point), integrated backwards with the classical RK4
 *         tableau (Sec. 3.1) in S sub-steps of h = dt/S, the velocity being
 *         interpolated linearly in time between u_h^n and u_h^{n+1}
 *         (eq. linear-interpolation);
 *   (iii) chat_i = c_h^n(X_i).
 *
 * Field evaluation (Sec. 2.3.2): pull the point back to the computational
 * domain, find the macro element by a walk from the macro that held the
 * previous evaluation, find the micro element in O(1) from the macro's
 * reference coordinates, and sum the P2 shape functions.
 *
 * Readings taken where the paper is silent (each also listed in the design
 * notes):
 *   - refinement: the macro's vertex order (v0..vd) induces Kuhn coordinates
 *     w = (s1+s2+s3, s2+s3, s3); the micro simplices are the Freudenthal
 *     simplices of the lattice w in (1/n)Z^d (identical to Bey's rule);
 *   - interface DoFs belong to the lowest-index macro containing them, and
 *     the unique DoF order is macro-major, first occurrence, nodes of a macro
 *     in lexicographic (I, J, K) order with m >= I >= J >= K >= 0;
 *   - walk: stay if min lambda >= -EPS_IN; else hop across the face with the
 *     most negative lambda among faces that have a neighbour (ties: lowest
 *     face); if no such face, the point is outside the domain and stays;
 *     after max_hops hops fall back to brute force (argmax over macros of
 *     min lambda, ties: lowest macro);
 *   - micro element of a point outside its macro: chosen from the clamped
 *     barycentrics, and the element's polynomial is evaluated at the
 *     unclamped point (extrapolation; exact for fields of degree <= 2);
 *   - stage times: theta = 1 - (j + a_s)/S for sub-step j and RK4 node a_s;
 *   - spherical shell and annulus: per-column radial blending
 *     Phi(x) = x (n.x)/(c |x|), Phi^-1(z) = z c |z| / (n.z), with the plane
 *     (2D: line) n.x = c through the tips of the column's unit directions.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EPS_IN 1e-12

enum { F_OUTSIDE = 1, F_MULTIHOP = 2, F_BRUTE = 4, F_NAN = 8 };

typedef struct orc_mesh {
    int dim, level, n, m, nv, nm, blend;
    int order;       /* 2: P2 (DoFs on the lattice of resolution m = 2n); 1: P1 (m = n) */
    double *vert;    /* nv*dim, computational-domain coordinates */
    int32_t *mv;     /* nm*(dim+1) global vertex ids */
    double *v0;      /* nm*dim */
    double *B;       /* nm*dim*dim, row-major, columns v_a - v0 */
    double *Binv;    /* nm*dim*dim, row-major */
    int32_t *nbr;    /* nm*(dim+1): macro across the face opposite local vertex k, or -1 */
    double *pn;      /* nm*3  shell column plane normal */
    double *pc;      /* nm    shell column plane offset */
    int64_t npm;     /* lattice nodes per macro */
    int64_t N;       /* unique DoFs */
    int32_t *uid;    /* nm*npm: unique index of lattice node (macro, idx) */
    int32_t *own;    /* N: owner macro */
    int32_t *olat;   /* N*3: lattice coordinates (I,J,K) in the owner */
} orc_mesh;

/* ---------------------------------------------------------------- lattice */

/* Position of lattice node (I,J,K) (m >= I >= J >= K >= 0) in lexicographic
 * order; equals the number of nodes that precede it in the nested loop
 * "for I, for J <= I, for K <= J". */
static int64_t lat_idx(int dim, int64_t I, int64_t J, int64_t K)
{
    if (dim == 2) return I * (I + 1) / 2 + J;
    return I * (I + 1) * (I + 2) / 6 + J * (J + 1) / 2 + K;
}

int64_t orc_lat_idx(int dim, int I, int J, int K) { return lat_idx(dim, I, J, K); }

/* barycentric weights (times m) of lattice node (I,J,K) w.r.t. v0..vd */
static void lat_weights(int dim, int m, int I, int J, int K, int w[4])
{
    if (dim == 2) { w[0] = m - I; w[1] = I - J; w[2] = J; w[3] = 0; }
    else { w[0] = m - I; w[1] = I - J; w[2] = J - K; w[3] = K; }
}

/* --------------------------------------------------------- blending (shell) */

static void phi_fwd(const orc_mesh *g, int M, const double *x, double *z)
{
    if (!g->blend) { for (int i = 0; i < g->dim; ++i) z[i] = x[i]; return; }
    const double *n = g->pn + 3 * M;
    double nx = 0, r2 = 0;
    for (int i = 0; i < g->dim; ++i) { nx += n[i] * x[i]; r2 += x[i] * x[i]; }
    double f = nx / (g->pc[M] * sqrt(r2));
    for (int i = 0; i < g->dim; ++i) z[i] = x[i] * f;
}

static void phi_inv(const orc_mesh *g, int M, const double *z, double *x)
{
    if (!g->blend) { for (int i = 0; i < g->dim; ++i) x[i] = z[i]; return; }
    const double *n = g->pn + 3 * M;
    double nz = 0, r2 = 0;
    for (int i = 0; i < g->dim; ++i) { nz += n[i] * z[i]; r2 += z[i] * z[i]; }
    double f = g->pc[M] * sqrt(r2) / nz;
    for (int i = 0; i < g->dim; ++i) x[i] = z[i] * f;
}

/* ------------------------------------------------------------- hash table */

typedef struct { uint64_t k[4]; int32_t val; int32_t used; } hslot;
typedef struct { hslot *s; uint64_t cap; } htab;

static uint64_t hmix(const uint64_t k[4])
{
    uint64_t h = 0x9E3779B97F4A7C15ull;
    for (int i = 0; i < 4; ++i) {
        h ^= k[i] + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 31;
    }
    return h;
}

/* returns existing value, or inserts val and returns -1 */
static int32_t hfind_or_insert(htab *t, const uint64_t k[4], int32_t val)
{
    uint64_t i = hmix(k) & (t->cap - 1);
    for (;;) {
        hslot *s = &t->s[i];
        if (!s->used) {
            memcpy(s->k, k, sizeof s->k);
            s->val = val;
            s->used = 1;
            return -1;
        }
        if (!memcmp(s->k, k, sizeof s->k)) return s->val;
        i = (i + 1) & (t->cap - 1);
    }
}

/* ------------------------------------------------------------ mesh set-up */

typedef struct { int32_t g[3]; int32_t M, k; } facerec;

static int dim_g;
static int face_cmp(const void *a, const void *b)
{
    const facerec *x = a, *y = b;
    for (int i = 0; i < dim_g; ++i) {
        if (x->g[i] != y->g[i]) return x->g[i] < y->g[i] ? -1 : 1;
    }
    if (x->M != y->M) return x->M < y->M ? -1 : 1;
    return 0;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

void orc_mesh_free(orc_mesh *g)
{
    if (!g) return;
    free(g->vert); free(g->mv); free(g->v0); free(g->B); free(g->Binv); free(g->nbr);
    free(g->pn); free(g->pc); free(g->uid); free(g->own); free(g->olat);
    free(g);
}

/* Returns NULL on invalid input (bad sizes, degenerate macro, non-manifold
 * face).  order 2: P2 elements (the default); order 1: P1 elements, whose
 * DoFs are the micro vertices (the lattice of resolution m = n). */
orc_mesh *orc_mesh_new_order(int dim, int level, int order, int nv, const double *vert, int nm,
                             const int32_t *mv, int blend)
{
    if (dim < 2 || dim > 3 || level < 0 || level > 10 || nv <= 0 || nm <= 0) return NULL;
    if (order != 1 && order != 2) return NULL;
    orc_mesh *g = calloc(1, sizeof *g);
    int d = dim, nvm = dim + 1;
    g->dim = dim; g->level = level; g->n = 1 << level; g->m = order * g->n; g->order = order;
    g->nv = nv; g->nm = nm; g->blend = blend;
    g->vert = malloc(sizeof(double) * nv * d);
    memcpy(g->vert, vert, sizeof(double) * nv * d);
    g->mv = malloc(sizeof(int32_t) * nm * nvm);
    memcpy(g->mv, mv, sizeof(int32_t) * nm * nvm);
    for (int i = 0; i < nm * nvm; ++i)
        if (mv[i] < 0 || mv[i] >= nv) { orc_mesh_free(g); return NULL; }

    /* affine geometry: x = v0 + B s, s = Binv (x - v0) */
    g->v0 = malloc(sizeof(double) * nm * d);
    g->B = malloc(sizeof(double) * nm * d * d);
    g->Binv = malloc(sizeof(double) * nm * d * d);
    for (int M = 0; M < nm; ++M) {
        const double *p0 = vert + (size_t)mv[M * nvm] * d;
        double *B = g->B + (size_t)M * d * d, *Bi = g->Binv + (size_t)M * d * d;
        for (int i = 0; i < d; ++i) g->v0[M * d + i] = p0[i];
        for (int a = 0; a < d; ++a) {
            const double *pa = vert + (size_t)mv[M * nvm + a + 1] * d;
            for (int i = 0; i < d; ++i) B[i * d + a] = pa[i] - p0[i];
        }
        double scale = 0;
        for (int i = 0; i < d * d; ++i) scale = fmax(scale, fabs(B[i]));
        if (d == 2) {
            double det = B[0] * B[3] - B[1] * B[2];
            if (!(fabs(det) > 1e-12 * scale * scale)) { orc_mesh_free(g); return NULL; }
            Bi[0] = B[3] / det; Bi[1] = -B[1] / det;
            Bi[2] = -B[2] / det; Bi[3] = B[0] / det;
        } else {
            double c00 = B[4] * B[8] - B[5] * B[7];
            double c01 = B[5] * B[6] - B[3] * B[8];
            double c02 = B[3] * B[7] - B[4] * B[6];
            double det = B[0] * c00 + B[1] * c01 + B[2] * c02;
            if (!(fabs(det) > 1e-12 * scale * scale * scale)) { orc_mesh_free(g); return NULL; }
            Bi[0] = c00 / det;
            Bi[1] = (B[2] * B[7] - B[1] * B[8]) / det;
            Bi[2] = (B[1] * B[5] - B[2] * B[4]) / det;
            Bi[3] = c01 / det;
            Bi[4] = (B[0] * B[8] - B[2] * B[6]) / det;
            Bi[5] = (B[2] * B[3] - B[0] * B[5]) / det;
            Bi[6] = c02 / det;
            Bi[7] = (B[1] * B[6] - B[0] * B[7]) / det;
            Bi[8] = (B[0] * B[4] - B[1] * B[3]) / det;
        }
    }

    /* radial blending: the column of a macro is spanned by its d distinct
     * unit directions (a shell prism in 3D, an annulus sector in 2D); its
     * plane (line in 2D) n.x = c passes through their tips, n unit, c > 0 */
    if (blend) {
        g->pn = calloc((size_t)nm * 3, sizeof(double));
        g->pc = malloc(sizeof(double) * nm);
        for (int M = 0; M < nm; ++M) {
            double dirs[4][3] = {{0}};
            int nd = 0;
            for (int a = 0; a < nvm; ++a) {
                const double *p = vert + (size_t)mv[M * nvm + a] * d;
                double r2 = 0;
                for (int i = 0; i < d; ++i) r2 += p[i] * p[i];
                double q[3] = {0, 0, 0};
                for (int i = 0; i < d; ++i) q[i] = p[i] / sqrt(r2);
                int dup = 0;
                for (int b = 0; b < nd; ++b) {
                    double e = fabs(q[0] - dirs[b][0]) + fabs(q[1] - dirs[b][1]) + fabs(q[2] - dirs[b][2]);
                    if (e < 1e-9) dup = 1;
                }
                if (!dup && nd < 4) { memcpy(dirs[nd], q, sizeof q); ++nd; }
            }
            if (nd != d) { orc_mesh_free(g); return NULL; }
            double nn[3];
            if (d == 3) {
                double e1[3], e2[3];
                for (int i = 0; i < 3; ++i) { e1[i] = dirs[1][i] - dirs[0][i]; e2[i] = dirs[2][i] - dirs[0][i]; }
                nn[0] = e1[1] * e2[2] - e1[2] * e2[1];
                nn[1] = e1[2] * e2[0] - e1[0] * e2[2];
                nn[2] = e1[0] * e2[1] - e1[1] * e2[0];
            } else {
                /* normal of the chord between the two directions */
                nn[0] = -(dirs[1][1] - dirs[0][1]);
                nn[1] = dirs[1][0] - dirs[0][0];
                nn[2] = 0;
            }
            double ln = sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
            double c = (nn[0] * dirs[0][0] + nn[1] * dirs[0][1] + nn[2] * dirs[0][2]) / ln;
            double sgn = c < 0 ? -1.0 : 1.0;
            for (int i = 0; i < 3; ++i) g->pn[M * 3 + i] = sgn * nn[i] / ln;
            g->pc[M] = sgn * c;
        }
    }

    /* face neighbours by matching sorted vertex-id tuples */
    g->nbr = malloc(sizeof(int32_t) * nm * nvm);
    facerec *fr = malloc(sizeof(facerec) * nm * nvm);
    for (int M = 0; M < nm; ++M) {
        for (int k = 0; k < nvm; ++k) {
            facerec *f = &fr[M * nvm + k];
            int c = 0;
            for (int a = 0; a < nvm; ++a) if (a != k) f->g[c++] = mv[M * nvm + a];
            qsort(f->g, d, sizeof(int32_t), cmp_i32);
            if (d == 2) f->g[2] = 0;
            f->M = M; f->k = k;
            g->nbr[M * nvm + k] = -1;
        }
    }
    dim_g = d;
    qsort(fr, (size_t)nm * nvm, sizeof(facerec), face_cmp);
    for (size_t i = 0; i < (size_t)nm * nvm;) {
        size_t j = i + 1;
        while (j < (size_t)nm * nvm && !memcmp(fr[j].g, fr[i].g, sizeof(int32_t) * d)) ++j;
        if (j - i > 2) { free(fr); orc_mesh_free(g); return NULL; }
        if (j - i == 2) {
            g->nbr[fr[i].M * nvm + fr[i].k] = fr[i + 1].M;
            g->nbr[fr[i + 1].M * nvm + fr[i + 1].k] = fr[i].M;
        }
        i = j;
    }
    free(fr);

    /* unique DoF enumeration: macro-major, first occurrence */
    int m = g->m;
    g->npm = (d == 2) ? (int64_t)(m + 1) * (m + 2) / 2 : (int64_t)(m + 1) * (m + 2) * (m + 3) / 6;
    int64_t total = g->npm * nm;
    if (total > 0x7fffffffLL) { orc_mesh_free(g); return NULL; }
    g->uid = malloc(sizeof(int32_t) * total);
    int64_t nbound = 0;
    for (int I = 0; I <= m; ++I)
        for (int J = 0; J <= I; ++J)
            for (int K = 0; K <= (d == 3 ? J : 0); ++K) {
                int w[4];
                lat_weights(d, m, I, J, K, w);
                int interior = 1;
                for (int a = 0; a < nvm; ++a) if (w[a] == 0) interior = 0;
                if (!interior) ++nbound;
            }
    htab t;
    t.cap = 1;
    while (t.cap < (uint64_t)(2 * nbound * nm + 16)) t.cap <<= 1;
    t.s = calloc(t.cap, sizeof(hslot));
    int32_t *own = malloc(sizeof(int32_t) * total);
    int32_t *olat = malloc(sizeof(int32_t) * total * 3);
    int64_t N = 0;
    for (int M = 0; M < nm; ++M) {
        int64_t idx = 0;
        for (int I = 0; I <= m; ++I)
            for (int J = 0; J <= I; ++J)
                for (int K = 0; K <= (d == 3 ? J : 0); ++K, ++idx) {
                    int w[4];
                    lat_weights(d, m, I, J, K, w);
                    int interior = 1;
                    for (int a = 0; a < nvm; ++a) if (w[a] == 0) interior = 0;
                    int32_t u;
                    int created = 0;
                    if (interior) {
                        u = (int32_t)N++;
                        created = 1;
                    } else {
                        /* key: (global id, weight) pairs of the nonzero weights, sorted by id */
                        uint64_t key[4];
                        int c = 0;
                        for (int a = 0; a < nvm; ++a)
                            if (w[a] > 0) key[c++] = ((uint64_t)(uint32_t)mv[M * nvm + a] << 32) | (uint32_t)w[a];
                        for (int x = 1; x < c; ++x)
                            for (int y = x; y > 0 && key[y - 1] > key[y]; --y) {
                                uint64_t tmp = key[y]; key[y] = key[y - 1]; key[y - 1] = tmp;
                            }
                        for (; c < 4; ++c) key[c] = ~0ull;
                        int32_t old = hfind_or_insert(&t, key, (int32_t)N);
                        if (old >= 0) {
                            u = old;
                        } else {
                            u = (int32_t)N++;
                            created = 1;
                        }
                    }
                    g->uid[M * g->npm + idx] = u;
                    if (created) {
                        own[u] = M;
                        olat[3 * (int64_t)u + 0] = I;
                        olat[3 * (int64_t)u + 1] = J;
                        olat[3 * (int64_t)u + 2] = K;
                    }
                }
    }
    free(t.s);
    g->N = N;
    g->own = realloc(own, sizeof(int32_t) * N);
    g->olat = realloc(olat, sizeof(int32_t) * N * 3);
    return g;
}

orc_mesh *orc_mesh_new(int dim, int level, int nv, const double *vert, int nm, const int32_t *mv, int blend)
{
    return orc_mesh_new_order(dim, level, 2, nv, vert, nm, mv, blend);
}

int64_t orc_num_dofs(const orc_mesh *g) { return g->N; }
int64_t orc_nodes_per_macro(const orc_mesh *g) { return g->npm; }

void orc_macro_geometry(const orc_mesh *g, int M, double *v0, double *B, double *Binv, int32_t *nbr)
{
    int d = g->dim;
    memcpy(v0, g->v0 + (size_t)M * d, sizeof(double) * d);
    memcpy(B, g->B + (size_t)M * d * d, sizeof(double) * d * d);
    memcpy(Binv, g->Binv + (size_t)M * d * d, sizeof(double) * d * d);
    memcpy(nbr, g->nbr + (size_t)M * (d + 1), sizeof(int32_t) * (d + 1));
}

void orc_plane(const orc_mesh *g, int M, double *n, double *c)
{
    if (!g->blend) return;
    memcpy(n, g->pn + 3 * M, sizeof(double) * 3);
    *c = g->pc[M];
}

/* physical position of lattice node (I,J,K) of macro M: Phi(v0 + B s) */
static void node_pos(const orc_mesh *g, int M, int I, int J, int K, double *x)
{
    int d = g->dim;
    double s[3];
    if (d == 2) { s[0] = (double)(I - J) / g->m; s[1] = (double)J / g->m; }
    else { s[0] = (double)(I - J) / g->m; s[1] = (double)(J - K) / g->m; s[2] = (double)K / g->m; }
    const double *v0 = g->v0 + (size_t)M * d, *B = g->B + (size_t)M * d * d;
    double p[3];
    for (int i = 0; i < d; ++i) {
        double acc = v0[i];
        for (int a = 0; a < d; ++a) acc = acc + B[i * d + a] * s[a];
        p[i] = acc;
    }
    phi_fwd(g, M, p, x);
}

/* DoF coordinates, SoA [dim][N] */
void orc_dof_coords(const orc_mesh *g, double *out)
{
    for (int64_t u = 0; u < g->N; ++u) {
        double x[3];
        node_pos(g, g->own[u], g->olat[3 * u], g->olat[3 * u + 1], g->olat[3 * u + 2], x);
        for (int i = 0; i < g->dim; ++i) out[(size_t)i * g->N + u] = x[i];
    }
}

void orc_dof_owner(const orc_mesh *g, int32_t *own, int32_t *lat)
{
    memcpy(own, g->own, sizeof(int32_t) * g->N);
    memcpy(lat, g->olat, sizeof(int32_t) * 3 * g->N);
}

/* unique index of every (macro, lattice idx) slot, [nm][npm] */
void orc_slot_uids(const orc_mesh *g, int32_t *out)
{
    memcpy(out, g->uid, sizeof(int32_t) * g->nm * g->npm);
}

/* ------------------------------------------------------------ location */

/* barycentric coordinates of physical point y w.r.t. macro M; s = lam[1..d] */
void orc_bary(const orc_mesh *g, int M, const double *y, double *lam)
{
    int d = g->dim;
    double p[3], q[3];
    phi_inv(g, M, y, p);
    const double *v0 = g->v0 + (size_t)M * d, *Bi = g->Binv + (size_t)M * d * d;
    for (int i = 0; i < d; ++i) q[i] = p[i] - v0[i];
    double sum = 0;
    for (int a = 0; a < d; ++a) {
        double acc = 0;
        for (int i = 0; i < d; ++i) acc = acc + Bi[a * d + i] * q[i];
        lam[a + 1] = acc;
        sum = sum + acc;
    }
    lam[0] = 1.0 - sum;
}

static double lam_min(int d, const double *lam)
{
    double mn = lam[0];
    for (int a = 1; a <= d; ++a) if (lam[a] < mn) mn = lam[a];
    return mn;
}

int orc_brute(const orc_mesh *g, const double *y)
{
    int best = 0;
    double bestv = -INFINITY;
    for (int M = 0; M < g->nm; ++M) {
        double lam[4];
        orc_bary(g, M, y, lam);
        double v = lam_min(g->dim, lam);
        if (v > bestv) { bestv = v; best = M; }
    }
    return best;
}

int orc_walk(const orc_mesh *g, int M, const double *y, int max_hops, int *flags)
{
    int d = g->dim;
    for (int hop = 0;; ++hop) {
        double lam[4];
        orc_bary(g, M, y, lam);
        if (lam_min(d, lam) >= -EPS_IN) return M;
        int kb = -1;
        for (int k = 0; k <= d; ++k)
            if (lam[k] < -EPS_IN && g->nbr[M * (d + 1) + k] >= 0 && (kb < 0 || lam[k] < lam[kb])) kb = k;
        if (kb < 0) { *flags |= F_OUTSIDE; return M; }
        if (hop >= max_hops) break;
        if (hop >= 1) *flags |= F_MULTIHOP;
        M = g->nbr[M * (d + 1) + kb];
    }
    *flags |= F_BRUTE;
    int Mb = orc_brute(g, y);
    double lam[4];
    orc_bary(g, Mb, y, lam);
    if (lam_min(d, lam) < -EPS_IN) *flags |= F_OUTSIDE;
    return Mb;
}

typedef struct {
    int V[4][3];      /* micro vertices in the n-lattice (Kuhn coordinates) */
    double mu[4];     /* micro barycentrics of the (unclamped) point */
    int64_t slot[10]; /* lattice idx of the P2 nodes: d+1 vertices, then edges (a<b) */
    double phi[10];   /* P2 shape function values */
    int nn;
} orc_loc;

/* Kuhn coordinates by nested sums: w_d = s_d, w_a = s_a + w_{a+1} */
static void kuhn(int d, const double *s, double *w)
{
    w[d - 1] = s[d - 1];
    for (int a = d - 2; a >= 0; --a) w[a] = s[a] + w[a + 1];
}

static void micro_locate(const orc_mesh *g, int M, const double *y, orc_loc *L)
{
    int d = g->dim, n = g->n;
    double lam[4] = {0}, s[3] = {0}, ssel[3] = {0}, W[3] = {0}, Wu[3] = {0}, f[3] = {0}, fu[3] = {0};
    orc_bary(g, M, y, lam);
    for (int a = 0; a < d; ++a) s[a] = lam[a + 1];
    if (lam_min(d, lam) >= 0) {
        for (int a = 0; a < d; ++a) ssel[a] = s[a];
    } else {
        double lp[4], sum = 0;
        for (int a = 0; a <= d; ++a) { lp[a] = lam[a] > 0 ? lam[a] : 0; sum = sum + lp[a]; }
        for (int a = 0; a < d; ++a) ssel[a] = lp[a + 1] / sum;
    }
    kuhn(d, ssel, W);
    kuhn(d, s, Wu);
    int k[3];
    for (int i = 0; i < d; ++i) {
        W[i] = W[i] * n;
        Wu[i] = Wu[i] * n;
        double fl = floor(W[i]);
        k[i] = (int)fl;
        if (k[i] > n - 1) k[i] = n - 1;
        if (k[i] < 0) k[i] = 0;
        f[i] = W[i] - k[i];
        fu[i] = Wu[i] - k[i];
    }
    /* axes by descending f; a stable insertion sort keeps ties in ascending axis order */
    int pi[3] = {0, 1, 2};
    for (int i = 1; i < d; ++i)
        for (int j = i; j > 0 && f[pi[j]] > f[pi[j - 1]]; --j) {
            int t = pi[j]; pi[j] = pi[j - 1]; pi[j - 1] = t;
        }
    for (int i = 0; i < d; ++i) L->V[0][i] = k[i];
    for (int a = 1; a <= d; ++a) {
        for (int i = 0; i < d; ++i) L->V[a][i] = L->V[a - 1][i];
        L->V[a][pi[a - 1]] += 1;
    }
    L->mu[0] = 1.0 - fu[pi[0]];
    for (int a = 1; a < d; ++a) L->mu[a] = fu[pi[a - 1]] - fu[pi[a]];
    L->mu[d] = fu[pi[d - 1]];
    int c = 0;
    if (g->order == 1) {
        /* P1: the vertices V_a themselves (m = n), shape functions mu_a */
        for (int a = 0; a <= d; ++a) {
            int P[3] = {0, 0, 0};
            for (int i = 0; i < d; ++i) P[i] = L->V[a][i];
            L->slot[c] = lat_idx(d, P[0], P[1], P[2]);
            L->phi[c] = L->mu[a];
            ++c;
        }
        L->nn = c;
        return;
    }
    /* P2 nodes: 2 V_a (vertices) and V_a + V_b (edge midpoints), m-lattice */
    for (int a = 0; a <= d; ++a) {
        int P[3] = {0, 0, 0};
        for (int i = 0; i < d; ++i) P[i] = 2 * L->V[a][i];
        L->slot[c] = lat_idx(d, P[0], P[1], P[2]);
        L->phi[c] = L->mu[a] * (2.0 * L->mu[a] - 1.0);
        ++c;
    }
    for (int a = 0; a <= d; ++a)
        for (int b = a + 1; b <= d; ++b) {
            int P[3] = {0, 0, 0};
            for (int i = 0; i < d; ++i) P[i] = L->V[a][i] + L->V[b][i];
            L->slot[c] = lat_idx(d, P[0], P[1], P[2]);
            L->phi[c] = 4.0 * L->mu[a] * L->mu[b];
            ++c;
        }
    L->nn = c;
}

/* Exposed for tests: micro simplex (n-lattice vertices, [d+1][3]) and micro
 * barycentrics chosen for point y in macro M. */
void orc_micro_simplex(const orc_mesh *g, int M, const double *y, int32_t *V, double *mu)
{
    orc_loc L;
    micro_locate(g, M, y, &L);
    for (int a = 0; a <= g->dim; ++a) {
        for (int i = 0; i < 3; ++i) V[a * 3 + i] = L.V[a][i];
        mu[a] = L.mu[a];
    }
}

static double eval_loc(const orc_mesh *g, int M, const orc_loc *L, const double *f)
{
    double acc = 0;
    for (int i = 0; i < L->nn; ++i) acc = acc + L->phi[i] * f[g->uid[M * g->npm + L->slot[i]]];
    return acc;
}

/* Evaluate ncomp P2 fields (SoA [ncomp][N]) at npts physical points (AoS
 * [npts][dim]).  start: per-point starting macro for the walk, or NULL for
 * brute-force location.  macro_out (optional) receives the macro used. */
void orc_eval(const orc_mesh *g, int ncomp, const double *field, int64_t npts, const double *pts,
              const int32_t *start, int max_hops, double *out, int32_t *macro_out, int32_t *flags_out)
{
    for (int64_t p = 0; p < npts; ++p) {
        const double *y = pts + (size_t)p * g->dim;
        int flags = 0;
        int M = start ? orc_walk(g, start[p], y, max_hops, &flags) : orc_brute(g, y);
        orc_loc L;
        micro_locate(g, M, y, &L);
        for (int c = 0; c < ncomp; ++c) out[(size_t)p * ncomp + c] = eval_loc(g, M, &L, field + (size_t)c * g->N);
        if (macro_out) macro_out[p] = M;
        if (flags_out) flags_out[p] = flags;
    }
}

/* ---------------------------------------------------------------- trace */

/* One MMOC advection step for the particles ids[0..n_ids) (all if ids==NULL,
 * then n_ids must equal N).  u0/u1: velocity at t_n / t_{n+1}, SoA
 * [dim][N]; u1 == NULL means the two levels are identical.  c: scalar at t_n.
 * Outputs chat[q] and X (SoA [dim][n_ids]).  stats[0..3] += number of
 * particles flagged outside / multi-hop / brute-force / NaN. */
int orc_trace(const orc_mesh *g, const double *u0, const double *u1, const double *c,
              double dt, int S, int max_hops, int64_t n_ids, const int64_t *ids,
              double *chat, double *X, int64_t *stats)
{
    if (!(dt > 0) || S < 1) return -1;
    int d = g->dim;
    double h = dt / S;
    static const double a_s[4] = {0.0, 0.5, 0.5, 1.0};
    for (int64_t q = 0; q < n_ids; ++q) {
        int64_t i = ids ? ids[q] : q;
        int M = g->own[i];
        int flags = 0;
        double Y[3], y[3], k[4][3];
        node_pos(g, M, g->olat[3 * i], g->olat[3 * i + 1], g->olat[3 * i + 2], Y);
        for (int j = 0; j < S; ++j) {
            for (int st = 0; st < 4; ++st) {
                /* stage point: Y, Y - h/2 k1, Y - h/2 k2, Y - h k3 */
                for (int x = 0; x < d; ++x) {
                    if (st == 0) y[x] = Y[x];
                    else if (st == 3) y[x] = Y[x] - h * k[2][x];
                    else y[x] = Y[x] - 0.5 * h * k[st - 1][x];
                }
                double theta = 1.0 - (j + a_s[st]) / S;
                M = orc_walk(g, M, y, max_hops, &flags);
                orc_loc L;
                micro_locate(g, M, y, &L);
                for (int x = 0; x < d; ++x) {
                    double ua = eval_loc(g, M, &L, u0 + (size_t)x * g->N);
                    if (u1) {
                        double ub = eval_loc(g, M, &L, u1 + (size_t)x * g->N);
                        k[st][x] = (1.0 - theta) * ua + theta * ub;
                    } else {
                        k[st][x] = ua;
                    }
                }
            }
            for (int x = 0; x < d; ++x)
                Y[x] = Y[x] - h / 6.0 * (k[0][x] + 2.0 * k[1][x] + 2.0 * k[2][x] + k[3][x]);
        }
        M = orc_walk(g, M, Y, max_hops, &flags);
        orc_loc L;
        micro_locate(g, M, Y, &L);
        double v = eval_loc(g, M, &L, c);
        chat[q] = v;
        int bad = v != v;
        for (int x = 0; x < d; ++x) {
            if (X) X[(size_t)x * n_ids + q] = Y[x];
            if (Y[x] != Y[x]) bad = 1;
        }
        if (bad) flags |= F_NAN;
        if (stats) {
            if (flags & F_OUTSIDE) stats[0]++;
            if (flags & F_MULTIHOP) stats[1]++;
            if (flags & F_BRUTE) stats[2]++;
            if (flags & F_NAN) stats[3]++;
        }
    }
    return 0;
}

/* ------------------------------------------- traces across steps, general RK */

/* A trace across several time steps (look-back b > 1 with a time-dependent
 * velocity, Sec. 2.3.3): the velocity is known at the levels t_l = t_0 + l
 * tau, l = 0..n_int (U[l], each [dim][N]), and is linear in time on every
 * interval [t_l, t_{l+1}] (eq. linear-interpolation, interval by interval).
 * A particle at its DoF at t_{n_int} is traced back to t_0 with S classical
 * RK4 sub-steps per interval (h = tau/S), and c (known at t_0) is evaluated
 * at the departure point.  The stage of sub-step jj (0 at the latest time)
 * with RK4 node a_s sits p = (jj + a_s)/S intervals before t_{n_int}; it lies
 * in interval q = min(floor(p), n_int - 1) counted from the end, at weight
 * theta = 1 - (p - q) of that interval's later level. */
int orc_trace_span(const orc_mesh *g, const double *const *U, int n_int, const double *c, double tau, int S,
                   int max_hops, int64_t n_ids, const int64_t *ids, double *chat, double *X, int64_t *stats)
{
    if (!(tau > 0) || S < 1 || n_int < 1) return -1;
    int d = g->dim;
    double h = tau / S;
    static const double a_s[4] = {0.0, 0.5, 0.5, 1.0};
    for (int64_t q = 0; q < n_ids; ++q) {
        int64_t i = ids ? ids[q] : q;
        int M = g->own[i];
        int flags = 0;
        double Y[3], y[3], k[4][3];
        node_pos(g, M, g->olat[3 * i], g->olat[3 * i + 1], g->olat[3 * i + 2], Y);
        for (int jj = 0; jj < n_int * S; ++jj) {
            for (int st = 0; st < 4; ++st) {
                for (int x = 0; x < d; ++x) {
                    if (st == 0) y[x] = Y[x];
                    else if (st == 3) y[x] = Y[x] - h * k[2][x];
                    else y[x] = Y[x] - 0.5 * h * k[st - 1][x];
                }
                double pos = (jj + a_s[st]) / S;
                int iv = (int)floor(pos);
                if (iv > n_int - 1) iv = n_int - 1;
                double theta = 1.0 - (pos - iv);
                const double *late = U[n_int - iv], *early = U[n_int - iv - 1];
                M = orc_walk(g, M, y, max_hops, &flags);
                orc_loc L;
                micro_locate(g, M, y, &L);
                for (int x = 0; x < d; ++x) {
                    double ua = eval_loc(g, M, &L, early + (size_t)x * g->N);
                    double ub = eval_loc(g, M, &L, late + (size_t)x * g->N);
                    k[st][x] = (1.0 - theta) * ua + theta * ub;
                }
            }
            for (int x = 0; x < d; ++x)
                Y[x] = Y[x] - h / 6.0 * (k[0][x] + 2.0 * k[1][x] + 2.0 * k[2][x] + k[3][x]);
        }
        M = orc_walk(g, M, Y, max_hops, &flags);
        orc_loc L;
        micro_locate(g, M, Y, &L);
        double v = eval_loc(g, M, &L, c);
        chat[q] = v;
        int bad = v != v;
        for (int x = 0; x < d; ++x) {
            if (X) X[(size_t)x * n_ids + q] = Y[x];
            if (Y[x] != Y[x]) bad = 1;
        }
        if (bad) flags |= F_NAN;
        if (stats) {
            if (flags & F_OUTSIDE) stats[0]++;
            if (flags & F_MULTIHOP) stats[1]++;
            if (flags & F_BRUTE) stats[2]++;
            if (flags & F_NAN) stats[3]++;
        }
    }
    return 0;
}

/* One advection step with a general explicit Runge-Kutta method (the paper
 * uses RK4 and notes that any explicit RK method applies, Sec. 3.1; Fig. 2
 * shows a two-stage one).  Butcher tableau of ns stages: A [ns][ns]
 * row-major (only the strictly lower part is read), weights b [ns], nodes
 * cn [ns].  Backwards in time, sub-step j of S (h = dt/S):
 *   y_i = Y - h sum_{l<i} A[i][l] k_l,   k_i = u~(y_i; theta_i),
 *   theta_i = 1 - (j + cn[i])/S,         Y <- Y - h sum_i b[i] k_i,
 * with u~ the linear-in-time velocity of eq. linear-interpolation, and the
 * field evaluation, walk and scalar step exactly as in orc_trace. */
int orc_trace_rk(const orc_mesh *g, const double *u0, const double *u1, const double *c,
                 double dt, int S, int ns, const double *A, const double *b, const double *cn,
                 int max_hops, int64_t n_ids, const int64_t *ids,
                 double *chat, double *X, int64_t *stats)
{
    if (!(dt > 0) || S < 1 || ns < 1 || ns > 16) return -1;
    int d = g->dim;
    double h = dt / S;
    for (int64_t q = 0; q < n_ids; ++q) {
        int64_t i = ids ? ids[q] : q;
        int M = g->own[i];
        int flags = 0;
        double Y[3], y[3], k[16][3];
        node_pos(g, M, g->olat[3 * i], g->olat[3 * i + 1], g->olat[3 * i + 2], Y);
        for (int j = 0; j < S; ++j) {
            for (int st = 0; st < ns; ++st) {
                for (int x = 0; x < d; ++x) {
                    double sum = 0.0;
                    for (int l = 0; l < st; ++l) sum += A[st * ns + l] * k[l][x];
                    y[x] = Y[x] - h * sum;
                }
                double theta = 1.0 - (j + cn[st]) / S;
                M = orc_walk(g, M, y, max_hops, &flags);
                orc_loc L;
                micro_locate(g, M, y, &L);
                for (int x = 0; x < d; ++x) {
                    double ua = eval_loc(g, M, &L, u0 + (size_t)x * g->N);
                    if (u1) {
                        double ub = eval_loc(g, M, &L, u1 + (size_t)x * g->N);
                        k[st][x] = (1.0 - theta) * ua + theta * ub;
                    } else {
                        k[st][x] = ua;
                    }
                }
            }
            for (int x = 0; x < d; ++x) {
                double sum = 0.0;
                for (int st = 0; st < ns; ++st) sum += b[st] * k[st][x];
                Y[x] = Y[x] - h * sum;
            }
        }
        M = orc_walk(g, M, Y, max_hops, &flags);
        orc_loc L;
        micro_locate(g, M, Y, &L);
        double v = eval_loc(g, M, &L, c);
        chat[q] = v;
        int bad = v != v;
        for (int x = 0; x < d; ++x) {
            if (X) X[(size_t)x * n_ids + q] = Y[x];
            if (Y[x] != Y[x]) bad = 1;
        }
        if (bad) flags |= F_NAN;
        if (stats) {
            if (flags & F_OUTSIDE) stats[0]++;
            if (flags & F_MULTIHOP) stats[1]++;
            if (flags & F_BRUTE) stats[2]++;
            if (flags & F_NAN) stats[3]++;
        }
    }
    return 0;
}

/* ------------------------------------------------------- P2 mass matrix */

/* Integral over a simplex T of prod_a lambda_a^e_a equals
 * d! |T| prod(e_a!) / (sum e + d)!  (standard barycentric monomial formula). */
static double fact(int k) { double r = 1; for (int i = 2; i <= k; ++i) r *= i; return r; }

static double mono_int(int d, const int e[4])
{
    double num = fact(d);
    int s = 0;
    for (int a = 0; a <= d; ++a) { num *= fact(e[a]); s += e[a]; }
    return num / fact(s + d);
}

/* P2 shape functions as sums of barycentric monomials of degree <= 2 */
typedef struct { int nt; double c[2]; int e[2][4]; } poly2;

static void p2_basis(int d, poly2 *b)
{
    int c = 0;
    for (int a = 0; a <= d; ++a) { /* lambda_a (2 lambda_a - 1) = 2 la^2 - la */
        memset(&b[c], 0, sizeof b[c]);
        b[c].nt = 2; b[c].c[0] = 2.0; b[c].e[0][a] = 2; b[c].c[1] = -1.0; b[c].e[1][a] = 1;
        ++c;
    }
    for (int a = 0; a <= d; ++a)
        for (int bb = a + 1; bb <= d; ++bb) {
            memset(&b[c], 0, sizeof b[c]);
            b[c].nt = 1; b[c].c[0] = 4.0; b[c].e[0][a] = 1; b[c].e[0][bb] = 1;
            ++c;
        }
}

/* reference mass matrix divided by |T|, nb x nb */
void orc_p2_mass_ref(int d, double *Mref)
{
    poly2 b[10];
    p2_basis(d, b);
    int nb = (d + 1) * (d + 2) / 2;
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
            double acc = 0;
            for (int ti = 0; ti < b[i].nt; ++ti)
                for (int tj = 0; tj < b[j].nt; ++tj) {
                    int e[4];
                    for (int a = 0; a < 4; ++a) e[a] = b[i].e[ti][a] + b[j].e[tj][a];
                    acc += b[i].c[ti] * b[j].c[tj] * mono_int(d, e);
                }
            Mref[i * nb + j] = acc;
        }
}

/* Enumerate the micro simplices of one macro: base k with n-1 >= k0 >= k1
 * (>= k2) >= 0 and axis orders pi whose chain k, k+e_pi0, ... stays in the
 * Kuhn simplex (when k_i == k_{i+1}, axis i must come before axis i+1).
 * Writes up to cap simplices as n-lattice vertices [(d+1)][3]; returns count. */
int64_t orc_micro_simplices(const orc_mesh *g, int32_t *V, int64_t cap)
{
    int d = g->dim, n = g->n;
    static const int perms3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int perms2[2][3] = {{0, 1, 2}, {1, 0, 2}};
    int np = d == 3 ? 6 : 2;
    int64_t cnt = 0;
    for (int k0 = 0; k0 < n; ++k0)
        for (int k1 = 0; k1 <= k0; ++k1)
            for (int k2 = 0; k2 <= (d == 3 ? k1 : 0); ++k2)
                for (int p = 0; p < np; ++p) {
                    const int *pi = d == 3 ? perms3[p] : perms2[p];
                    int cur[3] = {k0, k1, k2}, ok = 1, vv[4][3];
                    memcpy(vv[0], cur, sizeof cur);
                    for (int a = 0; a < d; ++a) {
                        cur[pi[a]] += 1;
                        memcpy(vv[a + 1], cur, sizeof cur);
                    }
                    for (int a = 0; a <= d && ok; ++a) {
                        for (int i = 0; i + 1 < d; ++i) if (vv[a][i] < vv[a][i + 1]) ok = 0;
                        if (vv[a][0] > n || vv[a][d - 1] < 0) ok = 0;
                    }
                    if (!ok) continue;
                    if (V && cnt < cap) memcpy(V + cnt * 12, vv, sizeof(int32_t) * 12);
                    ++cnt;
                }
    return cnt;
}

/* P1 reference mass matrix divided by |T|: int lambda_a lambda_b
 * = |T| d! (1 + [a == b]) / (d + 2)! by the monomial formula */
static void p1_mass_ref(int d, double *Mref)
{
    for (int a = 0; a <= d; ++a)
        for (int b = 0; b <= d; ++b) {
            int e[4] = {0, 0, 0, 0};
            e[a] += 1;
            e[b] += 1;
            Mref[a * (d + 1) + b] = mono_int(d, e);
        }
}

/* a^T M b for the mass matrix M of the mesh's elements (P2, or P1 for an
 * order-1 mesh) on the (unblended) mesh; a, b unique [N] */
double orc_mass_quadform(const orc_mesh *g, const double *a, const double *b)
{
    int d = g->dim;
    int nb = g->order == 1 ? d + 1 : (d + 1) * (d + 2) / 2;
    double Mref[100];
    if (g->order == 1) p1_mass_ref(d, Mref);
    else orc_p2_mass_ref(d, Mref);
    int64_t nsimp = orc_micro_simplices(g, NULL, 0);
    int32_t *V = malloc(sizeof(int32_t) * 12 * nsimp);
    orc_micro_simplices(g, V, nsimp);
    double total = 0;
    for (int M = 0; M < g->nm; ++M) {
        const double *B = g->B + (size_t)M * d * d;
        double det = d == 2 ? B[0] * B[3] - B[1] * B[2]
                            : B[0] * (B[4] * B[8] - B[5] * B[7]) - B[1] * (B[3] * B[8] - B[5] * B[6]) +
                                  B[2] * (B[3] * B[7] - B[4] * B[6]);
        double vol = fabs(det) / (d == 2 ? 2.0 : 6.0) / pow((double)g->n, d);
        for (int64_t s = 0; s < nsimp; ++s) {
            int32_t (*vv)[3] = (int32_t (*)[3])(V + s * 12);
            int64_t nodes[10];
            int c = 0;
            if (g->order == 1) {
                for (int x = 0; x <= d; ++x) nodes[c++] = lat_idx(d, vv[x][0], vv[x][1], d == 3 ? vv[x][2] : 0);
            } else {
                for (int x = 0; x <= d; ++x)
                    nodes[c++] = lat_idx(d, 2 * vv[x][0], 2 * vv[x][1], d == 3 ? 2 * vv[x][2] : 0);
                for (int x = 0; x <= d; ++x)
                    for (int y = x + 1; y <= d; ++y)
                        nodes[c++] = lat_idx(d, vv[x][0] + vv[y][0], vv[x][1] + vv[y][1], d == 3 ? vv[x][2] + vv[y][2] : 0);
            }
            double acc = 0;
            for (int i = 0; i < nb; ++i) {
                double ai = a[g->uid[M * g->npm + nodes[i]]];
                for (int j = 0; j < nb; ++j) acc += ai * Mref[i * nb + j] * b[g->uid[M * g->npm + nodes[j]]];
            }
            total += vol * acc;
        }
    }
    free(V);
    return total;
}

/* ------------------------------------------- Galerkin mass and stiffness
 * The matrices M and A of the linear system of the Theta-method (Sec. 2.2,
 * eq. linear-system): M_ij = (phi_j, phi_i), A_ij = (grad phi_j, grad phi_i)
 * over the physical domain Phi(Omega_comp).  On a blended mesh the element
 * map is Phi composed with the affine micro-simplex map, whose Jacobian is
 * not constant; both integrals are then taken with a quadrature rule on the
 * reference simplex that the caller passes in (points qp [nq][d] in
 * reference coordinates, weights qw [nq] summing to the reference volume
 * 1/d!).  Without blending the integrands are polynomials and a rule exact
 * to degree 2*order makes the matrices exact. */

/* Shape functions and their reference gradients at reference point xi:
 * lambda_0 = 1 - sum xi, lambda_a = xi_a; P1: phi_a = lambda_a; P2: the
 * vertex functions lambda_a (2 lambda_a - 1) for a = 0..d, then the edge
 * functions 4 lambda_a lambda_b for a < b in lexicographic order. */
static int shape_fn(int d, int order, const double *xi, double *phi, double dphi[10][3])
{
    double lam[4], dl[4][3];
    memset(dl, 0, sizeof dl);
    lam[0] = 1.0;
    for (int a = 0; a < d; ++a) {
        lam[0] -= xi[a];
        lam[a + 1] = xi[a];
        dl[0][a] = -1.0;
        dl[a + 1][a] = 1.0;
    }
    int c = 0;
    if (order == 1) {
        for (int a = 0; a <= d; ++a, ++c) {
            phi[c] = lam[a];
            for (int i = 0; i < d; ++i) dphi[c][i] = dl[a][i];
        }
        return c;
    }
    for (int a = 0; a <= d; ++a, ++c) {
        phi[c] = lam[a] * (2.0 * lam[a] - 1.0);
        for (int i = 0; i < d; ++i) dphi[c][i] = (4.0 * lam[a] - 1.0) * dl[a][i];
    }
    for (int a = 0; a <= d; ++a)
        for (int b = a + 1; b <= d; ++b, ++c) {
            phi[c] = 4.0 * lam[a] * lam[b];
            for (int i = 0; i < d; ++i) dphi[c][i] = 4.0 * (lam[b] * dl[a][i] + lam[a] * dl[b][i]);
        }
    return c;
}

/* D Phi at computational point x of macro M (row-major d x d):
 * Phi(x) = f(x) x, f = (n.x)/(c |x|), so DPhi = f I + x (grad f)^T with
 * grad f = n/(c |x|) - (n.x) x/(c |x|^3).  The identity without blending. */
static void phi_jacobian(const orc_mesh *g, int M, const double *x, double *D)
{
    int d = g->dim;
    for (int i = 0; i < d * d; ++i) D[i] = 0.0;
    if (!g->blend) {
        for (int i = 0; i < d; ++i) D[i * d + i] = 1.0;
        return;
    }
    const double *n = g->pn + 3 * M;
    double c = g->pc[M], nx = 0, r2 = 0;
    for (int i = 0; i < d; ++i) { nx += n[i] * x[i]; r2 += x[i] * x[i]; }
    double r = sqrt(r2), f = nx / (c * r), gf[3];
    for (int i = 0; i < d; ++i) gf[i] = n[i] / (c * r) - nx * x[i] / (c * r * r2);
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j) D[i * d + j] = x[i] * gf[j];
        D[i * d + i] += f;
    }
}

static double det_inv(int d, const double *J, double *Ji)
{
    if (d == 2) {
        double det = J[0] * J[3] - J[1] * J[2];
        Ji[0] = J[3] / det; Ji[1] = -J[1] / det; Ji[2] = -J[2] / det; Ji[3] = J[0] / det;
        return det;
    }
    double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
    double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
    Ji[0] = c00 / det;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    Ji[3] = c01 / det;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    Ji[6] = c02 / det;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

/* computational position of n-lattice vertex (I,J,K) of macro M */
static void nlat_pos(const orc_mesh *g, int M, const int32_t *v, double *x)
{
    int d = g->dim;
    double s[3];
    if (d == 2) { s[0] = (double)(v[0] - v[1]) / g->n; s[1] = (double)v[1] / g->n; }
    else { s[0] = (double)(v[0] - v[1]) / g->n; s[1] = (double)(v[1] - v[2]) / g->n; s[2] = (double)v[2] / g->n; }
    const double *v0 = g->v0 + (size_t)M * d, *B = g->B + (size_t)M * d * d;
    for (int i = 0; i < d; ++i) {
        double acc = v0[i];
        for (int a = 0; a < d; ++a) acc = acc + B[i * d + a] * s[a];
        x[i] = acc;
    }
}

/* Element matrices of every micro simplex as triplets (row, col, m, a):
 * for each macro, each micro simplex (in orc_micro_simplices order), each
 * local pair (i, j):
 *   m = sum_q w_q phi_i(xi_q) phi_j(xi_q) |det J(xi_q)|,
 *   a = sum_q w_q (J^-T grad phi_i).(J^-T grad phi_j) |det J(xi_q)|,
 * J(xi) = DPhi(x(xi)) [p_1 - p_0, ..., p_d - p_0], x(xi) = p_0 + sum_a
 * xi_a (p_a - p_0) with p_a the simplex's computational vertices.  Rows and
 * columns are unique DoF ids.  Returns the triplet count (written only when
 * it fits cap). */
int64_t orc_assemble(const orc_mesh *g, int nq, const double *qp, const double *qw, int64_t cap, int64_t *rows,
                     int64_t *cols, double *mvals, double *avals)
{
    int d = g->dim;
    int nb = g->order == 1 ? d + 1 : (d + 1) * (d + 2) / 2;
    int64_t nsimp = orc_micro_simplices(g, NULL, 0);
    int64_t total = (int64_t)g->nm * nsimp * nb * nb;
    if (!rows || total > cap) return total;
    int32_t *V = malloc(sizeof(int32_t) * 12 * nsimp);
    orc_micro_simplices(g, V, nsimp);
    int64_t t = 0;
    for (int M = 0; M < g->nm; ++M)
        for (int64_t s = 0; s < nsimp; ++s) {
            int32_t (*vv)[3] = (int32_t (*)[3])(V + s * 12);
            int64_t nodes[10];
            int c = 0;
            if (g->order == 1) {
                for (int x = 0; x <= d; ++x) nodes[c++] = lat_idx(d, vv[x][0], vv[x][1], d == 3 ? vv[x][2] : 0);
            } else {
                for (int x = 0; x <= d; ++x)
                    nodes[c++] = lat_idx(d, 2 * vv[x][0], 2 * vv[x][1], d == 3 ? 2 * vv[x][2] : 0);
                for (int x = 0; x <= d; ++x)
                    for (int y = x + 1; y <= d; ++y)
                        nodes[c++] = lat_idx(d, vv[x][0] + vv[y][0], vv[x][1] + vv[y][1],
                                             d == 3 ? vv[x][2] + vv[y][2] : 0);
            }
            double p[4][3], E[9];
            for (int a = 0; a <= d; ++a) nlat_pos(g, M, vv[a], p[a]);
            for (int i = 0; i < d; ++i)
                for (int a = 0; a < d; ++a) E[i * d + a] = p[a + 1][i] - p[0][i];
            double me[100] = {0}, ae[100] = {0};
            for (int q = 0; q < nq; ++q) {
                const double *xi = qp + (size_t)q * d;
                double x[3], D[9], J[9] = {0}, Ji[9], phi[10], dphi[10][3], gp[10][3];
                for (int i = 0; i < d; ++i) {
                    x[i] = p[0][i];
                    for (int a = 0; a < d; ++a) x[i] += xi[a] * E[i * d + a];
                }
                phi_jacobian(g, M, x, D);
                for (int i = 0; i < d; ++i)
                    for (int j = 0; j < d; ++j) {
                        double acc = 0;
                        for (int k = 0; k < d; ++k) acc += D[i * d + k] * E[k * d + j];
                        J[i * d + j] = acc;
                    }
                double wdet = qw[q] * fabs(det_inv(d, J, Ji));
                shape_fn(d, g->order, xi, phi, dphi);
                /* physical gradient: grad phi = J^-T grad_xi phi */
                for (int b = 0; b < nb; ++b)
                    for (int i = 0; i < d; ++i) {
                        double acc = 0;
                        for (int k = 0; k < d; ++k) acc += Ji[k * d + i] * dphi[b][k];
                        gp[b][i] = acc;
                    }
                for (int i = 0; i < nb; ++i)
                    for (int j = 0; j < nb; ++j) {
                        double dot = 0;
                        for (int k = 0; k < d; ++k) dot += gp[i][k] * gp[j][k];
                        me[i * nb + j] += wdet * phi[i] * phi[j];
                        ae[i * nb + j] += wdet * dot;
                    }
            }
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j, ++t) {
                    rows[t] = g->uid[(size_t)M * g->npm + nodes[i]];
                    cols[t] = g->uid[(size_t)M * g->npm + nodes[j]];
                    mvals[t] = me[i * nb + j];
                    avals[t] = ae[i * nb + j];
                }
        }
    free(V);
    return t;
}

/* mask[u] = 1 for DoFs on the domain boundary: lattice nodes of a macro face
 * that has no neighbouring macro (barycentric weight of the opposite vertex
 * zero); 0 elsewhere. */
void orc_boundary_mask(const orc_mesh *g, uint8_t *mask)
{
    int d = g->dim, m = g->m;
    memset(mask, 0, (size_t)g->N);
    for (int M = 0; M < g->nm; ++M)
        for (int I = 0; I <= m; ++I)
            for (int J = 0; J <= I; ++J)
                for (int K = 0; K <= (d == 3 ? J : 0); ++K) {
                    int w[4];
                    lat_weights(d, m, I, J, K, w);
                    for (int k = 0; k <= d; ++k)
                        if (w[k] == 0 && g->nbr[M * (d + 1) + k] < 0)
                            mask[g->uid[(size_t)M * g->npm + lat_idx(d, I, J, K)]] = 1;
                }
}
