/*
 * oracle.c -- plain FP64 CPU oracle (see oracle.h for conventions).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * benchmark's CPU-baseline leg; never by the GPU library.
 *
 * Paper passages followed (arXiv:2310.07607):
 *   Sec. 2, monodomain model (E1) with D = kappa/(chi C_m), I = I'/C_m;
 *   Sec. 2.1, DG primal form + SIPG numerical flux, Gauss-Legendre nodal
 *            basis with GL quadrature (diagonal mass, pointwise ionic term);
 *   Sec. 2.2, Kelly-type face-jump indicator and refine/coarsen thresholds
 *            (Algorithm 1's inequalities);
 *   Sec. 2.3, forward Euler for phi, exponential (Rush-Larsen type) step for
 *            the gate, Gershgorin CFL per element block, substeps 2^b,
 *            synchronous LTS (Algorithm 1: elements of level l updated at
 *            every 2^(lmax-l)-th substep, linear time interpolation of
 *            coarser neighbours).
 * Where the paper is silent or garbled, the reading taken is stated next to
 * the code it affects.
 *
 * The ionic model is the two-variable Aliev-Panfilov model (the workloads'
 * model; the paper's PCG model is not specified in the paper).
 *
 * Compile with -O2 -ffp-contract=off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define MAXM 4          /* up to p = 3 */
#define MAXNP 64        /* MAXM^3 */
#define MAXSTIM 16

typedef struct onode {
    int depth;
    int64_t c[3];              /* cell index in the level-`depth` grid */
    struct onode *kid[8];      /* all NULL for a leaf */
    int64_t leaf;              /* canonical index, -1 if refined */
    double *tu, *tv;           /* transfer scratch during or_adapt */
} onode;

typedef struct {
    int64_t nbr;               /* neighbour leaf */
    int k, s;                  /* face normal dim, side (0 lower, 1 upper) */
    double xk;                 /* face coordinate */
    double lo[3], h[3];        /* tangential extent of the segment */
} oseg;

struct or_sim {
    int dim, p, m, np, nfp, nkids;
    int n[3];
    double len[3];
    int max_depth;
    double xi[MAXM], w[MAXM];
    onode **roots;
    int64_t n_roots;
    onode **leaf;
    int64_t n_leaves;
    double D[3][3], gamma;
    double apk, apa, eps0, mu1, mu2;
    int n_stim;
    double stim[MAXSTIM][9];
    int assembled;
    double *Kee, *Mii;         /* [E][np][np], [E][np] */
    int64_t *seg_start;        /* [E+1] */
    oseg *seg;
    int64_t n_seg;
    double *Ken;               /* [n_seg][np][np] */
    double *u, *v;             /* [E][np] */
};

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1] by Newton iteration on P_m            */
/* ------------------------------------------------------------------ */
static void legendre(int m, double z, double *pm, double *dpm)
{
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= m; k++) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pm = p1;
    *dpm = m * (z * p1 - p0) / (z * z - 1.0);
}

static void gauss_legendre(int m, double *x, double *w)
{
    for (int i = 0; i < m; i++) {
        double z = cos(M_PI * (i + 0.75) / (m + 0.5));
        double pm, dpm;
        for (int it = 0; it < 100; it++) {
            legendre(m, z, &pm, &dpm);
            double dz = pm / dpm;
            z -= dz;
            if (fabs(dz) < 1e-17) break;
        }
        legendre(m, z, &pm, &dpm);
        x[m - 1 - i] = z;
        w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dpm * dpm);
    }
}

/* 1-D Lagrange basis through the GL nodes: values and d/dxi */
static void lagrange_1d(const or_sim *S, double xi, double *l, double *dl)
{
    for (int b = 0; b < S->m; b++) {
        double val = 1.0, der = 0.0;
        for (int c = 0; c < S->m; c++) {
            if (c == b) continue;
            double den = S->xi[b] - S->xi[c];
            double f = (xi - S->xi[c]) / den;
            der = der * f + val / den;
            val *= f;
        }
        l[b] = val;
        dl[b] = der;
    }
}

static int node_index_1d(const or_sim *S, int j, int k)
{
    for (int q = 0; q < k; q++) j /= S->m;
    return j % S->m;
}

static void leaf_box(const or_sim *S, const onode *nd, double *lo, double *h)
{
    for (int k = 0; k < 3; k++) { lo[k] = 0.0; h[k] = 1.0; }
    for (int k = 0; k < S->dim; k++) {
        h[k] = S->len[k] / ((double)S->n[k] * ldexp(1.0, nd->depth));
        lo[k] = (double)nd->c[k] * h[k];
    }
}

/* physical coordinates of node j of element nd */
static void node_xyz(const or_sim *S, const onode *nd, int j, double *X)
{
    double lo[3], h[3];
    leaf_box(S, nd, lo, h);
    for (int k = 0; k < 3; k++) X[k] = 0.0;
    for (int k = 0; k < S->dim; k++) {
        int a = node_index_1d(S, j, k);
        X[k] = lo[k] + 0.5 * (S->xi[a] + 1.0) * h[k];
    }
}

/* tensor-product basis of element nd at physical point X */
static void basis_at(const or_sim *S, const onode *nd, const double *X, double *phi,
                     double (*grad)[3])
{
    double lo[3], h[3], l[3][MAXM], dl[3][MAXM];
    leaf_box(S, nd, lo, h);
    for (int k = 0; k < S->dim; k++)
        lagrange_1d(S, 2.0 * (X[k] - lo[k]) / h[k] - 1.0, l[k], dl[k]);
    for (int j = 0; j < S->np; j++) {
        int jk[3];
        for (int k = 0; k < S->dim; k++) jk[k] = node_index_1d(S, j, k);
        double val = 1.0;
        for (int k = 0; k < S->dim; k++) val *= l[k][jk[k]];
        phi[j] = val;
        for (int k = 0; k < 3; k++) grad[j][k] = 0.0;
        for (int k = 0; k < S->dim; k++) {
            double g = 2.0 / h[k] * dl[k][jk[k]];
            for (int k2 = 0; k2 < S->dim; k2++)
                if (k2 != k) g *= l[k2][jk[k2]];
            grad[j][k] = g;
        }
    }
}

/* ------------------------------------------------------------------ */
/* forest                                                              */
/* ------------------------------------------------------------------ */
static onode *new_node(int depth, const int64_t *c)
{
    onode *nd = (onode *)calloc(1, sizeof(onode));
    nd->depth = depth;
    for (int k = 0; k < 3; k++) nd->c[k] = c[k];
    nd->leaf = -1;
    return nd;
}

static void free_tree(onode *nd)
{
    if (!nd) return;
    for (int i = 0; i < 8; i++) free_tree(nd->kid[i]);
    free(nd->tu);
    free(nd->tv);
    free(nd);
}

static void refine_node(const or_sim *S, onode *nd)
{
    for (int ci = 0; ci < S->nkids; ci++) {
        int64_t c[3] = {0, 0, 0};
        for (int k = 0; k < S->dim; k++) c[k] = 2 * nd->c[k] + ((ci >> k) & 1);
        nd->kid[ci] = new_node(nd->depth + 1, c);
    }
}

static int is_leaf(const onode *nd) { return nd->kid[0] == NULL; }

static void collect_leaves(onode *nd, onode **out, int64_t *cnt)
{
    if (is_leaf(nd)) {
        if (out) out[*cnt] = nd;
        nd->leaf = *cnt;
        (*cnt)++;
        return;
    }
    nd->leaf = -1;
    for (int ci = 0; ci < 8; ci++)
        if (nd->kid[ci]) collect_leaves(nd->kid[ci], out, cnt);
}

static void enumerate_leaves(or_sim *S)
{
    int64_t cnt = 0;
    for (int64_t r = 0; r < S->n_roots; r++) collect_leaves(S->roots[r], NULL, &cnt);
    free(S->leaf);
    S->leaf = (onode **)malloc(sizeof(onode *) * (size_t)(cnt > 0 ? cnt : 1));
    S->n_leaves = 0;
    for (int64_t r = 0; r < S->n_roots; r++) collect_leaves(S->roots[r], S->leaf, &S->n_leaves);
}

enum { NB_BOUNDARY = 0, NB_SAME = 1, NB_COARSER = 2, NB_FINER = 3, NB_ERROR = -1 };

/* Face neighbours of leaf nd across face (k, s).  For NB_FINER, out[] holds
 * the 2^(d-1) children of the same-size neighbour cell that touch the face,
 * in ascending child index. */
static int face_neighbours(const or_sim *S, const onode *nd, int k, int s, onode **out, int *nout)
{
    int64_t t[3] = {nd->c[0], nd->c[1], nd->c[2]};
    int l = nd->depth;
    t[k] += s ? 1 : -1;
    *nout = 0;
    if (t[k] < 0 || t[k] >= ((int64_t)S->n[k] << l)) return NB_BOUNDARY;
    int64_t rc[3] = {0, 0, 0};
    for (int q = 0; q < S->dim; q++) rc[q] = t[q] >> l;
    int64_t rid = rc[0] + (int64_t)S->n[0] * (rc[1] + (int64_t)S->n[1] * rc[2]);
    onode *cur = S->roots[rid];
    while (!is_leaf(cur) && cur->depth < l) {
        int sh = l - cur->depth - 1, ci = 0;
        for (int q = 0; q < S->dim; q++) ci |= (int)((t[q] >> sh) & 1) << q;
        cur = cur->kid[ci];
    }
    if (is_leaf(cur)) {
        out[0] = cur;
        *nout = 1;
        return cur->depth == l ? NB_SAME : NB_COARSER;
    }
    int want = s ? 0 : 1;
    for (int ci = 0; ci < S->nkids; ci++) {
        if (((ci >> k) & 1) != want) continue;
        if (!is_leaf(cur->kid[ci])) return NB_ERROR; /* 2:1 balance violated */
        out[(*nout)++] = cur->kid[ci];
    }
    return NB_FINER;
}

static int check_balance(const or_sim *S)
{
    onode *nb[4];
    int nn;
    for (int64_t e = 0; e < S->n_leaves; e++)
        for (int k = 0; k < S->dim; k++)
            for (int s = 0; s < 2; s++)
                if (face_neighbours(S, S->leaf[e], k, s, nb, &nn) == NB_ERROR) return OR_EINVAL;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* creation and state                                                  */
/* ------------------------------------------------------------------ */
static void invalidate(or_sim *S)
{
    S->assembled = 0;
    free(S->Kee); free(S->Mii); free(S->seg_start); free(S->seg); free(S->Ken);
    S->Kee = S->Mii = S->Ken = NULL;
    S->seg_start = NULL;
    S->seg = NULL;
    S->n_seg = 0;
}

static void reset_state(or_sim *S)
{
    free(S->u);
    free(S->v);
    size_t N = (size_t)S->n_leaves * S->np;
    S->u = (double *)calloc(N ? N : 1, sizeof(double));
    S->v = (double *)calloc(N ? N : 1, sizeof(double));
}

or_sim *or_create(int dim, int p, const int n[3], const double len[3], int max_depth)
{
    if (dim < 2 || dim > 3 || p < 1 || p >= MAXM || max_depth < 0 || max_depth > 20) return NULL;
    for (int k = 0; k < dim; k++)
        if (n[k] < 1 || !(len[k] > 0.0)) return NULL;
    or_sim *S = (or_sim *)calloc(1, sizeof(or_sim));
    S->dim = dim;
    S->p = p;
    S->m = p + 1;
    S->np = 1;
    S->nfp = 1;
    for (int k = 0; k < dim; k++) S->np *= S->m;
    for (int k = 0; k < dim - 1; k++) S->nfp *= S->m;
    S->nkids = 1 << dim;
    for (int k = 0; k < 3; k++) {
        S->n[k] = k < dim ? n[k] : 1;
        S->len[k] = k < dim ? len[k] : 1.0;
    }
    S->max_depth = max_depth;
    gauss_legendre(S->m, S->xi, S->w);
    S->n_roots = (int64_t)S->n[0] * S->n[1] * S->n[2];
    S->roots = (onode **)malloc(sizeof(onode *) * (size_t)S->n_roots);
    for (int64_t r = 0; r < S->n_roots; r++) {
        int64_t c[3] = {r % S->n[0], (r / S->n[0]) % S->n[1], r / ((int64_t)S->n[0] * S->n[1])};
        S->roots[r] = new_node(0, c);
    }
    enumerate_leaves(S);
    reset_state(S);
    /* defaults: identity diffusion, gamma 1, Aliev-Panfilov constants */
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) S->D[a][b] = a == b ? 1.0 : 0.0;
    S->gamma = 1.0;
    S->apk = 8.0; S->apa = 0.15; S->eps0 = 0.002; S->mu1 = 0.2; S->mu2 = 0.3;
    return S;
}

void or_free(or_sim *S)
{
    if (!S) return;
    invalidate(S);
    for (int64_t r = 0; r < S->n_roots; r++) free_tree(S->roots[r]);
    free(S->roots);
    free(S->leaf);
    free(S->u);
    free(S->v);
    free(S);
}

static int parse_tree(const or_sim *S, onode *nd, const uint8_t *bits, int64_t n_bits, int64_t *pos)
{
    if (*pos >= n_bits) return OR_EINVAL;
    uint8_t b = bits[(*pos)++];
    if (b > 1) return OR_EINVAL;
    if (b == 0) return OR_OK;
    if (nd->depth >= S->max_depth) return OR_EINVAL;
    refine_node(S, nd);
    for (int ci = 0; ci < S->nkids; ci++)
        if (parse_tree(S, nd->kid[ci], bits, n_bits, pos) != OR_OK) return OR_EINVAL;
    return OR_OK;
}

int or_set_tree(or_sim *S, const uint8_t *bits, int64_t n_bits)
{
    for (int64_t r = 0; r < S->n_roots; r++) {
        for (int ci = 0; ci < 8; ci++) {
            free_tree(S->roots[r]->kid[ci]);
            S->roots[r]->kid[ci] = NULL;
        }
    }
    int64_t pos = 0;
    int rc = OR_OK;
    for (int64_t r = 0; r < S->n_roots && rc == OR_OK; r++) rc = parse_tree(S, S->roots[r], bits, n_bits, &pos);
    if (rc == OR_OK && pos != n_bits) rc = OR_EINVAL;
    if (rc != OR_OK) {
        for (int64_t r = 0; r < S->n_roots; r++)
            for (int ci = 0; ci < 8; ci++) {
                free_tree(S->roots[r]->kid[ci]);
                S->roots[r]->kid[ci] = NULL;
            }
    }
    invalidate(S);
    enumerate_leaves(S);
    reset_state(S);
    if (rc == OR_OK) rc = check_balance(S);
    return rc;
}

static void write_bits(const onode *nd, uint8_t *out, int64_t cap, int64_t *pos)
{
    if (*pos < cap && out) out[*pos] = is_leaf(nd) ? 0 : 1;
    (*pos)++;
    if (!is_leaf(nd))
        for (int ci = 0; ci < 8; ci++)
            if (nd->kid[ci]) write_bits(nd->kid[ci], out, cap, pos);
}

int64_t or_tree_bits(const or_sim *S, uint8_t *out, int64_t cap)
{
    int64_t pos = 0;
    for (int64_t r = 0; r < S->n_roots; r++) write_bits(S->roots[r], out, cap, &pos);
    return pos;
}

int64_t or_n_leaves(const or_sim *S) { return S->n_leaves; }
int or_n_dof_per_leaf(const or_sim *S) { return S->np; }

void or_leaf_info(const or_sim *S, int32_t *depth, int64_t *coords)
{
    for (int64_t e = 0; e < S->n_leaves; e++) {
        if (depth) depth[e] = S->leaf[e]->depth;
        if (coords)
            for (int k = 0; k < 3; k++) coords[3 * e + k] = S->leaf[e]->c[k];
    }
}

int or_leaf_nodes(const or_sim *S, double *xyz)
{
    for (int64_t e = 0; e < S->n_leaves; e++)
        for (int j = 0; j < S->np; j++) node_xyz(S, S->leaf[e], j, &xyz[3 * (e * S->np + j)]);
    return OR_OK;
}

int or_set_params(or_sim *S, const double D[9], double gamma, const double ap[5])
{
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            if (D[3 * a + b] != D[3 * b + a]) return OR_EINVAL;
            S->D[a][b] = D[3 * a + b];
        }
    if (!(gamma >= 0.0)) return OR_EINVAL;
    S->gamma = gamma;
    if (ap) {
        S->apk = ap[0]; S->apa = ap[1]; S->eps0 = ap[2]; S->mu1 = ap[3]; S->mu2 = ap[4];
    }
    invalidate(S);
    return OR_OK;
}

int or_set_stimulus(or_sim *S, const double *boxes, int n)
{
    if (n < 0 || n > MAXSTIM) return OR_EINVAL;
    S->n_stim = n;
    for (int i = 0; i < n; i++)
        for (int q = 0; q < 9; q++) S->stim[i][q] = boxes[9 * i + q];
    return OR_OK;
}

int or_set_state(or_sim *S, const double *u, const double *v)
{
    size_t N = (size_t)S->n_leaves * S->np;
    if (u) memcpy(S->u, u, N * sizeof(double));
    if (v) memcpy(S->v, v, N * sizeof(double));
    return OR_OK;
}

int or_get_state(const or_sim *S, double *u, double *v)
{
    size_t N = (size_t)S->n_leaves * S->np;
    if (u) memcpy(u, S->u, N * sizeof(double));
    if (v) memcpy(v, S->v, N * sizeof(double));
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* assembly of element and face blocks (Sec. 2.1)                      */
/* ------------------------------------------------------------------ */

/* Collect the face segments of leaf e.  A segment is the common part of a
 * face of e and a face of one neighbour, i.e. the smaller of the two faces. */
static int leaf_segments(const or_sim *S, int64_t e, oseg *out, int *nout)
{
    const onode *nd = S->leaf[e];
    double lo[3], h[3];
    leaf_box(S, nd, lo, h);
    *nout = 0;
    for (int k = 0; k < S->dim; k++) {
        for (int s = 0; s < 2; s++) {
            onode *nb[4];
            int nn;
            int kind = face_neighbours(S, nd, k, s, nb, &nn);
            if (kind == NB_ERROR) return OR_EINVAL;
            if (kind == NB_BOUNDARY) continue;
            for (int q = 0; q < nn; q++) {
                oseg sg;
                memset(&sg, 0, sizeof(sg));
                sg.nbr = nb[q]->leaf;
                sg.k = k;
                sg.s = s;
                sg.xk = s ? lo[k] + h[k] : lo[k];
                const onode *small = (kind == NB_FINER) ? nb[q] : nd;
                double slo[3], sh[3];
                leaf_box(S, small, slo, sh);
                for (int t = 0; t < 3; t++) { sg.lo[t] = slo[t]; sg.h[t] = sh[t]; }
                out[(*nout)++] = sg;
            }
        }
    }
    return OR_OK;
}

/* tangential GL point g on a segment: physical point and weight */
static void seg_point(const or_sim *S, const oseg *sg, int g, double *X, double *W)
{
    int gi = g;
    *W = 1.0;
    for (int t = 0; t < 3; t++) X[t] = 0.0;
    for (int t = 0; t < S->dim; t++) {
        if (t == sg->k) {
            X[t] = sg->xk;
            continue;
        }
        int a = gi % S->m;
        gi /= S->m;
        X[t] = sg->lo[t] + 0.5 * (S->xi[a] + 1.0) * sg->h[t];
        *W *= S->w[a] * 0.5 * sg->h[t];
    }
}

/* n . D grad(phi) for the outward normal of side s in direction k */
static double normal_flux(const or_sim *S, int k, int s, const double *g)
{
    double f = 0.0;
    for (int a = 0; a < S->dim; a++) f += S->D[k][a] * g[a];
    return s ? f : -f;
}

int or_assemble(or_sim *S)
{
    if (S->assembled) return OR_OK;
    invalidate(S);
    int64_t E = S->n_leaves;
    int np = S->np;
    S->Kee = (double *)calloc((size_t)E * np * np + 1, sizeof(double));
    S->Mii = (double *)calloc((size_t)E * np + 1, sizeof(double));
    S->seg_start = (int64_t *)calloc((size_t)E + 1, sizeof(int64_t));
    int maxseg = 2 * S->dim * (1 << (S->dim - 1));
    oseg *tmp = (oseg *)malloc(sizeof(oseg) * maxseg);
    for (int64_t e = 0; e < E; e++) {
        int ns;
        if (leaf_segments(S, e, tmp, &ns) != OR_OK) { free(tmp); return OR_EINVAL; }
        S->seg_start[e + 1] = S->seg_start[e] + ns;
    }
    S->n_seg = S->seg_start[E];
    S->seg = (oseg *)malloc(sizeof(oseg) * (size_t)(S->n_seg + 1));
    S->Ken = (double *)calloc((size_t)S->n_seg * np * np + 1, sizeof(double));

    double phi[MAXNP], grad[MAXNP][3], phin[MAXNP], gradn[MAXNP][3];
    for (int64_t e = 0; e < E; e++) {
        const onode *nd = S->leaf[e];
        double lo[3], h[3];
        leaf_box(S, nd, lo, h);
        double *K = &S->Kee[(size_t)e * np * np];
        /* volume: -int D grad(phi_j) . grad(phi_i), GL rule at the nodes */
        for (int q = 0; q < np; q++) {
            double X[3], Wq = 1.0;
            node_xyz(S, nd, q, X);
            for (int k = 0; k < S->dim; k++) Wq *= S->w[node_index_1d(S, q, k)] * 0.5 * h[k];
            basis_at(S, nd, X, phi, grad);
            for (int i = 0; i < np; i++) {
                S->Mii[(size_t)e * np + i] += Wq * phi[i] * phi[i];
                for (int j = 0; j < np; j++) {
                    double a = 0.0;
                    for (int x = 0; x < S->dim; x++)
                        for (int y = 0; y < S->dim; y++) a += grad[i][x] * S->D[x][y] * grad[j][y];
                    K[i * np + j] -= Wq * a;
                }
            }
        }
        /* interior faces: SIPG terms (reading: standard SIPG signs, so -K >= 0) */
        int ns;
        leaf_segments(S, e, tmp, &ns);
        for (int q = 0; q < ns; q++) {
            oseg *sg = &S->seg[S->seg_start[e] + q];
            *sg = tmp[q];
            const onode *nb = S->leaf[sg->nbr];
            double nlo[3], nh[3];
            leaf_box(S, nb, nlo, nh);
            double Dkk = S->D[sg->k][sg->k];
            double sigma = S->gamma * 0.5 * (Dkk / h[sg->k] + Dkk / nh[sg->k]);
            double *Kn = &S->Ken[(size_t)(S->seg_start[e] + q) * np * np];
            for (int g = 0; g < S->nfp; g++) {
                double X[3], Wg;
                seg_point(S, sg, g, X, &Wg);
                basis_at(S, nd, X, phi, grad);
                basis_at(S, nb, X, phin, gradn);
                for (int i = 0; i < np; i++) {
                    double dni = normal_flux(S, sg->k, sg->s, grad[i]);
                    for (int j = 0; j < np; j++) {
                        double dnj = normal_flux(S, sg->k, sg->s, grad[j]);
                        double dnnj = normal_flux(S, sg->k, sg->s, gradn[j]);
                        K[i * np + j] += Wg * (0.5 * dnj * phi[i] + 0.5 * phi[j] * dni - sigma * phi[j] * phi[i]);
                        Kn[i * np + j] += Wg * (0.5 * dnnj * phi[i] - 0.5 * phin[j] * dni + sigma * phin[j] * phi[i]);
                    }
                }
            }
        }
    }
    free(tmp);
    S->assembled = 1;
    return OR_OK;
}

int or_dense_operators(or_sim *S, double *K, double *Mfull)
{
    if (or_assemble(S) != OR_OK) return OR_EINVAL;
    int64_t E = S->n_leaves;
    int np = S->np;
    int64_t N = E * np;
    if (K) {
        memset(K, 0, sizeof(double) * (size_t)N * N);
        for (int64_t e = 0; e < E; e++) {
            for (int i = 0; i < np; i++)
                for (int j = 0; j < np; j++)
                    K[(e * np + i) * N + e * np + j] += S->Kee[(size_t)e * np * np + i * np + j];
            for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++) {
                int64_t nb = S->seg[q].nbr;
                for (int i = 0; i < np; i++)
                    for (int j = 0; j < np; j++)
                        K[(e * np + i) * N + nb * np + j] += S->Ken[(size_t)q * np * np + i * np + j];
            }
        }
    }
    if (Mfull) {
        /* the full mass matrix by quadrature, to show that it is diagonal */
        double phi[MAXNP], grad[MAXNP][3];
        memset(Mfull, 0, sizeof(double) * (size_t)N * N);
        for (int64_t e = 0; e < E; e++) {
            const onode *nd = S->leaf[e];
            double lo[3], h[3];
            leaf_box(S, nd, lo, h);
            for (int q = 0; q < np; q++) {
                double X[3], Wq = 1.0;
                node_xyz(S, nd, q, X);
                for (int k = 0; k < S->dim; k++) Wq *= S->w[node_index_1d(S, q, k)] * 0.5 * h[k];
                basis_at(S, nd, X, phi, grad);
                for (int i = 0; i < np; i++)
                    for (int j = 0; j < np; j++) Mfull[(e * np + i) * N + e * np + j] += Wq * phi[i] * phi[j];
            }
        }
    }
    return OR_OK;
}

/* K applied element by element: (K u)_e = K_ee u_e + sum_segments K_en u_n */
static void element_Ku(const or_sim *S, int64_t e, const double *ue, double *const *un_seg, double *Ku)
{
    int np = S->np;
    const double *K = &S->Kee[(size_t)e * np * np];
    for (int i = 0; i < np; i++) {
        double a = 0.0;
        for (int j = 0; j < np; j++) a += K[i * np + j] * ue[j];
        Ku[i] = a;
    }
    for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++) {
        const double *Kn = &S->Ken[(size_t)q * np * np];
        const double *un = un_seg[q - S->seg_start[e]];
        for (int i = 0; i < np; i++) {
            double a = 0.0;
            for (int j = 0; j < np; j++) a += Kn[i * np + j] * un[j];
            Ku[i] += a;
        }
    }
}

int or_apply_K(or_sim *S, const double *u, double *Ku)
{
    if (or_assemble(S) != OR_OK) return OR_EINVAL;
    double *un_seg[32];
    for (int64_t e = 0; e < S->n_leaves; e++) {
        for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++)
            un_seg[q - S->seg_start[e]] = (double *)&u[S->seg[q].nbr * S->np];
        element_Ku(S, e, &u[e * S->np], un_seg, &Ku[e * S->np]);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* ionic model and pointwise update (Sec. 2.3)                          */
/* ------------------------------------------------------------------ */
static double stimulus_at(const or_sim *S, const double *X, double t)
{
    double s = 0.0;
    for (int b = 0; b < S->n_stim; b++) {
        const double *B = S->stim[b];
        if (!(t >= B[6] && t < B[7])) continue;
        int inside = 1;
        for (int k = 0; k < S->dim; k++)
            if (X[k] < B[k] || X[k] > B[3 + k]) inside = 0;
        if (inside) s += B[8];
    }
    return s;
}

/* Aliev-Panfilov: du/dt gets f(u,v) = -k u (u-a)(u-1) - u v;
 * dv/dt = eps(u,v) (v_inf - v) with v_inf = k u (1 + a - u),
 * eps = eps0 + mu1 v / (u + mu2), the denominator floored at 1e-6.
 * Forward Euler for u, exponential step for v with eps frozen at the
 * start-of-step state (the partitioned Rush-Larsen analogue). */
static void point_update(const or_sim *S, double u, double v, double lap, double stim, double dt,
                         double *un, double *vn)
{
    double f = -S->apk * u * (u - S->apa) * (u - 1.0) - u * v;
    double den = u + S->mu2;
    if (den < 1e-6) den = 1e-6;
    double eps = S->eps0 + S->mu1 * v / den;
    double vinf = S->apk * u * (1.0 + S->apa - u);
    *un = u + dt * (lap + f + stim);
    *vn = vinf + (v - vinf) * exp(-eps * dt);
}

/* new u, v of element e from its own start values ue and neighbour values */
static void element_update(const or_sim *S, int64_t e, const double *ue, const double *ve,
                           double *const *un_seg, double t, double dt, double *u_out, double *v_out)
{
    double Ku[MAXNP];
    element_Ku(S, e, ue, un_seg, Ku);
    for (int i = 0; i < S->np; i++) {
        double X[3];
        node_xyz(S, S->leaf[e], i, X);
        double lap = Ku[i] / S->Mii[(size_t)e * S->np + i];
        point_update(S, ue[i], ve[i], lap, stimulus_at(S, X, t), dt, &u_out[i], &v_out[i]);
    }
}

int or_element_update(or_sim *S, int64_t e, const double *u_at_t, double t, double dt, double *u_new,
                      double *v_new)
{
    if (or_assemble(S) != OR_OK || e < 0 || e >= S->n_leaves) return OR_EINVAL;
    double *un_seg[32];
    for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++)
        un_seg[q - S->seg_start[e]] = (double *)&u_at_t[S->seg[q].nbr * S->np];
    element_update(S, e, &u_at_t[e * S->np], &S->v[e * S->np], un_seg, t, dt, u_new, v_new);
    return OR_OK;
}

/* plain global forward Euler: t_n = t0 + n dt */
int or_step_global(or_sim *S, double dt, double t0, int64_t n_steps)
{
    if (or_assemble(S) != OR_OK) return OR_EINVAL;
    int np = S->np;
    size_t N = (size_t)S->n_leaves * np;
    double *u1 = (double *)malloc(sizeof(double) * (N + 1));
    double *v1 = (double *)malloc(sizeof(double) * (N + 1));
    double *un_seg[32];
    for (int64_t n = 0; n < n_steps; n++) {
        double t = t0 + (double)n * dt;
        for (int64_t e = 0; e < S->n_leaves; e++) {
            for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++)
                un_seg[q - S->seg_start[e]] = &S->u[S->seg[q].nbr * np];
            element_update(S, e, &S->u[e * np], &S->v[e * np], un_seg, t, dt, &u1[e * np], &v1[e * np]);
        }
        memcpy(S->u, u1, sizeof(double) * N);
        memcpy(S->v, v1, sizeof(double) * N);
    }
    free(u1);
    free(v1);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* CFL and substep levels (Sec. 2.3)                                   */
/* ------------------------------------------------------------------ */

/* Gershgorin bound on L_e = M_e^{-1} K_e, K_e the element's own block with
 * the neighbours frozen.  Reading: the disc radius plus |L_ii| (L_ii < 0),
 * i.e. CFL_e = 1 / max_i sum_j |L_ij|. */
int or_cfl(or_sim *S, double *cfl)
{
    if (or_assemble(S) != OR_OK) return OR_EINVAL;
    int np = S->np;
    for (int64_t e = 0; e < S->n_leaves; e++) {
        double worst = 0.0;
        for (int i = 0; i < np; i++) {
            double r = 0.0;
            for (int j = 0; j < np; j++) r += fabs(S->Kee[(size_t)e * np * np + i * np + j] / S->Mii[(size_t)e * np + i]);
            if (r > worst) worst = r;
        }
        cfl[e] = 1.0 / worst;
    }
    return OR_OK;
}

/* b_e = the smallest b >= 0 with dt_barrier 2^-b <= CFL_e (exact scaling,
 * a tie counts as satisfied); EUNSTABLE if some b_e exceeds n_levels-1. */
int or_levels(or_sim *S, double dt_barrier, int n_levels, int8_t *level)
{
    double *cfl = (double *)malloc(sizeof(double) * (size_t)(S->n_leaves + 1));
    if (or_cfl(S, cfl) != OR_OK) { free(cfl); return OR_EINVAL; }
    int rc = OR_OK;
    for (int64_t e = 0; e < S->n_leaves; e++) {
        int b = 0;
        while (b < 100 && ldexp(dt_barrier, -b) > cfl[e]) b++;
        if (b > n_levels - 1) rc = OR_EUNSTABLE;
        level[e] = (int8_t)(b > 127 ? 127 : b);
    }
    free(cfl);
    return rc;
}

/* ------------------------------------------------------------------ */
/* RV-T temporal indicator and the b^cell substeps (Sec. 2.3)           */
/* ------------------------------------------------------------------ */
/* The indicator of element e over a barrier [t_a, t_b] (Sec. 2.3, Ratti-
 * Veroni temporal indicator): the L2 norms over [t_a, t_b] x e of the
 * changes of the ionic current I and of the gating right-hand side g since
 * t_a, each divided by t_b - t_a, combined as a root sum of squares.
 * Readings: the time integrals use the midpoint rule (as the paper states)
 * at the state linear in time between the barrier's end values (the S-LTS
 * representation of a coarse element between its updates); I(u, v, t) is
 * the whole non-diffusive right-hand side of du/dt, f(u, v) + s(x, t); the
 * L2(e) norm uses the element's own quadrature (the diagonal mass).  So
 *   eta^2 = [ |I(m, t_m) - I(a, t_a)|^2 + |g(m) - g(a)|^2 ]_{L2(e)} / (t_b - t_a).
 * The state at t_b is the oracle's current state. */
static double ap_current(const or_sim *S, double u, double v)
{
    return -S->apk * u * (u - S->apa) * (u - 1.0) - u * v;
}

static double ap_gate_rate(const or_sim *S, double u, double v)
{
    double den = u + S->mu2;
    if (den < 1e-6) den = 1e-6;
    const double eps = S->eps0 + S->mu1 * v / den;
    const double vinf = S->apk * u * (1.0 + S->apa - u);
    return eps * (vinf - v);
}

int or_rvt_indicator(or_sim *S, const double *u_a, const double *v_a, double t_a, double t_b, double *eta_t)
{
    if (or_assemble(S) != OR_OK || !(t_b > t_a)) return OR_EINVAL;
    const double span = t_b - t_a, t_m = 0.5 * (t_a + t_b);
    const int np = S->np;
    for (int64_t e = 0; e < S->n_leaves; e++) {
        double sum = 0.0;
        for (int i = 0; i < np; i++) {
            const size_t q = (size_t)e * np + i;
            double X[3];
            node_xyz(S, S->leaf[e], i, X);
            const double um = 0.5 * (u_a[q] + S->u[q]), vm = 0.5 * (v_a[q] + S->v[q]);
            const double dI = (ap_current(S, um, vm) + stimulus_at(S, X, t_m)) -
                              (ap_current(S, u_a[q], v_a[q]) + stimulus_at(S, X, t_a));
            const double dg = ap_gate_rate(S, um, vm) - ap_gate_rate(S, u_a[q], v_a[q]);
            sum += S->Mii[q] * (dI * dI + dg * dg);
        }
        eta_t[e] = sqrt(sum / span);
    }
    return OR_OK;
}

/* Levels with both criteria of Sec. 2.3: b_e = max(b^CFL_e, b^cell_e), with
 * b^cell_e = ceil(log2(dt_barrier / dt_cell)) where eta_t[e] > tau_cell and
 * 0 elsewhere.  The ceiling is taken as the smallest b >= 0 with
 * dt_barrier 2^-b <= dt_cell (exact scaling, as for b^CFL). */
int or_levels_cell(or_sim *S, double dt_barrier, int n_levels, const double *eta_t, double tau_cell,
                   double dt_cell, int8_t *level)
{
    if (!(dt_cell > 0.0)) return OR_EINVAL;
    int rc = or_levels(S, dt_barrier, n_levels, level);
    if (rc != OR_OK && rc != OR_EUNSTABLE) return rc;
    int b_cell = 0;
    while (b_cell < 100 && ldexp(dt_barrier, -b_cell) > dt_cell) b_cell++;
    for (int64_t e = 0; e < S->n_leaves; e++) {
        int b = level[e];
        if (eta_t[e] > tau_cell && b_cell > b) b = b_cell;
        if (b > n_levels - 1) rc = OR_EUNSTABLE;
        level[e] = (int8_t)(b > 127 ? 127 : b);
    }
    return rc;
}

/* stable grouping by level, finest first (ties in canonical order) */
void or_bucket(int64_t E, const int8_t *level, int n_levels, int32_t *perm, int32_t *cnt_ge)
{
    int64_t pos = 0;
    for (int l = n_levels - 1; l >= 0; l--) {
        for (int64_t e = 0; e < E; e++)
            if (level[e] == l) perm[pos++] = (int32_t)e;
        cnt_ge[l] = (int32_t)pos;
    }
}

/* ------------------------------------------------------------------ */
/* one barrier interval of synchronous LTS (Algorithm 1)               */
/* ------------------------------------------------------------------ */
static void trace_row(double *trace, int64_t cap, int64_t *len, double a, double b, double c, double d)
{
    if (trace && *len < cap) {
        trace[4 * *len + 0] = a;
        trace[4 * *len + 1] = b;
        trace[4 * *len + 2] = c;
        trace[4 * *len + 3] = d;
    }
    (*len)++;
}

int or_lts_barrier(or_sim *S, double dt_barrier, double t_n, const int8_t *level, int mode,
                   double *trace, int64_t trace_cap, int64_t *trace_len, int64_t *n_updates)
{
    if (or_assemble(S) != OR_OK) return OR_EINVAL;
    int64_t E = S->n_leaves;
    int np = S->np;
    int lmax = 0;
    for (int64_t e = 0; e < E; e++) {
        if (level[e] < 0 || level[e] > 30) return OR_EINVAL;
        if (level[e] > lmax) lmax = level[e];
    }
    int64_t maxS = (int64_t)1 << lmax;
    double h_tick = dt_barrier / (double)maxS;
    int64_t tl = 0, nupd = 0;
    double *nbuf = (double *)malloc(sizeof(double) * 32 * MAXNP);
    double *un_seg[32];
    double unew[MAXNP], vnew[MAXNP];

    if (mode == 0) {
        /* Time-history form, from the definitions of Sec. 2.3: an element
         * of level l takes S = 2^l steps of dt/S, i.e. it is updated at the
         * ticks that are multiples of k = maxS/S, and its value is known at
         * those ticks and at maxS.  hist[e] holds the values of element e at
         * ticks 0, k_e, 2 k_e, ..., maxS.  At tick i a neighbour's value is
         * its known value at i if i is one of its ticks; otherwise the
         * neighbour is coarser and its value at t_i is linear in time
         * between its known values at the ticks enclosing i (both already
         * computed: the later one at the earlier tick).  Nothing written at
         * tick i is read at tick i, so the order inside a tick is free. */
        int64_t *hoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(E + 1));
        hoff[0] = 0;
        for (int64_t e = 0; e < E; e++) hoff[e + 1] = hoff[e] + (((int64_t)1 << level[e]) + 1) * np;
        double *hist = (double *)malloc(sizeof(double) * (size_t)(hoff[E] + 1));
        for (int64_t e = 0; e < E; e++) memcpy(&hist[hoff[e]], &S->u[e * np], sizeof(double) * np);
        for (int64_t i = 0; i < maxS; i++) {
            for (int64_t e = 0; e < E; e++) {
                int64_t ke = maxS >> level[e];
                if (i % ke != 0) continue;
                for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++) {
                    int64_t nb = S->seg[q].nbr;
                    int64_t kn = maxS >> level[nb];
                    int64_t m0 = i / kn;
                    const double *h0 = &hist[hoff[nb] + m0 * np];
                    double *dst = &nbuf[(q - S->seg_start[e]) * MAXNP];
                    double theta = (double)(i - m0 * kn) / (double)kn;
                    if (i == m0 * kn) {
                        memcpy(dst, h0, sizeof(double) * np);
                    } else {
                        const double *h1 = h0 + np;
                        for (int j = 0; j < np; j++) dst[j] = (1.0 - theta) * h0[j] + theta * h1[j];
                    }
                    un_seg[q - S->seg_start[e]] = dst;
                    trace_row(trace, trace_cap, &tl, (double)i, (double)e, (double)nb, theta);
                }
                double dt_e = ldexp(dt_barrier, -level[e]);
                double t_i = t_n + (double)i * h_tick;
                double *he = &hist[hoff[e] + (i / ke) * np];
                element_update(S, e, he, &S->v[e * np], un_seg, t_i, dt_e, unew, vnew);
                memcpy(he + np, unew, sizeof(double) * np);
                memcpy(&S->v[e * np], vnew, sizeof(double) * np);
                nupd++;
            }
        }
        for (int64_t e = 0; e < E; e++)
            memcpy(&S->u[e * np], &hist[hoff[e] + ((int64_t)1 << level[e]) * np], sizeof(double) * np);
        free(hist);
        free(hoff);
    } else {
        /* two-slot level-bucket form: slot[e] holds the element's value at
         * its last update tick, other[e] its value one step later.  At
         * substep i the active set is {e : level_e >= lmin(i)}; an inactive
         * neighbour is coarser and is interpolated with theta = (i mod k)/k. */
        double *slot0 = (double *)malloc(sizeof(double) * (size_t)(E * np + 1));
        double *slot1 = (double *)malloc(sizeof(double) * (size_t)(E * np + 1));
        int *cur = (int *)calloc((size_t)E + 1, sizeof(int));
        memcpy(slot0, S->u, sizeof(double) * (size_t)E * np);
        memcpy(slot1, S->u, sizeof(double) * (size_t)E * np);
        for (int64_t i = 0; i < maxS; i++) {
            int v2 = 0;
            while (i > 0 && ((i >> v2) & 1) == 0) v2++;
            int lmin = i == 0 ? 0 : lmax - v2;
            for (int64_t e = 0; e < E; e++) {
                if (level[e] < lmin) continue;
                for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++) {
                    int64_t nb = S->seg[q].nbr;
                    double *dst = &nbuf[(q - S->seg_start[e]) * MAXNP];
                    int64_t kn = maxS >> level[nb];
                    double theta = (double)(i % kn) / (double)kn;
                    double *a = (cur[nb] ? slot1 : slot0) + nb * np;
                    double *b = (cur[nb] ? slot0 : slot1) + nb * np;
                    if (level[nb] >= lmin) {
                        memcpy(dst, a, sizeof(double) * np);
                    } else {
                        /* inactive: `a` is its value now being the newer one */
                        double *older = b, *newer = a;
                        for (int j = 0; j < np; j++) dst[j] = (1.0 - theta) * older[j] + theta * newer[j];
                    }
                    un_seg[q - S->seg_start[e]] = dst;
                    trace_row(trace, trace_cap, &tl, (double)i, (double)e, (double)nb, theta);
                }
                double *ue = (cur[e] ? slot1 : slot0) + e * np;
                double *uo = (cur[e] ? slot0 : slot1) + e * np;
                double dt_e = ldexp(dt_barrier, -level[e]);
                double t_i = t_n + (double)i * h_tick;
                element_update(S, e, ue, &S->v[e * np], un_seg, t_i, dt_e, unew, vnew);
                memcpy(uo, unew, sizeof(double) * np);
                memcpy(&S->v[e * np], vnew, sizeof(double) * np);
                nupd++;
            }
            /* flip after the whole sweep so that reads above saw pre-sweep slots */
            for (int64_t e = 0; e < E; e++)
                if (level[e] >= lmin) cur[e] ^= 1;
        }
        for (int64_t e = 0; e < E; e++)
            memcpy(&S->u[e * np], (cur[e] ? slot1 : slot0) + e * np, sizeof(double) * np);
        free(slot0); free(slot1); free(cur);
    }
    free(nbuf);
    if (trace_len) *trace_len = tl;
    if (n_updates) *n_updates = nupd;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Kelly-type indicator (Sec. 2.2)                                     */
/* ------------------------------------------------------------------ */
/* eta_e^2 = sum over interior face pieces F of e of
 *     h_F/(2p) * W_F^2 * int_F [[D grad(u) . n]]^2 dS
 * Readings: a piece is the common part of a face of e and one neighbour
 * face; |F| its measure, h_F = |F|^(1/(d-1)), W_F = |F| (the Jacobian of
 * the map from the reference face [0,1]^(d-1)); boundary faces are skipped. */
int or_indicator(or_sim *S, double *eta)
{
    if (or_assemble(S) != OR_OK) return OR_EINVAL;
    int np = S->np;
    double phi[MAXNP], grad[MAXNP][3], phin[MAXNP], gradn[MAXNP][3];
    for (int64_t e = 0; e < S->n_leaves; e++) {
        const onode *nd = S->leaf[e];
        double acc = 0.0;
        for (int64_t q = S->seg_start[e]; q < S->seg_start[e + 1]; q++) {
            const oseg *sg = &S->seg[q];
            const onode *nb = S->leaf[sg->nbr];
            double area = 1.0;
            for (int t = 0; t < S->dim; t++)
                if (t != sg->k) area *= sg->h[t];
            double hF = S->dim == 2 ? area : sqrt(area);
            double WF = area;
            double integral = 0.0;
            for (int g = 0; g < S->nfp; g++) {
                double X[3], Wg;
                seg_point(S, sg, g, X, &Wg);
                basis_at(S, nd, X, phi, grad);
                basis_at(S, nb, X, phin, gradn);
                double gm[3] = {0, 0, 0}, gp[3] = {0, 0, 0};
                for (int j = 0; j < np; j++)
                    for (int a = 0; a < S->dim; a++) {
                        gm[a] += grad[j][a] * S->u[e * np + j];
                        gp[a] += gradn[j][a] * S->u[sg->nbr * np + j];
                    }
                double jump = normal_flux(S, sg->k, sg->s, gm) - normal_flux(S, sg->k, sg->s, gp);
                integral += Wg * jump * jump;
            }
            acc += hF / (2.0 * S->p) * WF * WF * integral;
        }
        eta[e] = sqrt(acc);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* adaptivity (Algorithm 1: refine eta >= tau_r, coarsen eta <= tau_c)  */
/* ------------------------------------------------------------------ */
static void prolong_to_child(const or_sim *S, const onode *parent, const double *up, const onode *child,
                             double *uc)
{
    double phi[MAXNP], grad[MAXNP][3];
    for (int i = 0; i < S->np; i++) {
        double X[3];
        node_xyz(S, child, i, X);
        basis_at(S, parent, X, phi, grad);
        double a = 0.0;
        for (int j = 0; j < S->np; j++) a += phi[j] * up[j];
        uc[i] = a;
    }
}

/* L2 projection of the children's fields onto the parent space, with each
 * child's own GL rule (exact for the degree-2p integrands) */
static void restrict_to_parent(const or_sim *S, const onode *parent, double *const *uc, double *up)
{
    double phi[MAXNP], grad[MAXNP][3];
    double rhs[MAXNP], mass[MAXNP];
    for (int i = 0; i < S->np; i++) { rhs[i] = 0.0; mass[i] = 0.0; }
    for (int ci = 0; ci < S->nkids; ci++) {
        const onode *ch = parent->kid[ci];
        double lo[3], h[3];
        leaf_box(S, ch, lo, h);
        for (int q = 0; q < S->np; q++) {
            double X[3], Wq = 1.0;
            node_xyz(S, ch, q, X);
            for (int k = 0; k < S->dim; k++) Wq *= S->w[node_index_1d(S, q, k)] * 0.5 * h[k];
            basis_at(S, parent, X, phi, grad);
            for (int i = 0; i < S->np; i++) {
                rhs[i] += Wq * uc[ci][q] * phi[i];
                mass[i] += Wq * phi[i] * phi[i];
            }
        }
    }
    for (int i = 0; i < S->np; i++) up[i] = rhs[i] / mass[i];
}

static int collect_coarsenable(or_sim *S, onode *nd, const double *eta, double tau_c, const uint8_t *refine,
                               onode **list, int64_t *cnt)
{
    if (is_leaf(nd)) return 0;
    int all_leaves = 1;
    for (int ci = 0; ci < S->nkids; ci++)
        if (!is_leaf(nd->kid[ci])) all_leaves = 0;
    if (!all_leaves) {
        for (int ci = 0; ci < S->nkids; ci++) collect_coarsenable(S, nd->kid[ci], eta, tau_c, refine, list, cnt);
        return 0;
    }
    for (int ci = 0; ci < S->nkids; ci++) {
        const onode *ch = nd->kid[ci];
        if (!(eta[ch->leaf] <= tau_c) || refine[ch->leaf]) return 0;
    }
    /* keep 2:1 balance after this round's refinement: no leaf outside the
     * parent that touches a child may end up deeper than the child */
    for (int ci = 0; ci < S->nkids; ci++) {
        const onode *ch = nd->kid[ci];
        for (int k = 0; k < S->dim; k++)
            for (int s = 0; s < 2; s++) {
                int64_t t = ch->c[k] + (s ? 1 : -1);
                if ((t >> 1) == nd->c[k]) continue; /* sibling inside the parent */
                onode *nb[4];
                int nn;
                int kind = face_neighbours(S, ch, k, s, nb, &nn);
                if (kind == NB_BOUNDARY || kind == NB_COARSER) continue;
                if (kind == NB_FINER || kind == NB_ERROR) return 0;
                if (refine[nb[0]->leaf]) return 0; /* same depth, being refined */
            }
    }
    list[(*cnt)++] = nd;
    return 1;
}

int or_adapt(or_sim *S, const double *eta, double tau_refine, double tau_coarsen, int64_t *n_refined,
             int64_t *n_coarsened)
{
    int64_t E = S->n_leaves;
    int np = S->np;
    uint8_t *refine = (uint8_t *)calloc((size_t)E + 1, 1);
    for (int64_t e = 0; e < E; e++)
        refine[e] = (eta[e] >= tau_refine && S->leaf[e]->depth < S->max_depth) ? 1 : 0;
    /* 2:1 closure: a leaf being refined forces every coarser face neighbour
     * to be refined as well; iterate to the (unique) least fixed point */
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int64_t e = 0; e < E; e++) {
            if (!refine[e]) continue;
            for (int k = 0; k < S->dim; k++)
                for (int s = 0; s < 2; s++) {
                    onode *nb[4];
                    int nn;
                    int kind = face_neighbours(S, S->leaf[e], k, s, nb, &nn);
                    if (kind == NB_COARSER && !refine[nb[0]->leaf]) {
                        refine[nb[0]->leaf] = 1;
                        changed = 1;
                    }
                }
        }
    }
    onode **clist = (onode **)malloc(sizeof(onode *) * (size_t)(E + 1));
    int64_t nc = 0;
    for (int64_t r = 0; r < S->n_roots; r++) collect_coarsenable(S, S->roots[r], eta, tau_coarsen, refine, clist, &nc);

    /* carry old values on the nodes, then change the tree */
    for (int64_t e = 0; e < E; e++) {
        onode *nd = S->leaf[e];
        nd->tu = (double *)malloc(sizeof(double) * np);
        nd->tv = (double *)malloc(sizeof(double) * np);
        memcpy(nd->tu, &S->u[e * np], sizeof(double) * np);
        memcpy(nd->tv, &S->v[e * np], sizeof(double) * np);
    }
    int64_t nr = 0;
    for (int64_t e = 0; e < E; e++) {
        if (!refine[e]) continue;
        onode *nd = S->leaf[e];
        refine_node(S, nd);
        for (int ci = 0; ci < S->nkids; ci++) {
            onode *ch = nd->kid[ci];
            ch->tu = (double *)malloc(sizeof(double) * np);
            ch->tv = (double *)malloc(sizeof(double) * np);
            prolong_to_child(S, nd, nd->tu, ch, ch->tu);
            prolong_to_child(S, nd, nd->tv, ch, ch->tv);
        }
        free(nd->tu); free(nd->tv);
        nd->tu = nd->tv = NULL;
        nr++;
    }
    for (int64_t c = 0; c < nc; c++) {
        onode *P = clist[c];
        double *cu[8], *cv[8];
        for (int ci = 0; ci < S->nkids; ci++) { cu[ci] = P->kid[ci]->tu; cv[ci] = P->kid[ci]->tv; }
        P->tu = (double *)malloc(sizeof(double) * np);
        P->tv = (double *)malloc(sizeof(double) * np);
        restrict_to_parent(S, P, cu, P->tu);
        restrict_to_parent(S, P, cv, P->tv);
        for (int ci = 0; ci < S->nkids; ci++) {
            free_tree(P->kid[ci]);
            P->kid[ci] = NULL;
        }
    }
    invalidate(S);
    enumerate_leaves(S);
    reset_state(S);
    for (int64_t e = 0; e < S->n_leaves; e++) {
        onode *nd = S->leaf[e];
        memcpy(&S->u[e * np], nd->tu, sizeof(double) * np);
        memcpy(&S->v[e * np], nd->tv, sizeof(double) * np);
        free(nd->tu); free(nd->tv);
        nd->tu = nd->tv = NULL;
    }
    free(refine);
    free(clist);
    if (n_refined) *n_refined = nr;
    if (n_coarsened) *n_coarsened = nc;
    return check_balance(S);
}

/* ------------------------------------------------------------------ */
/* point evaluation (for activation times)                             */
/* ------------------------------------------------------------------ */
/* A point on an internal element boundary is taken from the element on its
 * upper side (the half-open convention lo <= x < hi). */
int or_eval_points(or_sim *S, const double *xyz, int64_t n_pts, double *out)
{
    double phi[MAXNP], grad[MAXNP][3];
    for (int64_t p = 0; p < n_pts; p++) {
        const double *X = &xyz[3 * p];
        int64_t rc[3] = {0, 0, 0};
        double f[3] = {0, 0, 0};
        for (int k = 0; k < S->dim; k++) {
            double r = X[k] / S->len[k] * S->n[k];
            if (r < 0.0 || r > S->n[k]) return OR_EINVAL;
            rc[k] = (int64_t)floor(r);
            if (rc[k] >= S->n[k]) rc[k] = S->n[k] - 1;
            f[k] = r - (double)rc[k];
        }
        onode *cur = S->roots[rc[0] + (int64_t)S->n[0] * (rc[1] + (int64_t)S->n[1] * rc[2])];
        while (!is_leaf(cur)) {
            int ci = 0;
            for (int k = 0; k < S->dim; k++) {
                double scaled = f[k] * ldexp(1.0, cur->depth + 1);
                int64_t cell = (int64_t)floor(scaled);
                if (cell > (2 * (cur->c[k] - (rc[k] << cur->depth)) + 1))
                    cell = 2 * (cur->c[k] - (rc[k] << cur->depth)) + 1;
                ci |= (int)(cell & 1) << k;
            }
            cur = cur->kid[ci];
        }
        basis_at(S, cur, X, phi, grad);
        double a = 0.0;
        for (int j = 0; j < S->np; j++) a += phi[j] * S->u[cur->leaf * S->np + j];
        out[p] = a;
    }
    return OR_OK;
}
