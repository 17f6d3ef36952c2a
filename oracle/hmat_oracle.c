/*
 * hmat_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 reference for the mixed-precision
 * H-matrix-vector product of Ooi, Iwashita, Fukaya, Ida and Yokota,
 * "Effect of Mixed Precision Computing on H-Matrix Vector Multiplication in
 * BEM Analysis" (arXiv:1911.00093), and for the BiCGSTAB loop that repeats
 * it.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library; the product path never does, and this
 * file shares no code with the GPU library.
 *
 * Every routine follows the definition it cites, in natural loop order, with
 * no blocking or reordering.  Where the paper is silent (the BEM entries, the
 * cluster tree, the admissibility rule, the ACA variant) the reading used is
 * stated at the routine.
 *
 * Index convention: the cluster tree fixes a permutation perm[k] = original
 * panel index of position k; every block refers to contiguous ranges of
 * permuted positions (Sec. 2 writes each block by its first and last index),
 * and all vectors handed to the matvec and the solver are in permuted order.
 *
 * Block data layout (FP64): a dense block is stored column-major, #I x #J;
 * a low-rank block stores V_m (#I x r, column-major) followed by the
 * transpose of W_m (#J x r, column-major), so that A|^m ~ V_m W_m (Eq. 3).
 *
 * Parity pins live in tests/test_oracle_*.py.  The BF16-scaled variant and
 * the learned-preconditioner pieces are not from the paper; they are
 * checked against the definitions stated at each routine.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_PI 3.14159265358979323846

typedef struct {
    int64_t lo, hi;    /* permuted positions [lo, hi) */
    int64_t child[2];  /* -1 for a leaf */
    double bmin[3], bmax[3];
} ora_node;

typedef struct {
    int64_t row0, nrows, col0, ncols;
    int32_t kind; /* 0 dense, 1 low rank */
    int32_t rank;
    int64_t off;
} ora_block;

typedef struct {
    int64_t n;
    int64_t *perm;
    double *cent; /* permuted order, n x 3 */
    double *area; /* permuted order */
    int64_t nnodes, cap_nodes;
    ora_node *nodes;
    int64_t nblocks, cap_blocks;
    ora_block *blocks;
    int64_t ndata, cap_data;
    double *data;
    int64_t leaf;
    double eta, eps;
} ora_hmat;

/* ------------------------------------------------------------------------- */
/* BEM entries.  The paper gives no discretisation (Sec. 4.1.2 only names an
 * electrostatic surface-charge analysis with triangular elements).  Reading:
 * piecewise-constant charge density per flat panel, collocation at the
 * centroids, free-space kernel 1/(4 pi |x - y|) with a one-point centroid
 * rule off the diagonal, and for the self term the potential at the centre
 * of a disc of equal area: the integral of 1/(4 pi r) over a disc of radius
 * R is R/2, with R = sqrt(a/pi). */
double ora_entry(const ora_hmat *h, int64_t i, int64_t j)
{
    if (i == j)
        return 0.5 * sqrt(h->area[i] / ORA_PI);
    double dx = h->cent[3 * i + 0] - h->cent[3 * j + 0];
    double dy = h->cent[3 * i + 1] - h->cent[3 * j + 1];
    double dz = h->cent[3 * i + 2] - h->cent[3 * j + 2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    return h->area[j] / (4.0 * ORA_PI * r);
}

/* ------------------------------------------------------------------------- */
/* Cluster tree.  Reading: recursive bisection of the axis-aligned box of the
 * panel centroids across its longest side (ties: x before y before z) at the
 * midpoint; centroids strictly below the midpoint go left, the rest right,
 * both keeping their relative order; if one side would be empty the list is
 * cut in halves instead.  A cluster with at most `leaf` panels is a leaf.
 * The permutation lists the leaves depth-first, left child first. */
static int64_t ora_new_node(ora_hmat *h)
{
    if (h->nnodes == h->cap_nodes) {
        h->cap_nodes = h->cap_nodes ? 2 * h->cap_nodes : 64;
        h->nodes = (ora_node *)realloc(h->nodes, (size_t)h->cap_nodes * sizeof(ora_node));
    }
    return h->nnodes++;
}

static void ora_bbox(const double *cent_orig, const int64_t *idx, int64_t m, double *bmin, double *bmax)
{
    for (int d = 0; d < 3; d++) {
        bmin[d] = INFINITY;
        bmax[d] = -INFINITY;
    }
    for (int64_t k = 0; k < m; k++)
        for (int d = 0; d < 3; d++) {
            double v = cent_orig[3 * idx[k] + d];
            if (v < bmin[d]) bmin[d] = v;
            if (v > bmax[d]) bmax[d] = v;
        }
}

/* idx: original panel indices of this cluster, in current order.
 * pos: next free permuted position.  Returns the node id. */
static int64_t ora_split(ora_hmat *h, const double *cent_orig, int64_t *idx, int64_t m,
                         int64_t *pos, int64_t *scratch)
{
    int64_t id = ora_new_node(h);
    double bmin[3], bmax[3];
    ora_bbox(cent_orig, idx, m, bmin, bmax);
    for (int d = 0; d < 3; d++) {
        h->nodes[id].bmin[d] = bmin[d];
        h->nodes[id].bmax[d] = bmax[d];
    }
    h->nodes[id].child[0] = h->nodes[id].child[1] = -1;
    h->nodes[id].lo = *pos;
    if (m <= h->leaf) {
        for (int64_t k = 0; k < m; k++)
            h->perm[*pos + k] = idx[k];
        *pos += m;
        h->nodes[id].hi = *pos;
        return id;
    }
    int axis = 0;
    double ext = bmax[0] - bmin[0];
    for (int d = 1; d < 3; d++)
        if (bmax[d] - bmin[d] > ext) {
            ext = bmax[d] - bmin[d];
            axis = d;
        }
    double mid = 0.5 * (bmin[axis] + bmax[axis]);
    int64_t nl = 0, nr = 0;
    for (int64_t k = 0; k < m; k++)
        if (cent_orig[3 * idx[k] + axis] < mid) nl++;
    if (nl == 0 || nl == m) {
        nl = m / 2;
    } else {
        /* stable partition through the scratch buffer */
        int64_t a = 0;
        for (int64_t k = 0; k < m; k++)
            if (cent_orig[3 * idx[k] + axis] < mid) scratch[a++] = idx[k];
        for (int64_t k = 0; k < m; k++)
            if (!(cent_orig[3 * idx[k] + axis] < mid)) scratch[a++] = idx[k];
        memcpy(idx, scratch, (size_t)m * sizeof(int64_t));
    }
    nr = m - nl;
    int64_t l = ora_split(h, cent_orig, idx, nl, pos, scratch);
    int64_t r = ora_split(h, cent_orig, idx + nl, nr, pos, scratch);
    h->nodes[id].child[0] = l;
    h->nodes[id].child[1] = r;
    h->nodes[id].hi = *pos;
    return id;
}

/* ------------------------------------------------------------------------- */
/* Admissibility.  Reading: diam = length of the diagonal of the centroid box,
 * dist = Euclidean distance between the two boxes (0 if they touch or
 * overlap); a pair is admissible when dist > 0 and
 * min(diam(tau), diam(sigma)) <= eta * dist. */
static double ora_diam(const ora_node *a)
{
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = a->bmax[d] - a->bmin[d];
        s += e * e;
    }
    return sqrt(s);
}

static double ora_dist(const ora_node *a, const ora_node *b)
{
    double s = 0.0;
    for (int d = 0; d < 3; d++) {
        double g = 0.0;
        if (b->bmin[d] > a->bmax[d]) g = b->bmin[d] - a->bmax[d];
        else if (a->bmin[d] > b->bmax[d]) g = a->bmin[d] - b->bmax[d];
        s += g * g;
    }
    return sqrt(s);
}

int ora_admissible(const ora_hmat *h, int64_t t, int64_t s)
{
    const ora_node *a = &h->nodes[t], *b = &h->nodes[s];
    double dist = ora_dist(a, b);
    if (!(dist > 0.0)) return 0;
    double da = ora_diam(a), db = ora_diam(b);
    double dm = da < db ? da : db;
    return dm <= h->eta * dist;
}

static void ora_push_block(ora_hmat *h, int64_t t, int64_t s, int kind)
{
    if (h->nblocks == h->cap_blocks) {
        h->cap_blocks = h->cap_blocks ? 2 * h->cap_blocks : 256;
        h->blocks = (ora_block *)realloc(h->blocks, (size_t)h->cap_blocks * sizeof(ora_block));
    }
    ora_block *b = &h->blocks[h->nblocks++];
    b->row0 = h->nodes[t].lo;
    b->nrows = h->nodes[t].hi - h->nodes[t].lo;
    b->col0 = h->nodes[s].lo;
    b->ncols = h->nodes[s].hi - h->nodes[s].lo;
    b->kind = kind;
    b->rank = 0;
    b->off = -1;
}

/* Block partition M (Eqs. 1-2): starting from (root, root), an admissible
 * pair becomes a low-rank candidate, a pair of leaves a dense block; when
 * only one side is a leaf the other side is refined, otherwise all four
 * child pairs are visited.  Blocks are listed depth-first. */
static void ora_block_rec(ora_hmat *h, int64_t t, int64_t s)
{
    const ora_node *a = &h->nodes[t], *b = &h->nodes[s];
    if (ora_admissible(h, t, s)) {
        ora_push_block(h, t, s, 1);
        return;
    }
    int la = a->child[0] < 0, lb = b->child[0] < 0;
    if (la && lb) {
        ora_push_block(h, t, s, 0);
        return;
    }
    int64_t ac0 = a->child[0], ac1 = a->child[1], bc0 = b->child[0], bc1 = b->child[1];
    if (la) {
        ora_block_rec(h, t, bc0);
        ora_block_rec(h, t, bc1);
    } else if (lb) {
        ora_block_rec(h, ac0, s);
        ora_block_rec(h, ac1, s);
    } else {
        ora_block_rec(h, ac0, bc0);
        ora_block_rec(h, ac0, bc1);
        ora_block_rec(h, ac1, bc0);
        ora_block_rec(h, ac1, bc1);
    }
}

/* ------------------------------------------------------------------------- */
static double *ora_reserve(ora_hmat *h, int64_t count, int64_t *off)
{
    if (h->ndata + count > h->cap_data) {
        int64_t nc = h->cap_data ? h->cap_data : 1 << 16;
        while (nc < h->ndata + count) nc *= 2;
        h->data = (double *)realloc(h->data, (size_t)nc * sizeof(double));
        h->cap_data = nc;
    }
    *off = h->ndata;
    h->ndata += count;
    return h->data + *off;
}

static void ora_fill_dense(ora_hmat *h, ora_block *b)
{
    int64_t off;
    double *A = ora_reserve(h, b->nrows * b->ncols, &off);
    for (int64_t j = 0; j < b->ncols; j++)
        for (int64_t i = 0; i < b->nrows; i++)
            A[i + j * b->nrows] = ora_entry(h, b->row0 + i, b->col0 + j);
    b->kind = 0;
    b->rank = 0;
    b->off = off;
}

/* Adaptive cross approximation with partial pivoting (the low-rank method the
 * paper names in Sec. 1, ref. [18]; the generation itself is left to the
 * library, Sec. 4.1.3).  Reading:
 *  - the first pivot row is the first row of the block;
 *  - each step takes the residual of the pivot row, its column pivot j* is
 *    the entry of largest magnitude (lowest index on ties); a residual row
 *    that is zero up to 1e-14 of the largest entry seen is skipped in favour
 *    of the lowest unused row;
 *  - v = row / row[j*], u = residual of column j*;
 *  - the squared Frobenius norm of the running approximation S_k is updated
 *    incrementally, and the loop stops once |u| |v| <= eps |S_k|_F or the
 *    rank reaches min(#I, #J);
 *  - the next pivot row is the unused row where |u| is largest;
 *  - if r (#I + #J) >= #I #J the block is stored dense instead. */
static void ora_aca(ora_hmat *h, ora_block *b)
{
    int64_t m = b->nrows, n = b->ncols;
    int64_t kmax = m < n ? m : n;
    double *U = (double *)malloc((size_t)(m * kmax) * sizeof(double));
    double *V = (double *)malloc((size_t)(n * kmax) * sizeof(double));
    double *row = (double *)malloc((size_t)n * sizeof(double));
    double *col = (double *)malloc((size_t)m * sizeof(double));
    char *used = (char *)calloc((size_t)m, 1);
    int64_t k = 0, istar = 0;
    double S2 = 0.0, seen = 0.0;
    while (k < kmax) {
        for (int64_t j = 0; j < n; j++) {
            double a = ora_entry(h, b->row0 + istar, b->col0 + j);
            if (fabs(a) > seen) seen = fabs(a);
            double s = a;
            for (int64_t l = 0; l < k; l++)
                s -= U[istar + l * m] * V[j + l * n];
            row[j] = s;
        }
        used[istar] = 1;
        int64_t jstar = 0;
        for (int64_t j = 1; j < n; j++)
            if (fabs(row[j]) > fabs(row[jstar])) jstar = j;
        if (fabs(row[jstar]) <= 1e-14 * seen) {
            int64_t nxt = -1;
            for (int64_t i = 0; i < m; i++)
                if (!used[i]) {
                    nxt = i;
                    break;
                }
            if (nxt < 0) break;
            istar = nxt;
            continue;
        }
        double piv = row[jstar];
        for (int64_t j = 0; j < n; j++)
            V[j + k * n] = row[j] / piv;
        for (int64_t i = 0; i < m; i++) {
            double a = ora_entry(h, b->row0 + i, b->col0 + jstar);
            if (fabs(a) > seen) seen = fabs(a);
            double s = a;
            for (int64_t l = 0; l < k; l++)
                s -= V[jstar + l * n] * U[i + l * m];
            col[i] = s;
        }
        for (int64_t i = 0; i < m; i++)
            U[i + k * m] = col[i];
        double uu = 0.0, vv = 0.0;
        for (int64_t i = 0; i < m; i++) uu += U[i + k * m] * U[i + k * m];
        for (int64_t j = 0; j < n; j++) vv += V[j + k * n] * V[j + k * n];
        double cross = 0.0;
        for (int64_t l = 0; l < k; l++) {
            double pu = 0.0, pv = 0.0;
            for (int64_t i = 0; i < m; i++) pu += U[i + l * m] * U[i + k * m];
            for (int64_t j = 0; j < n; j++) pv += V[j + l * n] * V[j + k * n];
            cross += pu * pv;
        }
        S2 += 2.0 * cross + uu * vv;
        k++;
        if (sqrt(uu) * sqrt(vv) <= h->eps * sqrt(S2)) break;
        int64_t nxt = -1;
        double best = -1.0;
        for (int64_t i = 0; i < m; i++)
            if (!used[i] && fabs(U[i + (k - 1) * m]) > best) {
                best = fabs(U[i + (k - 1) * m]);
                nxt = i;
            }
        if (nxt < 0) break;
        istar = nxt;
    }
    if (k * (m + n) >= m * n) {
        ora_fill_dense(h, b);
    } else {
        int64_t off;
        double *dst = ora_reserve(h, k * (m + n), &off);
        memcpy(dst, U, (size_t)(m * k) * sizeof(double));
        memcpy(dst + m * k, V, (size_t)(n * k) * sizeof(double));
        b->kind = 1;
        b->rank = (int32_t)k;
        b->off = off;
    }
    free(U);
    free(V);
    free(row);
    free(col);
    free(used);
}

/* Assemble the FP64 H-matrix: cluster tree, block partition, then dense
 * leaves by direct evaluation and admissible blocks by ACA (the paper
 * generates the H-matrix in FP64 first and converts afterwards, Sec. 4.1.3).
 * cent: n x 3 and area: n, in original panel order. */
ora_hmat *ora_assemble(int64_t n, const double *cent, const double *area, int64_t leaf, double eta, double eps)
{
    if (n <= 0 || leaf <= 0) return NULL;
    ora_hmat *h = (ora_hmat *)calloc(1, sizeof(ora_hmat));
    h->n = n;
    h->leaf = leaf;
    h->eta = eta;
    h->eps = eps;
    h->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *idx = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *scratch = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) idx[i] = i;
    int64_t pos = 0;
    ora_split(h, cent, idx, n, &pos, scratch);
    free(idx);
    free(scratch);
    h->cent = (double *)malloc((size_t)(3 * n) * sizeof(double));
    h->area = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; k++) {
        for (int d = 0; d < 3; d++) h->cent[3 * k + d] = cent[3 * h->perm[k] + d];
        h->area[k] = area[h->perm[k]];
    }
    ora_block_rec(h, 0, 0);
    for (int64_t b = 0; b < h->nblocks; b++) {
        if (h->blocks[b].kind == 0) ora_fill_dense(h, &h->blocks[b]);
        else ora_aca(h, &h->blocks[b]);
    }
    return h;
}

/* An H-matrix given directly by its blocks (no geometry): used to check the
 * product and the solver on hand-made matrices.  The permutation is the
 * identity; the arrays are copied. */
ora_hmat *ora_from_blocks(int64_t n, int64_t nblocks, const int64_t *row0, const int64_t *nrows,
                          const int64_t *col0, const int64_t *ncols, const int32_t *kind, const int32_t *rank,
                          const int64_t *off, int64_t ndata, const double *data)
{
    ora_hmat *h = (ora_hmat *)calloc(1, sizeof(ora_hmat));
    h->n = n;
    h->perm = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) h->perm[i] = i;
    h->nblocks = h->cap_blocks = nblocks;
    h->blocks = (ora_block *)malloc((size_t)(nblocks > 0 ? nblocks : 1) * sizeof(ora_block));
    for (int64_t b = 0; b < nblocks; b++) {
        h->blocks[b].row0 = row0[b];
        h->blocks[b].nrows = nrows[b];
        h->blocks[b].col0 = col0[b];
        h->blocks[b].ncols = ncols[b];
        h->blocks[b].kind = kind[b];
        h->blocks[b].rank = kind[b] ? rank[b] : 0;
        h->blocks[b].off = off[b];
    }
    h->ndata = h->cap_data = ndata;
    h->data = (double *)malloc((size_t)(ndata > 0 ? ndata : 1) * sizeof(double));
    if (ndata > 0) memcpy(h->data, data, (size_t)ndata * sizeof(double));
    return h;
}

void ora_free(ora_hmat *h)
{
    if (!h) return;
    free(h->perm);
    free(h->cent);
    free(h->area);
    free(h->nodes);
    free(h->blocks);
    free(h->data);
    free(h);
}

/* accessors for the ctypes wrapper */
int64_t ora_n(const ora_hmat *h) { return h->n; }
int64_t ora_nblocks(const ora_hmat *h) { return h->nblocks; }
int64_t ora_ndata(const ora_hmat *h) { return h->ndata; }
int64_t ora_nnodes(const ora_hmat *h) { return h->nnodes; }
const int64_t *ora_perm(const ora_hmat *h) { return h->perm; }
const double *ora_data(const ora_hmat *h) { return h->data; }
void ora_get_blocks(const ora_hmat *h, int64_t *row0, int64_t *nrows, int64_t *col0, int64_t *ncols,
                    int32_t *kind, int32_t *rank, int64_t *off)
{
    for (int64_t b = 0; b < h->nblocks; b++) {
        row0[b] = h->blocks[b].row0;
        nrows[b] = h->blocks[b].nrows;
        col0[b] = h->blocks[b].col0;
        ncols[b] = h->blocks[b].ncols;
        kind[b] = h->blocks[b].kind;
        rank[b] = h->blocks[b].rank;
        off[b] = h->blocks[b].off;
    }
}
void ora_get_nodes(const ora_hmat *h, int64_t *lo, int64_t *hi, int64_t *child, double *bbox)
{
    for (int64_t k = 0; k < h->nnodes; k++) {
        lo[k] = h->nodes[k].lo;
        hi[k] = h->nodes[k].hi;
        child[2 * k] = h->nodes[k].child[0];
        child[2 * k + 1] = h->nodes[k].child[1];
        for (int d = 0; d < 3; d++) {
            bbox[6 * k + d] = h->nodes[k].bmin[d];
            bbox[6 * k + 3 + d] = h->nodes[k].bmax[d];
        }
    }
}

/* Exact dense entries (permuted order) for brute-force checks. */
void ora_dense_rows(const ora_hmat *h, int64_t r0, int64_t nr, double *out /* nr x n, row-major */)
{
    for (int64_t i = 0; i < nr; i++)
        for (int64_t j = 0; j < h->n; j++)
            out[i * h->n + j] = ora_entry(h, r0 + i, j);
}

/* Exact y = A x with every entry evaluated on the fly (O(N^2)). */
void ora_exact_matvec(const ora_hmat *h, const double *x, double *y)
{
    for (int64_t i = 0; i < h->n; i++) {
        double s = 0.0;
        for (int64_t j = 0; j < h->n; j++) s += ora_entry(h, i, j) * x[j];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------- */
/* Precision variants (Sec. 3, Table 1).
 *   0 M1-Double  1 M1-Single  2 M1-Mixed   (Sec. 3.1)
 *   3 M2-Double  4 M2-Single  5 M2-Mixed   (Sec. 3.2, Eqs. 11-16)
 *   6 M3 with split constant c             (Sec. 3.3, Eqs. 17-20)
 *   7 BF16-scaled low-rank factors, FP32 dense (not in the paper: per-block
 *     power-of-two scale, factors rounded to bfloat16, FP64 z). */
enum { V_M1D = 0, V_M1S, V_M1M, V_M2D, V_M2S, V_M2M, V_M3, V_BF16 };

typedef struct {
    int variant, c;
    int64_t n, nblocks;
    const ora_hmat *h;
    int dense32;    /* dense leaves stored in FP32 */
    int x32;        /* source vector rounded to FP32 before the product */
    int z32;        /* z_m kept in FP32 */
    double *data;   /* converted stored values, same layout as h->data */
    int64_t *toff;  /* per block: offset into dterm/tprec (ranks), -1 dense */
    int32_t *trank; /* per block: number of stored rank terms after conversion */
    double *dterm;  /* per stored term: D_m diagonal (1 for Method 1) */
    int8_t *tprec;  /* per stored term: 64, 32 or 16 (bf16) storage */
    int64_t *toff_data; /* per block: offset of converted V (#I x r) then W^T (#J x r) */
} ora_conv;

static double ora_rnd32(double v) { return (double)(float)v; }

/* Round a double to the nearest bfloat16 value (8 significant bits), ties
 * to even, subnormals on the bfloat16 grid. */
double ora_rnd_bf16(double v)
{
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    (void)frexp(v, &e); /* |v| = f 2^e, f in [0.5, 1) */
    if (e < -125) e = -125;
    double q = ldexp(1.0, e - 8);
    return nearbyint(v / q) * q;
}

/* smallest power of two >= m (m > 0) */
static double ora_pow2_ceil(double m)
{
    int e;
    double f = frexp(m, &e);
    return f == 0.5 ? ldexp(1.0, e - 1) : ldexp(1.0, e);
}

/* drop (Methods 2 and 3): 0, or omit the terms with d_i < d_max 10^-drop,
 * the deletion of much smaller terms that Sec. 4.5 proposes.
 * dense_split (Method 3 only): Method 3's split applied to the dense leaves
 * as well, the other proposal of Sec. 4.5: column j of a dense block, whose
 * entries all multiply x_j as the entries of a low-rank term all scale one
 * z entry, is stored in FP32 when its largest magnitude is below
 * (largest magnitude in the block) 10^-c, in FP64 otherwise (ties FP64, as
 * in Eq. 20). */
ora_conv *ora_convert_opts(const ora_hmat *h, int variant, int c, int drop, int dense_split)
{
    if (variant < 0 || variant > 7) return NULL;
    if (drop < 0 || (drop > 0 && !(variant == V_M2D || variant == V_M2S || variant == V_M2M || variant == V_M3)))
        return NULL;
    if (dense_split && variant != V_M3) return NULL;
    ora_conv *v = (ora_conv *)calloc(1, sizeof(ora_conv));
    v->variant = variant;
    v->c = c;
    v->h = h;
    v->n = h->n;
    v->nblocks = h->nblocks;
    v->dense32 = (variant == V_M1S || variant == V_M1M || variant == V_M2S || variant == V_M2M || variant == V_BF16);
    v->x32 = (variant == V_M1S || variant == V_M2S);
    v->z32 = (variant == V_M1S || variant == V_M1M);
    v->data = (double *)malloc((size_t)(h->ndata > 0 ? h->ndata : 1) * sizeof(double));
    v->toff = (int64_t *)malloc((size_t)(h->nblocks + 1) * sizeof(int64_t));
    v->trank = (int32_t *)calloc((size_t)(h->nblocks + 1), sizeof(int32_t));
    v->toff_data = (int64_t *)malloc((size_t)(h->nblocks + 1) * sizeof(int64_t));
    int64_t nterms = 0;
    for (int64_t b = 0; b < h->nblocks; b++)
        if (h->blocks[b].kind == 1) nterms += h->blocks[b].rank;
    v->dterm = (double *)malloc((size_t)(nterms + 1) * sizeof(double));
    v->tprec = (int8_t *)malloc((size_t)(nterms + 1));
    int64_t tpos = 0, dpos = 0;
    for (int64_t bi = 0; bi < h->nblocks; bi++) {
        const ora_block *b = &h->blocks[bi];
        const double *src = h->data + b->off;
        if (b->kind == 0) {
            int64_t cnt = b->nrows * b->ncols;
            if (dense_split) {
                double bmax = 0.0;
                for (int64_t e = 0; e < cnt; e++) if (fabs(src[e]) > bmax) bmax = fabs(src[e]);
                double thr = bmax * pow(10.0, -(double)c);
                for (int64_t j = 0; j < b->ncols; j++) {
                    const double *col = src + j * b->nrows;
                    double cmax = 0.0;
                    for (int64_t i = 0; i < b->nrows; i++) if (fabs(col[i]) > cmax) cmax = fabs(col[i]);
                    for (int64_t i = 0; i < b->nrows; i++)
                        v->data[dpos + j * b->nrows + i] = cmax < thr ? ora_rnd32(col[i]) : col[i];
                }
            } else {
                for (int64_t e = 0; e < cnt; e++)
                    v->data[dpos + e] = v->dense32 ? ora_rnd32(src[e]) : src[e];
            }
            v->toff[bi] = -1;
            v->toff_data[bi] = dpos;
            dpos += cnt;
            continue;
        }
        int64_t m = b->nrows, n = b->ncols, r = b->rank;
        const double *U = src, *Wt = src + m * r;
        double *dU = v->data + dpos, *dW = v->data + dpos + m * r;
        v->toff[bi] = tpos;
        v->toff_data[bi] = dpos;
        if (variant <= V_M1M) {
            /* Method 1: the original factors, cast to the storage type */
            for (int64_t e = 0; e < m * r; e++) dU[e] = variant == V_M1D ? U[e] : ora_rnd32(U[e]);
            for (int64_t e = 0; e < n * r; e++) dW[e] = variant == V_M1D ? Wt[e] : ora_rnd32(Wt[e]);
            for (int64_t l = 0; l < r; l++) {
                v->dterm[tpos + l] = 1.0;
                v->tprec[tpos + l] = variant == V_M1D ? 64 : 32;
            }
            v->trank[bi] = (int32_t)r;
        } else if (variant == V_BF16) {
            double mu = 0.0, mw = 0.0;
            for (int64_t e = 0; e < m * r; e++) if (fabs(U[e]) > mu) mu = fabs(U[e]);
            for (int64_t e = 0; e < n * r; e++) if (fabs(Wt[e]) > mw) mw = fabs(Wt[e]);
            double sv = mu > 0 ? ora_pow2_ceil(mu) : 1.0, sw = mw > 0 ? ora_pow2_ceil(mw) : 1.0;
            /* stored (decoded) values: s * bf16(value / s) */
            for (int64_t e = 0; e < m * r; e++) dU[e] = sv * ora_rnd_bf16(U[e] / sv);
            for (int64_t e = 0; e < n * r; e++) dW[e] = sw * ora_rnd_bf16(Wt[e] / sw);
            for (int64_t l = 0; l < r; l++) {
                v->dterm[tpos + l] = 1.0;
                v->tprec[tpos + l] = 16;
            }
            v->trank[bi] = (int32_t)r;
        } else {
            /* Method 2 scaling (Eqs. 13-16): D_V = column max of |V|,
             * D_W = row max of |W|, V' = V D_V^{-1}, W' = D_W^{-1} W,
             * D = D_V D_W.  A term whose column or row is entirely zero is
             * dropped (the paper does not cover that case). */
            int64_t kept = 0;
            double dmax = 0.0;
            double *dv = (double *)malloc((size_t)r * sizeof(double));
            double *dw = (double *)malloc((size_t)r * sizeof(double));
            for (int64_t l = 0; l < r; l++) {
                double a = 0.0, w = 0.0;
                for (int64_t i = 0; i < m; i++) if (fabs(U[i + l * m]) > a) a = fabs(U[i + l * m]);
                for (int64_t j = 0; j < n; j++) if (fabs(Wt[j + l * n]) > w) w = fabs(Wt[j + l * n]);
                dv[l] = a;
                dw[l] = w;
                if (a * w > dmax) dmax = a * w;
            }
            /* Method 3 split (Eqs. 17-20): a term is FP32 when
             * d_i < d_max 10^-c, FP64 otherwise; FP64 terms are stored first
             * (the paper notes the terms may be reordered freely). */
            double thr = dmax * pow(10.0, -(double)c);
            double cut = drop > 0 ? dmax * pow(10.0, -(double)drop) : 0.0;
            for (int pass = 0; pass < 2; pass++) {
                for (int64_t l = 0; l < r; l++) {
                    if (!(dv[l] > 0.0 && dw[l] > 0.0)) continue;
                    double d = dv[l] * dw[l];
                    if (d < cut) continue; /* deleted (drop) */
                    int p64;
                    if (variant == V_M2D) p64 = 1;
                    else if (variant == V_M2S || variant == V_M2M) p64 = 0;
                    else p64 = d >= thr;
                    if ((pass == 0) != (p64 == 1)) continue;
                    for (int64_t i = 0; i < m; i++) {
                        double s = U[i + l * m] / dv[l];
                        dU[i + kept * m] = p64 ? s : ora_rnd32(s);
                    }
                    for (int64_t j = 0; j < n; j++) {
                        double s = Wt[j + l * n] / dw[l];
                        /* W' is written after all kept V' columns below */
                        dW[j + kept * n] = p64 ? s : ora_rnd32(s);
                    }
                    v->dterm[tpos + kept] = d;
                    v->tprec[tpos + kept] = p64 ? 64 : 32;
                    kept++;
                }
            }
            /* compact: V' occupies m*kept, W'^T follows immediately */
            if (kept < r) memmove(v->data + dpos + m * kept, dW, (size_t)(n * kept) * sizeof(double));
            v->trank[bi] = (int32_t)kept;
            free(dv);
            free(dw);
        }
        tpos += v->trank[bi];
        dpos += (m + n) * v->trank[bi];
    }
    return v;
}

ora_conv *ora_convert_drop(const ora_hmat *h, int variant, int c, int drop)
{
    return ora_convert_opts(h, variant, c, drop, 0);
}

ora_conv *ora_convert(const ora_hmat *h, int variant, int c) { return ora_convert_opts(h, variant, c, 0, 0); }

void ora_conv_free(ora_conv *v)
{
    if (!v) return;
    free(v->data);
    free(v->toff);
    free(v->trank);
    free(v->dterm);
    free(v->tprec);
    free(v->toff_data);
    free(v);
}

/* converted-structure accessors: per block rank after conversion, term
 * scales and storage precisions, and the converted values */
int32_t ora_conv_rank(const ora_conv *v, int64_t b) { return v->trank[b]; }
int64_t ora_conv_term_off(const ora_conv *v, int64_t b) { return v->toff[b]; }
int64_t ora_conv_data_off(const ora_conv *v, int64_t b) { return v->toff_data[b]; }
const double *ora_conv_dterm(const ora_conv *v) { return v->dterm; }
const int8_t *ora_conv_tprec(const ora_conv *v) { return v->tprec; }
const double *ora_conv_data(const ora_conv *v) { return v->data; }

/* ------------------------------------------------------------------------- */
/* H-matrix-vector product, "build" arithmetic: every stored value has the
 * type Table 1 gives it, the source vector is rounded to FP32 first in the
 * Single variants (Sec. 3.5: an FP32 copy of x is made just before each
 * product), and every product and sum is then carried out in FP64; z_m is
 * rounded once to FP32 where Table 1 stores it in FP32.
 *   dense:    y^_m[i] += A|^m[i][j] x_m[j]                      (Eq. 21)
 *   low rank: z_m[i] += W'_m[i][j] x_m[j]; z_m[i] *= D_m[i][i]  (Eqs. 22-23)
 *             y^_m[i] += V'_m[i][j] z_m[j]                      (Eq. 24)
 *   result:   y~[i] += y^_m[i - i_m^(s) + 1]                    (Eq. 25)
 * Method 3 adds the y^_m of its FP64 part and of its FP32 part. */
void ora_matvec(const ora_conv *v, const double *x, double *y)
{
    const ora_hmat *h = v->h;
    int64_t n = h->n;
    double *xe = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; i++) xe[i] = v->x32 ? ora_rnd32(x[i]) : x[i];
    for (int64_t i = 0; i < n; i++) y[i] = 0.0;
    int64_t maxm = 1, maxr = 1;
    for (int64_t b = 0; b < h->nblocks; b++) {
        if (h->blocks[b].nrows > maxm) maxm = h->blocks[b].nrows;
        if (h->blocks[b].rank > maxr) maxr = h->blocks[b].rank;
    }
    double *yh = (double *)malloc((size_t)maxm * sizeof(double));
    double *yh2 = (double *)malloc((size_t)maxm * sizeof(double));
    double *z = (double *)malloc((size_t)maxr * sizeof(double));
    for (int64_t bi = 0; bi < h->nblocks; bi++) {
        const ora_block *b = &h->blocks[bi];
        int64_t m = b->nrows, nc = b->ncols;
        const double *xm = xe + b->col0;
        const double *d = v->data + v->toff_data[bi];
        if (b->kind == 0) {
            for (int64_t i = 0; i < m; i++) {
                double s = 0.0;
                for (int64_t j = 0; j < nc; j++) s += d[i + j * m] * xm[j];
                yh[i] = s;
            }
        } else {
            int64_t r = v->trank[bi];
            const double *Vp = d, *Wt = d + m * r;
            const double *D = v->dterm + v->toff[bi];
            const int8_t *P = v->tprec + v->toff[bi];
            for (int64_t i = 0; i < m; i++) yh[i] = yh2[i] = 0.0;
            for (int64_t l = 0; l < r; l++) {
                double s = 0.0;
                for (int64_t j = 0; j < nc; j++) s += Wt[j + l * nc] * xm[j];
                s *= D[l];
                z[l] = v->z32 ? ora_rnd32(s) : s;
            }
            /* Method 3: FP64 terms into yh, FP32 terms into yh2, then added */
            for (int64_t i = 0; i < m; i++) {
                double s64 = 0.0, s32 = 0.0;
                for (int64_t l = 0; l < r; l++) {
                    if (v->variant == V_M3 && P[l] == 32) s32 += Vp[i + l * m] * z[l];
                    else s64 += Vp[i + l * m] * z[l];
                }
                yh[i] = s64;
                yh2[i] = s32;
            }
            if (v->variant == V_M3)
                for (int64_t i = 0; i < m; i++) yh[i] = yh[i] + yh2[i];
        }
        for (int64_t i = 0; i < m; i++) y[b->row0 + i] += yh[i];
    }
    free(xe);
    free(yh);
    free(yh2);
    free(z);
}

/* Same product with every operation in the type Table 1 gives its operands
 * ("literal" arithmetic): when two operands differ in precision the lower
 * one is promoted first (Sec. 3.4), so a product of two FP32 values is an
 * FP32 product, and an FP32 z_m accumulates in FP32 (rounded after every
 * update).  Defined for Methods 1-3; BF16 falls back to build arithmetic. */
void ora_matvec_literal(const ora_conv *v, const double *x, double *y)
{
    if (v->variant == V_BF16) {
        ora_matvec(v, x, y);
        return;
    }
    const ora_hmat *h = v->h;
    int64_t n = h->n;
    for (int64_t i = 0; i < n; i++) y[i] = 0.0;
    int64_t maxm = 1, maxr = 1;
    for (int64_t b = 0; b < h->nblocks; b++) {
        if (h->blocks[b].nrows > maxm) maxm = h->blocks[b].nrows;
        if (h->blocks[b].rank > maxr) maxr = h->blocks[b].rank;
    }
    double *yh = (double *)malloc((size_t)maxm * sizeof(double));
    double *z = (double *)malloc((size_t)maxr * sizeof(double));
    float *xf = (float *)malloc((size_t)n * sizeof(float));
    for (int64_t i = 0; i < n; i++) xf[i] = (float)x[i];
    for (int64_t bi = 0; bi < h->nblocks; bi++) {
        const ora_block *b = &h->blocks[bi];
        int64_t m = b->nrows, nc = b->ncols;
        const double *d = v->data + v->toff_data[bi];
        if (b->kind == 0) {
            for (int64_t i = 0; i < m; i++) {
                double s = 0.0; /* y^_m is FP64 in every variant */
                for (int64_t j = 0; j < nc; j++) {
                    if (!v->dense32) s += d[i + j * m] * x[b->col0 + j];
                    else if (v->x32) s += (double)((float)d[i + j * m] * xf[b->col0 + j]);
                    else s += (double)(float)d[i + j * m] * x[b->col0 + j];
                }
                yh[i] = s;
            }
        } else {
            int64_t r = v->trank[bi];
            const double *Vp = d, *Wt = d + m * r;
            const double *D = v->dterm + v->toff[bi];
            const int8_t *P = v->tprec + v->toff[bi];
            for (int64_t l = 0; l < r; l++) {
                int lo = P[l] != 64; /* this term is stored in FP32 */
                if (v->z32) {
                    float zs = 0.0f; /* Method 1 Single/Mixed: z_m in FP32 */
                    for (int64_t j = 0; j < nc; j++) {
                        if (v->x32) zs = zs + (float)Wt[j + l * nc] * xf[b->col0 + j];
                        else zs = (float)((double)zs + Wt[j + l * nc] * x[b->col0 + j]);
                    }
                    z[l] = (double)zs;
                } else {
                    double zs = 0.0; /* z_m in FP64 */
                    for (int64_t j = 0; j < nc; j++) {
                        if (lo && v->x32) zs += (double)((float)Wt[j + l * nc] * xf[b->col0 + j]);
                        else zs += Wt[j + l * nc] * x[b->col0 + j];
                    }
                    z[l] = zs * D[l];
                }
            }
            for (int64_t i = 0; i < m; i++) {
                double s64 = 0.0, s32 = 0.0;
                for (int64_t l = 0; l < r; l++) {
                    double t;
                    if (v->z32) t = (double)((float)Vp[i + l * m] * (float)z[l]);
                    else t = Vp[i + l * m] * z[l];
                    if (v->variant == V_M3 && P[l] == 32) s32 += t;
                    else s64 += t;
                }
                yh[i] = v->variant == V_M3 ? s64 + s32 : s64;
            }
        }
        for (int64_t i = 0; i < m; i++) y[b->row0 + i] += yh[i];
    }
    free(yh);
    free(z);
    free(xf);
}

/* ------------------------------------------------------------------------- */
/* Block-Jacobi preconditioner (not in the paper): the inverse of every dense
 * diagonal leaf block, by Gaussian elimination with partial pivoting in
 * FP64.  Applied as y_tau = A_tautau^{-1} x_tau on each diagonal leaf. */
typedef struct {
    int64_t nleaf;
    int64_t *r0, *m, *off;
    double *inv;
} ora_jacobi;

/* Invert an m x m column-major matrix A into Ainv (Gauss-Jordan with partial
 * pivoting on [A | I]).  Returns 0 on success, -1 if a pivot is zero. */
int ora_invert(int64_t m, const double *A, double *Ainv)
{
    double *W = (double *)malloc((size_t)(m * 2 * m) * sizeof(double)); /* row-major m x 2m */
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < m; j++) {
            W[i * 2 * m + j] = A[i + j * m];
            W[i * 2 * m + m + j] = i == j ? 1.0 : 0.0;
        }
    for (int64_t k = 0; k < m; k++) {
        int64_t p = k;
        for (int64_t i = k + 1; i < m; i++)
            if (fabs(W[i * 2 * m + k]) > fabs(W[p * 2 * m + k])) p = i;
        if (W[p * 2 * m + k] == 0.0) {
            free(W);
            return -1;
        }
        if (p != k)
            for (int64_t j = 0; j < 2 * m; j++) {
                double t = W[k * 2 * m + j];
                W[k * 2 * m + j] = W[p * 2 * m + j];
                W[p * 2 * m + j] = t;
            }
        double piv = W[k * 2 * m + k];
        for (int64_t j = 0; j < 2 * m; j++) W[k * 2 * m + j] /= piv;
        for (int64_t i = 0; i < m; i++) {
            if (i == k) continue;
            double f = W[i * 2 * m + k];
            if (f == 0.0) continue;
            for (int64_t j = 0; j < 2 * m; j++) W[i * 2 * m + j] -= f * W[k * 2 * m + j];
        }
    }
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < m; j++) Ainv[i + j * m] = W[i * 2 * m + m + j];
    free(W);
    return 0;
}

ora_jacobi *ora_jacobi_create(const ora_hmat *h)
{
    ora_jacobi *J = (ora_jacobi *)calloc(1, sizeof(ora_jacobi));
    int64_t cnt = 0, tot = 0;
    for (int64_t b = 0; b < h->nblocks; b++)
        if (h->blocks[b].row0 == h->blocks[b].col0 && h->blocks[b].nrows == h->blocks[b].ncols &&
            h->blocks[b].kind == 0) {
            cnt++;
            tot += h->blocks[b].nrows * h->blocks[b].nrows;
        }
    J->nleaf = cnt;
    J->r0 = (int64_t *)malloc((size_t)(cnt + 1) * sizeof(int64_t));
    J->m = (int64_t *)malloc((size_t)(cnt + 1) * sizeof(int64_t));
    J->off = (int64_t *)malloc((size_t)(cnt + 1) * sizeof(int64_t));
    J->inv = (double *)malloc((size_t)(tot + 1) * sizeof(double));
    int64_t k = 0, o = 0;
    for (int64_t b = 0; b < h->nblocks; b++) {
        const ora_block *B = &h->blocks[b];
        if (!(B->row0 == B->col0 && B->nrows == B->ncols && B->kind == 0)) continue;
        J->r0[k] = B->row0;
        J->m[k] = B->nrows;
        J->off[k] = o;
        if (ora_invert(B->nrows, h->data + B->off, J->inv + o) != 0) {
            free(J->r0); free(J->m); free(J->off); free(J->inv); free(J);
            return NULL;
        }
        o += B->nrows * B->nrows;
        k++;
    }
    return J;
}

void ora_jacobi_free(ora_jacobi *J)
{
    if (!J) return;
    free(J->r0);
    free(J->m);
    free(J->off);
    free(J->inv);
    free(J);
}

int64_t ora_jacobi_nleaf(const ora_jacobi *J) { return J->nleaf; }
void ora_jacobi_leaf(const ora_jacobi *J, int64_t k, int64_t *r0, int64_t *m, const double **inv)
{
    *r0 = J->r0[k];
    *m = J->m[k];
    *inv = J->inv + J->off[k];
}

/* Apply: y = K x.  Leaves not covered by a diagonal dense block pass x
 * through unchanged. */
void ora_jacobi_apply(const ora_jacobi *J, int64_t n, const double *x, double *y)
{
    for (int64_t i = 0; i < n; i++) y[i] = x[i];
    for (int64_t k = 0; k < J->nleaf; k++) {
        int64_t r0 = J->r0[k], m = J->m[k];
        const double *M = J->inv + J->off[k];
        for (int64_t i = 0; i < m; i++) {
            double s = 0.0;
            for (int64_t j = 0; j < m; j++) s += M[i + j * m] * x[r0 + j];
            y[r0 + i] = s;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* BiCGSTAB (Sec. 3.5, Algorithm 1; van der Vorst's method, ref. [26]) with the
 * mixed-precision product as the operator and every vector and scalar in
 * FP64.  Readings: the shadow residual is r~ = r_0; the iteration stops when
 * |s|/|b| or |r|/|b| falls below tol; convergence is then confirmed with the
 * true residual b - A x computed with the FP64 H-matrix (Sec. 4.1.3); if the
 * true residual is still too large the iteration restarts from the current
 * x, with r = r~ = that true residual and p = r.  Right preconditioning:
 * the operator is A K
 * and x is updated with K p and K s.  rho = 0, r~^T v = 0 and omega = 0 are
 * breakdowns.  b = 0 returns x = 0 at once.
 *
 * status: 0 converged, 5 breakdown, 6 no convergence within maxiter.
 * hist[i] (i = 0..iters) receives |r_i|/|b| of the recurrence and
 * shist[i] (i = 1..iters) receives |s_i|/|b|. */
typedef void (*ora_op)(const void *ctx, const double *x, double *y);

static double ora_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

typedef struct {
    const ora_conv *v;
    int literal;
} ora_opctx;

static void ora_apply_op(const ora_opctx *o, const double *x, double *y)
{
    if (o->literal) ora_matvec_literal(o->v, x, y);
    else ora_matvec(o->v, x, y);
}

/* BiCGSTAB with an optional early true-residual check (not in the paper):
 * with refine > 0 the FP64 true residual is also taken whenever the
 * recurrence residual has fallen below refine times the last true residual
 * (|r_0| at the start); a check that does not meet tol restarts exactly as a
 * failed convergence check does.  refine = 0 is ora_bicgstab. */
int ora_bicgstab_refine(const ora_conv *op, const ora_conv *op64, const ora_jacobi *K, int literal, const double *b,
                        double *x, double tol, double refine, int64_t maxiter, int64_t *iters_out,
                        int64_t *nmatvec_out, int64_t *nmatvec64_out, double *hist, double *shist,
                        double *relres_out, double *truerel_out)
{
    int64_t n = op->n;
    ora_opctx oc = {op, literal}, oc64 = {op64, 0};
    double *r = (double *)calloc((size_t)n, sizeof(double));
    double *rt = (double *)calloc((size_t)n, sizeof(double));
    double *p = (double *)calloc((size_t)n, sizeof(double));
    double *ph = (double *)calloc((size_t)n, sizeof(double));
    double *v = (double *)calloc((size_t)n, sizeof(double));
    double *s = (double *)calloc((size_t)n, sizeof(double));
    double *sh = (double *)calloc((size_t)n, sizeof(double));
    double *t = (double *)calloc((size_t)n, sizeof(double));
    double *tmp = (double *)calloc((size_t)n, sizeof(double));
    int64_t nmv = 0, nmv64 = 0, it = 0;
    int status = 6;
    double bn = sqrt(ora_dot(n, b, b));
    double rho = 0, rho_prev = 1, alpha = 1, omega = 1, relres = 0, truerel = 0, rlast = 1;
    int restart = 1;
    if (bn == 0.0) {
        for (int64_t i = 0; i < n; i++) x[i] = 0.0;
        status = 0;
        if (hist) hist[0] = 0.0;
        goto done;
    }
    /* r_0 = b - A x_0 */
    ora_apply_op(&oc, x, tmp);
    nmv++;
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - tmp[i];
    memcpy(rt, r, (size_t)n * sizeof(double));
    relres = sqrt(ora_dot(n, r, r)) / bn;
    if (hist) hist[0] = relres;
    rlast = relres;
    for (it = 1; it <= maxiter; it++) {
        rho = ora_dot(n, rt, r);
        if (rho == 0.0) {
            status = 5;
            it--;
            break;
        }
        if (restart) {
            memcpy(p, r, (size_t)n * sizeof(double));
            restart = 0;
        } else {
            double beta = (rho / rho_prev) * (alpha / omega);
            for (int64_t i = 0; i < n; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        }
        if (K) ora_jacobi_apply(K, n, p, ph);
        else memcpy(ph, p, (size_t)n * sizeof(double));
        ora_apply_op(&oc, ph, v);
        nmv++;
        double rtv = ora_dot(n, rt, v);
        if (rtv == 0.0) {
            status = 5;
            it--;
            break;
        }
        alpha = rho / rtv;
        for (int64_t i = 0; i < n; i++) s[i] = r[i] - alpha * v[i];
        double sn = sqrt(ora_dot(n, s, s)) / bn;
        if (shist) shist[it] = sn;
        int conv = 0;
        if (sn < tol) {
            for (int64_t i = 0; i < n; i++) x[i] += alpha * ph[i];
            memcpy(r, s, (size_t)n * sizeof(double));
            relres = sn;
            conv = 1;
        } else {
            if (K) ora_jacobi_apply(K, n, s, sh);
            else memcpy(sh, s, (size_t)n * sizeof(double));
            ora_apply_op(&oc, sh, t);
            nmv++;
            double tt = ora_dot(n, t, t);
            double ts = ora_dot(n, t, s);
            omega = tt == 0.0 ? 0.0 : ts / tt;
            if (omega == 0.0) {
                status = 5;
                if (hist) hist[it] = sqrt(ora_dot(n, s, s)) / bn;
                break;
            }
            for (int64_t i = 0; i < n; i++) x[i] += alpha * ph[i] + omega * sh[i];
            for (int64_t i = 0; i < n; i++) r[i] = s[i] - omega * t[i];
            relres = sqrt(ora_dot(n, r, r)) / bn;
            conv = relres < tol || (refine > 0.0 && relres < refine * rlast);
        }
        rho_prev = rho;
        if (hist) hist[it] = relres;
        if (conv) {
            /* true residual with the FP64 H-matrix */
            ora_apply_op(&oc64, x, tmp);
            nmv64++;
            for (int64_t i = 0; i < n; i++) tmp[i] = b[i] - tmp[i];
            truerel = sqrt(ora_dot(n, tmp, tmp)) / bn;
            if (truerel < tol) {
                status = 0;
                relres = truerel;
                break;
            }
            memcpy(r, tmp, (size_t)n * sizeof(double));
            memcpy(rt, tmp, (size_t)n * sizeof(double));
            relres = truerel;
            rlast = truerel;
            restart = 1;
        }
    }
    if (it > maxiter) it = maxiter;
done:
    if (status != 0 && op64) {
        ora_apply_op(&oc64, x, tmp);
        nmv64++;
        for (int64_t i = 0; i < n; i++) tmp[i] = b[i] - tmp[i];
        truerel = bn > 0 ? sqrt(ora_dot(n, tmp, tmp)) / bn : 0.0;
    } else if (status == 0 && bn > 0) {
        truerel = relres;
    }
    if (iters_out) *iters_out = it;
    if (nmatvec_out) *nmatvec_out = nmv;
    if (nmatvec64_out) *nmatvec64_out = nmv64;
    if (relres_out) *relres_out = relres;
    if (truerel_out) *truerel_out = truerel;
    free(r);
    free(rt);
    free(p);
    free(ph);
    free(v);
    free(s);
    free(sh);
    free(t);
    free(tmp);
    return status;
}

int ora_bicgstab(const ora_conv *op, const ora_conv *op64, const ora_jacobi *K, int literal, const double *b,
                 double *x, double tol, int64_t maxiter, int64_t *iters_out,
                 int64_t *nmatvec_out, int64_t *nmatvec64_out, double *hist, double *shist, double *relres_out,
                 double *truerel_out)
{
    return ora_bicgstab_refine(op, op64, K, literal, b, x, tol, 0.0, maxiter, iters_out, nmatvec_out, nmatvec64_out,
                               hist, shist, relres_out, truerel_out);
}
