/*
 * Plain FP64 CPU oracle for Electric Vertex Splitting (EVS) and the Virtual
 * Transmission Method (VTM) of Wei & Yang, "Virtual Transmission Method, A New
 * Distributed Algorithm to Solve Sparse Linear System".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  It shares no code with
 * the library (no headers, helpers or tables) and the library never calls it.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 *
 * What it computes, in the paper's order:
 *   1. EVS (Section 4, four steps): choose the boundary (membership S(v) of each
 *      vertex in the subgraphs), split every boundary vertex into one child per
 *      subgraph, split vertex weights, edge weights and sources, and attach
 *      ports (inflow currents).  Multilevel splitting (Fig. 7) pairs the
 *      children of a vertex with one virtual transmission line (VTL) per
 *      face-adjacent pair.
 *   2. VTM (Section 5, eq. (5.6)-(5.8), Table 1): every subgraph solves its
 *      port-augmented local system (5.8) with a Cholesky factor computed once,
 *      and the ports exchange waves through the transmission delay equations
 *      (5.6) with a delay of one iteration (the synchronous schedule of
 *      Example 5.1, where both sides use iteration k-1 data).
 *   3. The stopping test of Table 1 step 6, read as the relative residual of
 *      the merged potentials (mean over the children of each vertex).
 *   4. Coupled VTLs (Section 7.2, Theorem 7.1): Z_j an SPD matrix over the
 *      ports of a subgraph instead of a diagonal one (or_setup_coupled).
 *
 * Readings where the paper leaves a choice (documented with the design):
 *   - membership rules GRID / RCB / GRAPH / USER and the FACE pairing rule;
 *   - the BRANCH split of weights (Kirchhoff split) that keeps every piece
 *     weakly diagonally dominant, hence SNND (Corollary 4.1) for M-matrices;
 *   - the source split b_v / |S(v)|;
 *   - the diagonal impedance rule Z = 1 / a_vv;
 *   - zero initial waves (Example 5.1).
 *
 * Local factorisation: envelope (profile) Cholesky in the subgraph's natural
 * order (vertices sorted by global id).  Any symmetric ordering yields the same
 * solution up to rounding; the envelope form keeps the code short.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_OK = 0, OR_ERR_INVALID = -1, OR_ERR_PARTITION = -2, OR_ERR_NOT_SPD = -3, OR_ERR_OOM = -4 };
enum { OR_GRID = 0, OR_RCB = 1, OR_GRAPH = 2, OR_USER = 3 };
enum { OR_SPLIT_BRANCH = 0, OR_SPLIT_EQUAL = 1 };
enum { OR_TOPO_FACE = 0, OR_TOPO_COMPLETE = 1, OR_TOPO_TREE = 2 };

typedef struct {
    /* input copy */
    int64_t n;
    int64_t *rowptr;
    int32_t *col;
    double *val;
    /* membership S(v) */
    int32_t nsub;
    int64_t *s_ptr;
    int32_t *s_idx;
    /* local vertex lists: subdomain k holds loc_vtx[loc_ptr[k] .. loc_ptr[k+1]) (sorted) */
    int64_t *loc_ptr;
    int64_t *loc_vtx;
    /* local matrices (split pieces A~_k), CSR over local indices */
    int64_t *lrp;   /* row pointers, indexed by global local-row id (loc_ptr offset), size n_split+1 */
    int32_t *lcol;  /* local column index */
    double *lval;
    /* VTLs and ports */
    int64_t nvtl;
    int64_t *vtl_v;
    int32_t *vtl_k, *vtl_k2;
    int64_t *port_ptr;     /* per subdomain, size nsub+1 */
    int64_t *port_v;       /* global vertex of each port */
    int32_t *port_other;   /* subdomain at the other end */
    int64_t *port_twin;    /* index of the twin port */
    int64_t *port_vtl;     /* VTL of each port */
    int32_t *port_lidx;    /* local index of the port vertex in its subdomain */
    double *zdiag;         /* Z = 1/a_vv per VTL */
    int64_t rcb_seed_used;
} or_part;

/* ---------------------------------------------------------------- utilities */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* splitmix64 (Steele, Lea & Flood 2014): state += golden gamma, then mix. */
static uint64_t splitmix64(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static int sorted_intersect_count(const int32_t *a, int na, const int32_t *b, int nb) {
    int i = 0, j = 0, c = 0;
    while (i < na && j < nb) {
        if (a[i] == b[j]) { c++; i++; j++; }
        else if (a[i] < b[j]) i++;
        else j++;
    }
    return c;
}

static int sorted_contains(const int32_t *a, int na, int32_t x) {
    for (int i = 0; i < na; i++) if (a[i] == x) return 1;
    return 0;
}

void or_free(or_part *p) {
    if (!p) return;
    free(p->rowptr); free(p->col); free(p->val);
    free(p->s_ptr); free(p->s_idx); free(p->loc_ptr); free(p->loc_vtx);
    free(p->lrp); free(p->lcol); free(p->lval);
    free(p->vtl_v); free(p->vtl_k); free(p->vtl_k2);
    free(p->port_ptr); free(p->port_v); free(p->port_other); free(p->port_twin);
    free(p->port_vtl); free(p->port_lidx); free(p->zdiag);
    free(p);
}

/* ------------------------------------------------------ membership: GRID */
/* Tiles share their separator lines: per axis with nv vertices and P tiles,
 * m = nv/P if exact else (nv-1)/P; tile I covers [I*m, (I+1)*m] (last tile up
 * to nv-1).  Subdomain id is row-major over tile indices, x fastest. */
static int member_grid(or_part *p, const int32_t dims[3], const int32_t parts[3]) {
    int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    if (nv != p->n) return OR_ERR_INVALID;
    int32_t m[3];
    for (int a = 0; a < 3; a++) {
        if (parts[a] < 1 || dims[a] < 1) return OR_ERR_INVALID;
        if (parts[a] == 1) { m[a] = dims[a]; continue; }
        m[a] = (dims[a] % parts[a] == 0) ? dims[a] / parts[a] : (dims[a] - 1) / parts[a];
        if (m[a] < 1 || (int64_t)(parts[a] - 1) * m[a] > dims[a] - 1) return OR_ERR_PARTITION;
    }
    p->nsub = parts[0] * parts[1] * parts[2];
    p->s_ptr = calloc(p->n + 1, sizeof(int64_t));
    p->s_idx = malloc(sizeof(int32_t) * p->n * 8);
    if (!p->s_ptr || !p->s_idx) return OR_ERR_OOM;
    int64_t pos = 0;
    for (int64_t v = 0; v < p->n; v++) {
        int32_t c[3] = {(int32_t)(v % dims[0]), (int32_t)((v / dims[0]) % dims[1]), (int32_t)(v / ((int64_t)dims[0] * dims[1]))};
        int32_t tl[3][2], nt[3];
        for (int a = 0; a < 3; a++) {
            nt[a] = 0;
            for (int32_t I = 0; I < parts[a]; I++) {
                int32_t lo = I * m[a];
                int32_t hi = (I == parts[a] - 1) ? dims[a] - 1 : (I + 1) * m[a];
                if (c[a] >= lo && c[a] <= hi) tl[a][nt[a]++] = I;
            }
        }
        for (int iz = 0; iz < nt[2]; iz++)
            for (int iy = 0; iy < nt[1]; iy++)
                for (int ix = 0; ix < nt[0]; ix++)
                    p->s_idx[pos++] = (tl[2][iz] * parts[1] + tl[1][iy]) * parts[0] + tl[0][ix];
        p->s_ptr[v + 1] = pos;
    }
    return OR_OK;
}

/* ------------------------------------------------------- membership: RCB */
/* Seeded random recursive coordinate bisection of the vertex grid into boxes
 * that share their cut planes.  At each node (depth-first, pre-order) the
 * longest axis (ties: lowest axis) with length len = hi - lo is cut at
 * c = lo + (len * q + 50) / 100, q = 49 + (splitmix64 mod 3) percent; both
 * children contain plane c.  Leaves are numbered in visiting order.  The
 * partition is accepted when every box's owned size lies in the bounds;
 * otherwise it is drawn again from seed + 1, seed + 2, ... (64 seeds). */
typedef struct { int32_t lo[3], hi[3]; } or_box;

static int rcb_rec(or_box b, int depth, int levels, uint64_t *st, or_box *leaves, int32_t *nleaf) {
    if (depth == levels) { leaves[(*nleaf)++] = b; return OR_OK; }
    int ax = 0;
    for (int a = 1; a < 3; a++) if (b.hi[a] - b.lo[a] > b.hi[ax] - b.lo[ax]) ax = a;
    int32_t len = b.hi[ax] - b.lo[ax];
    if (len < 2) return OR_ERR_PARTITION;
    uint64_t z = splitmix64(st);
    int32_t q = 49 + (int32_t)(z % 3);
    int32_t c = b.lo[ax] + (int32_t)(((int64_t)len * q + 50) / 100);
    or_box l = b, r = b;
    l.hi[ax] = c;
    r.lo[ax] = c;
    int rc = rcb_rec(l, depth + 1, levels, st, leaves, nleaf);
    if (rc) return rc;
    return rcb_rec(r, depth + 1, levels, st, leaves, nleaf);
}

static int member_rcb_seed(or_part *p, const int32_t dims[3], int levels, uint64_t seed, double min_size,
                           double max_size) {
    int64_t nv = (int64_t)dims[0] * dims[1] * dims[2];
    if (nv != p->n || levels < 0 || levels > 20) return OR_ERR_INVALID;
    int32_t nleaf = 0;
    or_box *leaves = malloc(sizeof(or_box) << levels);
    if (!leaves) return OR_ERR_OOM;
    or_box root;
    for (int a = 0; a < 3; a++) { root.lo[a] = 0; root.hi[a] = dims[a] - 1; }
    uint64_t st = seed;
    int rc = rcb_rec(root, 0, levels, &st, leaves, &nleaf);
    if (rc) { free(leaves); return rc; }
    p->nsub = nleaf;
    /* count memberships */
    int32_t *cnt = calloc(p->n, sizeof(int32_t));
    for (int k = 0; k < nleaf; k++)
        for (int32_t z = leaves[k].lo[2]; z <= leaves[k].hi[2]; z++)
            for (int32_t y = leaves[k].lo[1]; y <= leaves[k].hi[1]; y++)
                for (int32_t x = leaves[k].lo[0]; x <= leaves[k].hi[0]; x++)
                    cnt[((int64_t)z * dims[1] + y) * dims[0] + x]++;
    p->s_ptr = calloc(p->n + 1, sizeof(int64_t));
    for (int64_t v = 0; v < p->n; v++) p->s_ptr[v + 1] = p->s_ptr[v] + cnt[v];
    p->s_idx = malloc(sizeof(int32_t) * (p->s_ptr[p->n] > 0 ? p->s_ptr[p->n] : 1));
    memset(cnt, 0, sizeof(int32_t) * p->n);
    for (int k = 0; k < nleaf; k++)  /* k ascending => each S(v) filled in sorted order */
        for (int32_t z = leaves[k].lo[2]; z <= leaves[k].hi[2]; z++)
            for (int32_t y = leaves[k].lo[1]; y <= leaves[k].hi[1]; y++)
                for (int32_t x = leaves[k].lo[0]; x <= leaves[k].hi[0]; x++) {
                    int64_t v = ((int64_t)z * dims[1] + y) * dims[0] + x;
                    p->s_idx[p->s_ptr[v] + cnt[v]++] = k;
                }
    /* acceptance: owned size sum_{v in k} 1/|S(v)|, summed in ascending vertex order */
    rc = OR_OK;
    for (int k = 0; k < nleaf && rc == OR_OK; k++) {
        double own = 0.0;
        for (int32_t z = leaves[k].lo[2]; z <= leaves[k].hi[2]; z++)
            for (int32_t y = leaves[k].lo[1]; y <= leaves[k].hi[1]; y++)
                for (int32_t x = leaves[k].lo[0]; x <= leaves[k].hi[0]; x++) {
                    int64_t v = ((int64_t)z * dims[1] + y) * dims[0] + x;
                    own += 1.0 / (double)(p->s_ptr[v + 1] - p->s_ptr[v]);
                }
        if (own < min_size || own > max_size) rc = OR_ERR_PARTITION;
    }
    free(cnt);
    free(leaves);
    return rc;
}

static int member_rcb(or_part *p, const int32_t dims[3], int levels, uint64_t seed, double min_size, double max_size) {
    for (int t = 0; t < 64; t++) {
        int rc = member_rcb_seed(p, dims, levels, seed + (uint64_t)t, min_size, max_size);
        if (rc == OR_OK) { p->rcb_seed_used = (int64_t)(seed + (uint64_t)t); return OR_OK; }
        free(p->s_ptr); p->s_ptr = NULL;
        free(p->s_idx); p->s_idx = NULL;
        if (rc != OR_ERR_PARTITION) return rc;
    }
    return OR_ERR_PARTITION;
}

/* ----------------------------------------------------- membership: GRAPH */
/* Point RCB: split the vertex set along the axis of largest coordinate extent
 * (ties: lowest axis) after sorting by (coordinate, vertex id); the left part
 * takes floor(count * floor(np/2) / np) vertices.  Then every cut edge (u,v)
 * with owner(u) < owner(v) makes u a boundary vertex shared with owner(v). */
static const double *g_coords;
static int g_dim, g_axis;
static int cmp_pt(const void *a, const void *b) {
    int64_t u = *(const int64_t *)a, v = *(const int64_t *)b;
    double cu = g_coords[u * g_dim + g_axis], cv = g_coords[v * g_dim + g_axis];
    if (cu < cv) return -1;
    if (cu > cv) return 1;
    return (u > v) - (u < v);
}

static void point_rcb(int64_t *vs, int64_t cnt, int32_t np, int32_t *next_id, int32_t *owner) {
    if (np == 1) {
        int32_t id = (*next_id)++;
        for (int64_t i = 0; i < cnt; i++) owner[vs[i]] = id;
        return;
    }
    int ax = 0;
    double best = -1.0;
    for (int a = 0; a < g_dim; a++) {
        double lo = g_coords[vs[0] * g_dim + a], hi = lo;
        for (int64_t i = 1; i < cnt; i++) {
            double c = g_coords[vs[i] * g_dim + a];
            if (c < lo) lo = c;
            if (c > hi) hi = c;
        }
        if (hi - lo > best) { best = hi - lo; ax = a; }
    }
    g_axis = ax;
    qsort(vs, (size_t)cnt, sizeof(int64_t), cmp_pt);
    int32_t nl = np / 2;
    int64_t cut = (cnt * (int64_t)nl) / np;
    point_rcb(vs, cut, nl, next_id, owner);
    point_rcb(vs + cut, cnt - cut, np - nl, next_id, owner);
}

/* Connected parts: for part k = 0, 1, ... in turn, the vertices it owns at that moment fall into
 * connected components (edges of A between two of them).  The largest component stays (equal sizes:
 * the one holding the smallest vertex).  Each other component moves, whole, to the part owning the
 * most far ends of its edges that leave part k (equal counts: the smallest part id); with no such
 * edge (a component of A by itself) it stays.  Plain version: the members of part k (its first
 * owners and the vertices moved into it) are sorted, and components are labelled by an
 * explicit-stack depth-first search started at the smallest unlabelled member. */
static void connect_parts(const or_part *p, int32_t *owner, int32_t nsub) {
    const int64_t n = p->n;
    int32_t *lab = malloc(sizeof(int32_t) * n);
    int64_t *stack = malloc(sizeof(int64_t) * n);
    int64_t *mem = malloc(sizeof(int64_t) * n);
    int64_t *csize = malloc(sizeof(int64_t) * (n + 1));
    int32_t *votes = calloc((size_t)nsub, sizeof(int32_t));
    /* members by part: the initial owners in vertex order, then the vertices moved in (linked list) */
    int64_t *first = calloc((size_t)nsub + 1, sizeof(int64_t));
    int64_t *byp = malloc(sizeof(int64_t) * n);
    int64_t *head = malloc(sizeof(int64_t) * nsub), *nxt = malloc(sizeof(int64_t) * n);
    for (int64_t v = 0; v < n; v++) first[owner[v] + 1]++;
    for (int32_t q = 0; q < nsub; q++) first[q + 1] += first[q];
    {
        int64_t *fill = malloc(sizeof(int64_t) * nsub);
        for (int32_t q = 0; q < nsub; q++) { fill[q] = first[q]; head[q] = -1; }
        for (int64_t v = 0; v < n; v++) byp[fill[owner[v]]++] = v;
        free(fill);
    }
    for (int64_t v = 0; v < n; v++) lab[v] = -1;
    for (int32_t k = 0; k < nsub; k++) {
        int64_t m = 0;
        for (int64_t i = first[k]; i < first[k + 1]; i++) mem[m++] = byp[i];
        for (int64_t v = head[k]; v >= 0; v = nxt[v]) mem[m++] = v;
        qsort(mem, (size_t)m, sizeof(int64_t), cmp_i64);
        int32_t ncomp = 0;
        for (int64_t i = 0; i < m; i++) {
            if (lab[mem[i]] >= 0) continue;
            int64_t top = 0, size = 0;
            stack[top++] = mem[i];
            lab[mem[i]] = ncomp;
            while (top > 0) {
                int64_t v = stack[--top];
                size++;
                for (int64_t e = p->rowptr[v]; e < p->rowptr[v + 1]; e++) {
                    int32_t u = p->col[e];
                    if (owner[u] == k && lab[u] < 0) { lab[u] = ncomp; stack[top++] = u; }
                }
            }
            csize[ncomp++] = size;
        }
        int32_t keep = 0;
        for (int32_t c = 1; c < ncomp; c++) if (csize[c] > csize[keep]) keep = c;
        for (int32_t c = 0; c < ncomp; c++) {
            if (c == keep) continue;
            int32_t best = -1;
            for (int64_t i = 0; i < m; i++) {
                int64_t v = mem[i];
                if (lab[v] != c) continue;
                for (int64_t e = p->rowptr[v]; e < p->rowptr[v + 1]; e++) {
                    int32_t q = owner[p->col[e]];
                    if (q == k) continue;
                    votes[q]++;
                    if (best < 0 || votes[q] > votes[best] || (votes[q] == votes[best] && q < best)) best = q;
                }
            }
            for (int64_t i = 0; i < m; i++) {  /* clear the votes */
                int64_t v = mem[i];
                if (lab[v] != c) continue;
                for (int64_t e = p->rowptr[v]; e < p->rowptr[v + 1]; e++) votes[owner[p->col[e]]] = 0;
            }
            if (best < 0) continue;
            for (int64_t i = 0; i < m; i++)
                if (lab[mem[i]] == c) {
                    owner[mem[i]] = best;
                    nxt[mem[i]] = head[best];
                    head[best] = mem[i];
                }
        }
        for (int64_t i = 0; i < m; i++) lab[mem[i]] = -1;
    }
    free(lab); free(stack); free(mem); free(csize); free(votes); free(first); free(byp); free(head); free(nxt);
}

static int member_graph(or_part *p, const double *coords, int dim, int32_t nblocks, const int64_t *bstart,
                        const int64_t *bcount, const int32_t *bparts) {
    if (!coords || dim < 1 || dim > 3 || nblocks < 1) return OR_ERR_INVALID;
    int32_t *owner = malloc(sizeof(int32_t) * p->n);
    int64_t *vs = malloc(sizeof(int64_t) * p->n);
    for (int64_t v = 0; v < p->n; v++) owner[v] = -1;
    int32_t next_id = 0;
    g_coords = coords;
    g_dim = dim;
    for (int32_t b = 0; b < nblocks; b++) {
        if (bparts[b] < 1 || bcount[b] < bparts[b]) { free(owner); free(vs); return OR_ERR_PARTITION; }
        for (int64_t i = 0; i < bcount[b]; i++) vs[i] = bstart[b] + i;
        point_rcb(vs, bcount[b], bparts[b], &next_id, owner);
    }
    free(vs);
    for (int64_t v = 0; v < p->n; v++) if (owner[v] < 0) { free(owner); return OR_ERR_PARTITION; }
    connect_parts(p, owner, next_id);
    p->nsub = next_id;
    p->s_ptr = calloc(p->n + 1, sizeof(int64_t));
    int64_t cap = p->n * 2 + 16, pos = 0;
    p->s_idx = malloc(sizeof(int32_t) * cap);
    int32_t *tmp = malloc(sizeof(int32_t) * 1024);
    for (int64_t v = 0; v < p->n; v++) {
        int nt = 0;
        tmp[nt++] = owner[v];
        for (int64_t e = p->rowptr[v]; e < p->rowptr[v + 1]; e++) {
            int32_t u = p->col[e];
            if (u == v || owner[u] <= owner[v]) continue;
            if (!sorted_contains(tmp, nt, owner[u]) && nt < 1024) tmp[nt++] = owner[u];
        }
        qsort(tmp, (size_t)nt, sizeof(int32_t), cmp_i32);
        if (pos + nt > cap) { cap = 2 * cap + nt; p->s_idx = realloc(p->s_idx, sizeof(int32_t) * cap); }
        memcpy(p->s_idx + pos, tmp, sizeof(int32_t) * nt);
        pos += nt;
        p->s_ptr[v + 1] = pos;
    }
    free(tmp);
    free(owner);
    return OR_OK;
}

/* -------------------------------------------------------- partition entry */
int or_partition(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                 int32_t kind, const int32_t *dims, const int32_t *parts, int32_t levels, uint64_t seed,
                 double min_size, double max_size, const double *coords, int32_t dim, int32_t nblocks,
                 const int64_t *bstart, const int64_t *bcount, const int32_t *bparts,
                 const int64_t *user_sptr, const int32_t *user_sidx, int32_t user_nsub,
                 int32_t split_rule, int32_t topology, or_part **out) {
    *out = NULL;
    if (n < 1 || !rowptr || !col || !val) return OR_ERR_INVALID;
    or_part *p = calloc(1, sizeof(or_part));
    p->n = n;
    int64_t nnz = rowptr[n];
    p->rowptr = malloc(sizeof(int64_t) * (n + 1));
    p->col = malloc(sizeof(int32_t) * nnz);
    p->val = malloc(sizeof(double) * nnz);
    memcpy(p->rowptr, rowptr, sizeof(int64_t) * (n + 1));
    memcpy(p->col, col, sizeof(int32_t) * nnz);
    memcpy(p->val, val, sizeof(double) * nnz);
    int rc = OR_OK;

    /* validate: sorted columns, explicit positive diagonal, finite, symmetric */
    for (int64_t v = 0; v < n && rc == OR_OK; v++) {
        int has_diag = 0;
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
            if (col[e] < 0 || col[e] >= n || !isfinite(val[e])) { rc = OR_ERR_INVALID; break; }
            if (e > rowptr[v] && col[e] <= col[e - 1]) { rc = OR_ERR_INVALID; break; }
            if (col[e] == v) { has_diag = 1; if (!(val[e] > 0.0)) rc = OR_ERR_INVALID; }
            else {
                /* find the mirror entry */
                int32_t u = col[e];
                int found = 0;
                for (int64_t f = rowptr[u]; f < rowptr[u + 1]; f++)
                    if (col[f] == v) { found = (val[f] == val[e]); break; }
                if (!found) rc = OR_ERR_INVALID;
            }
        }
        if (!has_diag) rc = OR_ERR_INVALID;
    }
    if (rc) { or_free(p); return rc; }

    switch (kind) {
        case OR_GRID: rc = member_grid(p, dims, parts); break;
        case OR_RCB: rc = member_rcb(p, dims, levels, seed, min_size, max_size); break;
        case OR_GRAPH: rc = member_graph(p, coords, dim, nblocks, bstart, bcount, bparts); break;
        case OR_USER:
            p->nsub = user_nsub;
            p->s_ptr = malloc(sizeof(int64_t) * (n + 1));
            memcpy(p->s_ptr, user_sptr, sizeof(int64_t) * (n + 1));
            p->s_idx = malloc(sizeof(int32_t) * (user_sptr[n] > 0 ? user_sptr[n] : 1));
            memcpy(p->s_idx, user_sidx, sizeof(int32_t) * user_sptr[n]);
            for (int64_t v = 0; v < n && rc == OR_OK; v++) {
                if (user_sptr[v + 1] <= user_sptr[v]) rc = OR_ERR_PARTITION;
                for (int64_t i = user_sptr[v]; i < user_sptr[v + 1]; i++) {
                    if (user_sidx[i] < 0 || user_sidx[i] >= user_nsub) rc = OR_ERR_PARTITION;
                    if (i > user_sptr[v] && user_sidx[i] <= user_sidx[i - 1]) rc = OR_ERR_PARTITION;
                }
            }
            break;
        default: rc = OR_ERR_INVALID;
    }
    if (rc) { or_free(p); return rc; }

    /* every edge must lie inside at least one subgraph: S(u) and S(v) intersect */
    for (int64_t v = 0; v < n && rc == OR_OK; v++)
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
            int32_t u = col[e];
            if (u == v) continue;
            if (!sorted_intersect_count(p->s_idx + p->s_ptr[v], (int)(p->s_ptr[v + 1] - p->s_ptr[v]),
                                        p->s_idx + p->s_ptr[u], (int)(p->s_ptr[u + 1] - p->s_ptr[u]))) {
                rc = OR_ERR_PARTITION;
                break;
            }
        }
    if (rc) { or_free(p); return rc; }

    /* local vertex lists (sorted by global id since v ascends) */
    int32_t nsub = p->nsub;
    p->loc_ptr = calloc(nsub + 1, sizeof(int64_t));
    for (int64_t i = 0; i < p->s_ptr[n]; i++) p->loc_ptr[p->s_idx[i] + 1]++;
    for (int32_t k = 0; k < nsub; k++) {
        if (p->loc_ptr[k + 1] == 0) rc = OR_ERR_PARTITION;
        p->loc_ptr[k + 1] += p->loc_ptr[k];
    }
    if (rc) { or_free(p); return rc; }
    int64_t nsplit = p->loc_ptr[nsub];
    p->loc_vtx = malloc(sizeof(int64_t) * nsplit);
    int64_t *fill = calloc(nsub, sizeof(int64_t));
    for (int64_t v = 0; v < n; v++)
        for (int64_t i = p->s_ptr[v]; i < p->s_ptr[v + 1]; i++) {
            int32_t k = p->s_idx[i];
            p->loc_vtx[p->loc_ptr[k] + fill[k]++] = v;
        }
    free(fill);

    /* EVS step 3: split vertex weights and edge weights into the pieces A~_k. */
    p->lrp = calloc(nsplit + 1, sizeof(int64_t));
    /* count entries per local row */
    for (int32_t k = 0; k < nsub; k++)
        for (int64_t li = p->loc_ptr[k]; li < p->loc_ptr[k + 1]; li++) {
            int64_t v = p->loc_vtx[li];
            int64_t c = 0;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
                int32_t u = col[e];
                if (u == v || sorted_contains(p->s_idx + p->s_ptr[u], (int)(p->s_ptr[u + 1] - p->s_ptr[u]), k)) c++;
            }
            p->lrp[li + 1] = c;
        }
    for (int64_t li = 0; li < nsplit; li++) p->lrp[li + 1] += p->lrp[li];
    p->lcol = malloc(sizeof(int32_t) * (p->lrp[nsplit] > 0 ? p->lrp[nsplit] : 1));
    p->lval = malloc(sizeof(double) * (p->lrp[nsplit] > 0 ? p->lrp[nsplit] : 1));
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t k = 0; k < nsub; k++) {
        const int64_t *lv = p->loc_vtx + p->loc_ptr[k];
        int64_t nk = p->loc_ptr[k + 1] - p->loc_ptr[k];
        for (int64_t i = 0; i < nk; i++) {
            int64_t v = lv[i];
            const int32_t *Sv = p->s_idx + p->s_ptr[v];
            int nSv = (int)(p->s_ptr[v + 1] - p->s_ptr[v]);
            double a_vv = 0.0, absum = 0.0, share = 0.0;
            int64_t out = p->lrp[p->loc_ptr[k] + i], diag_pos = -1;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
                int32_t u = col[e];
                if (u == v) { a_vv = val[e]; continue; }
                absum += fabs(val[e]);
            }
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) {
                int32_t u = col[e];
                const int32_t *Su = p->s_idx + p->s_ptr[u];
                int nSu = (int)(p->s_ptr[u + 1] - p->s_ptr[u]);
                if (u == v) { diag_pos = out; p->lcol[out] = (int32_t)i; p->lval[out] = 0.0; out++; continue; }
                if (!sorted_contains(Su, nSu, k)) continue;
                /* local index of u: binary search in the sorted local list */
                int64_t lo = 0, hi = nk - 1;
                while (lo < hi) { int64_t mid = (lo + hi) / 2; if (lv[mid] < u) lo = mid + 1; else hi = mid; }
                int cnt = sorted_intersect_count(Sv, nSv, Su, nSu);
                double w = val[e] / (double)cnt;  /* edge weight shared by the |S(u) ∩ S(v)| pieces */
                p->lcol[out] = (int32_t)lo;
                p->lval[out] = w;
                share += fabs(w);
                out++;
            }
            double d;
            if (nSv == 1) d = a_vv;
            else if (split_rule == OR_SPLIT_EQUAL) d = a_vv / (double)nSv;
            else d = share + (a_vv - absum) / (double)nSv; /* branch weight + equal share of the excess */
            p->lval[diag_pos] = d;
        }
    }

    /* VTL topology at every boundary vertex (multilevel splitting, Fig. 7). */
    /* face pairs F = { S(w) : |S(w)| = 2 }, kept as a sorted unique list of (k,k') keys */
    int64_t nf = 0;
    uint64_t *fkeys = malloc(sizeof(uint64_t) * (n + 1));
    for (int64_t v = 0; v < n; v++)
        if (p->s_ptr[v + 1] - p->s_ptr[v] == 2)
            fkeys[nf++] = ((uint64_t)(uint32_t)p->s_idx[p->s_ptr[v]] << 32) | (uint32_t)p->s_idx[p->s_ptr[v] + 1];
    int64_t cap = 1024;
    p->vtl_v = malloc(sizeof(int64_t) * cap);
    p->vtl_k = malloc(sizeof(int32_t) * cap);
    p->vtl_k2 = malloc(sizeof(int32_t) * cap);
    p->nvtl = 0;
    /* sort the face keys (shell sort) and drop duplicates */
    {
        int64_t gap;
        for (gap = nf / 2; gap > 0; gap /= 2)
            for (int64_t i = gap; i < nf; i++) {
                uint64_t t = fkeys[i];
                int64_t j = i;
                while (j >= gap && fkeys[j - gap] > t) { fkeys[j] = fkeys[j - gap]; j -= gap; }
                fkeys[j] = t;
            }
    }
    int64_t nfu = 0;
    for (int64_t i = 0; i < nf; i++) if (nfu == 0 || fkeys[nfu - 1] != fkeys[i]) fkeys[nfu++] = fkeys[i];
    for (int64_t v = 0; v < n; v++) {
        const int32_t *Sv = p->s_idx + p->s_ptr[v];
        int m = (int)(p->s_ptr[v + 1] - p->s_ptr[v]);
        if (m < 2) continue;
        int npair = m * (m - 1) / 2;
        char *use = calloc(npair, 1);
        int nuse = 0;
        if (topology == OR_TOPO_FACE || topology == OR_TOPO_TREE) {
            int q = 0;
            for (int a = 0; a < m; a++)
                for (int b = a + 1; b < m; b++, q++) {
                    uint64_t key = ((uint64_t)(uint32_t)Sv[a] << 32) | (uint32_t)Sv[b];
                    int64_t lo = 0, hi = nfu;
                    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (fkeys[mid] < key) lo = mid + 1; else hi = mid; }
                    if (lo < nfu && fkeys[lo] == key) { use[q] = 1; nuse++; }
                }
            /* connectivity of the children graph on S(v) */
            int *comp = malloc(sizeof(int) * m);
            for (int a = 0; a < m; a++) comp[a] = a;
            int changed = 1;
            while (changed) {
                changed = 0;
                q = 0;
                for (int a = 0; a < m; a++)
                    for (int b = a + 1; b < m; b++, q++)
                        if (use[q] && comp[a] != comp[b]) {
                            int c = comp[a] < comp[b] ? comp[a] : comp[b];
                            comp[a] = comp[b] = c;
                            changed = 1;
                        }
            }
            int connected = 1;
            for (int a = 0; a < m; a++) if (comp[a] != comp[0]) connected = 0;
            free(comp);
            if (!connected) { memset(use, 1, npair); nuse = npair; }
        } else {
            memset(use, 1, npair);
            nuse = npair;
        }
        if (topology == OR_TOPO_TREE) {
            /* repeated binary splitting: each further split of a child adds one VTL, so the VTLs of v
               form a tree.  Keep the FACE pairs, taken in (a, b) order, that join two children not yet
               connected (a spanning tree of the FACE pairs, which connect S(v)). */
            int *lab = malloc(sizeof(int) * m);
            for (int a = 0; a < m; a++) lab[a] = a;
            int q2 = 0;
            for (int a = 0; a < m; a++)
                for (int b = a + 1; b < m; b++, q2++) {
                    if (!use[q2]) continue;
                    if (lab[a] == lab[b]) { use[q2] = 0; nuse--; continue; }
                    const int gone = lab[b], into = lab[a];
                    for (int c = 0; c < m; c++) if (lab[c] == gone) lab[c] = into;
                }
            free(lab);
        }
        int q = 0;
        for (int a = 0; a < m; a++)
            for (int b = a + 1; b < m; b++, q++) {
                if (!use[q]) continue;
                if (p->nvtl == cap) {
                    cap *= 2;
                    p->vtl_v = realloc(p->vtl_v, sizeof(int64_t) * cap);
                    p->vtl_k = realloc(p->vtl_k, sizeof(int32_t) * cap);
                    p->vtl_k2 = realloc(p->vtl_k2, sizeof(int32_t) * cap);
                }
                p->vtl_v[p->nvtl] = v;
                p->vtl_k[p->nvtl] = Sv[a];
                p->vtl_k2[p->nvtl] = Sv[b];
                p->nvtl++;
            }
        free(use);
        (void)nuse;
    }
    free(fkeys);

    /* ports: two per VTL; within subdomain k ordered by (v, other end) */
    int64_t nports = 2 * p->nvtl;
    p->port_ptr = calloc(nsub + 1, sizeof(int64_t));
    for (int64_t l = 0; l < p->nvtl; l++) { p->port_ptr[p->vtl_k[l] + 1]++; p->port_ptr[p->vtl_k2[l] + 1]++; }
    for (int32_t k = 0; k < nsub; k++) p->port_ptr[k + 1] += p->port_ptr[k];
    p->port_v = malloc(sizeof(int64_t) * (nports + 1));
    p->port_other = malloc(sizeof(int32_t) * (nports + 1));
    p->port_twin = malloc(sizeof(int64_t) * (nports + 1));
    p->port_vtl = malloc(sizeof(int64_t) * (nports + 1));
    p->port_lidx = malloc(sizeof(int32_t) * (nports + 1));
    /* VTLs are ordered by (v, k, k'); scanning them in order and appending to
     * each end gives, per subdomain, ports ordered by v and then by the other
     * end, because for a fixed v the other ends of subdomain k appear in
     * increasing order (pairs (j,k) with j<k come before pairs (k,j') with j'>k). */
    int64_t *pf = calloc(nsub, sizeof(int64_t));
    int64_t *end_a = malloc(sizeof(int64_t) * (p->nvtl + 1)), *end_b = malloc(sizeof(int64_t) * (p->nvtl + 1));
    for (int64_t l = 0; l < p->nvtl; l++) {
        int32_t k = p->vtl_k[l], k2 = p->vtl_k2[l];
        int64_t pa = p->port_ptr[k] + pf[k]++;
        int64_t pb = p->port_ptr[k2] + pf[k2]++;
        p->port_v[pa] = p->vtl_v[l]; p->port_other[pa] = k2; p->port_vtl[pa] = l;
        p->port_v[pb] = p->vtl_v[l]; p->port_other[pb] = k; p->port_vtl[pb] = l;
        end_a[l] = pa;
        end_b[l] = pb;
    }
    for (int64_t l = 0; l < p->nvtl; l++) { p->port_twin[end_a[l]] = end_b[l]; p->port_twin[end_b[l]] = end_a[l]; }
    free(end_a); free(end_b); free(pf);
    /* check the (v, other) order claimed above, and find local indices */
    for (int32_t k = 0; k < nsub && rc == OR_OK; k++) {
        const int64_t *lv = p->loc_vtx + p->loc_ptr[k];
        int64_t nk = p->loc_ptr[k + 1] - p->loc_ptr[k];
        for (int64_t q = p->port_ptr[k]; q < p->port_ptr[k + 1]; q++) {
            if (q > p->port_ptr[k] && (p->port_v[q] < p->port_v[q - 1] ||
                (p->port_v[q] == p->port_v[q - 1] && p->port_other[q] <= p->port_other[q - 1]))) rc = OR_ERR_PARTITION;
            int64_t lo = 0, hi = nk - 1;
            while (lo < hi) { int64_t mid = (lo + hi) / 2; if (lv[mid] < p->port_v[q]) lo = mid + 1; else hi = mid; }
            p->port_lidx[q] = (int32_t)lo;
        }
    }
    /* diagonal impedance rule Z = 1 / a_vv (original diagonal) */
    p->zdiag = malloc(sizeof(double) * (p->nvtl + 1));
    for (int64_t l = 0; l < p->nvtl; l++) {
        int64_t v = p->vtl_v[l];
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; e++) if (col[e] == v) p->zdiag[l] = 1.0 / val[e];
    }
    if (rc) { or_free(p); return rc; }
    *out = p;
    return OR_OK;
}

/* RCB: the seed whose boxes met the owned-size bounds (0 for other membership rules). */
int64_t or_rcb_seed(const or_part *p) { return p->rcb_seed_used; }

/* sizes: n, nsub, n_split, local nnz, nvtl, nports, s_idx size */
void or_sizes(const or_part *p, int64_t *out) {
    out[0] = p->n;
    out[1] = p->nsub;
    out[2] = p->loc_ptr[p->nsub];
    out[3] = p->lrp[p->loc_ptr[p->nsub]];
    out[4] = p->nvtl;
    out[5] = 2 * p->nvtl;
    out[6] = p->s_ptr[p->n];
}

void or_get(const or_part *p, int64_t *s_ptr, int32_t *s_idx, int64_t *loc_ptr, int64_t *loc_vtx,
            int64_t *lrp, int32_t *lcol, double *lval, int64_t *vtl_v, int32_t *vtl_k, int32_t *vtl_k2,
            int64_t *port_ptr, int64_t *port_v, int32_t *port_other, int64_t *port_twin, int64_t *port_vtl,
            double *zdiag) {
    int64_t n = p->n, ns = p->loc_ptr[p->nsub], nl = p->lrp[ns], np = 2 * p->nvtl;
    if (s_ptr) memcpy(s_ptr, p->s_ptr, sizeof(int64_t) * (n + 1));
    if (s_idx) memcpy(s_idx, p->s_idx, sizeof(int32_t) * p->s_ptr[n]);
    if (loc_ptr) memcpy(loc_ptr, p->loc_ptr, sizeof(int64_t) * (p->nsub + 1));
    if (loc_vtx) memcpy(loc_vtx, p->loc_vtx, sizeof(int64_t) * ns);
    if (lrp) memcpy(lrp, p->lrp, sizeof(int64_t) * (ns + 1));
    if (lcol) memcpy(lcol, p->lcol, sizeof(int32_t) * nl);
    if (lval) memcpy(lval, p->lval, sizeof(double) * nl);
    if (vtl_v) memcpy(vtl_v, p->vtl_v, sizeof(int64_t) * p->nvtl);
    if (vtl_k) memcpy(vtl_k, p->vtl_k, sizeof(int32_t) * p->nvtl);
    if (vtl_k2) memcpy(vtl_k2, p->vtl_k2, sizeof(int32_t) * p->nvtl);
    if (port_ptr) memcpy(port_ptr, p->port_ptr, sizeof(int64_t) * (p->nsub + 1));
    if (port_v) memcpy(port_v, p->port_v, sizeof(int64_t) * np);
    if (port_other) memcpy(port_other, p->port_other, sizeof(int32_t) * np);
    if (port_twin) memcpy(port_twin, p->port_twin, sizeof(int64_t) * np);
    if (port_vtl) memcpy(port_vtl, p->port_vtl, sizeof(int64_t) * np);
    if (zdiag) memcpy(zdiag, p->zdiag, sizeof(double) * p->nvtl);
}

/* ------------------------------------------------------------- VTM solve */

/* Envelope Cholesky of one port-augmented local matrix (5.8):
 *   K_k = A~_k + sum_{ports p in k} (1/Z_p) e_v(p) e_v(p)^T.
 * Row i of L is stored for columns fnz[i]..i, at env[eptr[i] + (j - fnz[i])]. */
typedef struct {
    int64_t nk;
    int64_t *fnz, *eptr;
    double *env;
} or_factor;

/* Coupled VTLs (Section 7.2): per port p, the ports q of the same subgraph whose VTLs are coupled
 * with p's (p itself included), with (Z_j^{-1})_pq and (Z_j)_pq; cptr == NULL when Z is diagonal. */
typedef struct {
    int64_t *cptr, *cq;
    double *cy, *cz;
} or_coupling;

static int factor_local(const or_part *p, int32_t k, const double *zport, const or_coupling *cp, or_factor *F) {
    int64_t base = p->loc_ptr[k], nk = p->loc_ptr[k + 1] - base;
    F->nk = nk;
    F->fnz = malloc(sizeof(int64_t) * nk);
    F->eptr = malloc(sizeof(int64_t) * (nk + 1));
    for (int64_t i = 0; i < nk; i++) {
        int64_t f = i;
        for (int64_t e = p->lrp[base + i]; e < p->lrp[base + i + 1]; e++) if (p->lcol[e] < f) f = p->lcol[e];
        F->fnz[i] = f;
    }
    if (cp->cptr)  /* the dense port blocks Z_j^{-1} widen the envelope */
        for (int64_t q = p->port_ptr[k]; q < p->port_ptr[k + 1]; q++)
            for (int64_t e = cp->cptr[q]; e < cp->cptr[q + 1]; e++) {
                int64_t i = p->port_lidx[q], j = p->port_lidx[cp->cq[e]];
                if (j < F->fnz[i]) F->fnz[i] = j;
            }
    F->eptr[0] = 0;
    for (int64_t i = 0; i < nk; i++) F->eptr[i + 1] = F->eptr[i] + (i - F->fnz[i] + 1);
    F->env = calloc(F->eptr[nk], sizeof(double));
    if (!F->env) return OR_ERR_OOM;
    /* scatter K (lower part) into the envelope */
    for (int64_t i = 0; i < nk; i++)
        for (int64_t e = p->lrp[base + i]; e < p->lrp[base + i + 1]; e++) {
            int64_t j = p->lcol[e];
            if (j <= i) F->env[F->eptr[i] + (j - F->fnz[i])] = p->lval[e];
        }
    if (cp->cptr) {  /* K_k = A~_k + R^T Z_j^{-1} R: the whole port block, lower part */
        for (int64_t q = p->port_ptr[k]; q < p->port_ptr[k + 1]; q++)
            for (int64_t e = cp->cptr[q]; e < cp->cptr[q + 1]; e++) {
                int64_t i = p->port_lidx[q], j = p->port_lidx[cp->cq[e]];
                if (j <= i) F->env[F->eptr[i] + (j - F->fnz[i])] += cp->cy[e];
            }
    } else {
        for (int64_t q = p->port_ptr[k]; q < p->port_ptr[k + 1]; q++) {
            int64_t i = p->port_lidx[q];
            F->env[F->eptr[i] + (i - F->fnz[i])] += 1.0 / zport[q];
        }
    }
    /* row-by-row Cholesky inside the envelope */
    for (int64_t i = 0; i < nk; i++) {
        double *Li = F->env + F->eptr[i];
        int64_t fi = F->fnz[i];
        for (int64_t j = fi; j < i; j++) {
            double *Lj = F->env + F->eptr[j];
            int64_t fj = F->fnz[j];
            int64_t s = fi > fj ? fi : fj;
            double acc = Li[j - fi];
            for (int64_t t = s; t < j; t++) acc -= Li[t - fi] * Lj[t - fj];
            Li[j - fi] = acc / Lj[j - fj];
        }
        double d = Li[i - fi];
        for (int64_t t = fi; t < i; t++) d -= Li[t - fi] * Li[t - fi];
        if (!(d > 0.0) || !isfinite(d)) return OR_ERR_NOT_SPD;
        Li[i - fi] = sqrt(d);
    }
    return OR_OK;
}

static void solve_local(const or_factor *F, double *x) {
    int64_t nk = F->nk;
    for (int64_t i = 0; i < nk; i++) {  /* L y = r */
        const double *Li = F->env + F->eptr[i];
        int64_t fi = F->fnz[i];
        double acc = x[i];
        for (int64_t t = fi; t < i; t++) acc -= Li[t - fi] * x[t];
        x[i] = acc / Li[i - fi];
    }
    for (int64_t i = nk - 1; i >= 0; i--) {  /* L^T x = y */
        const double *Li = F->env + F->eptr[i];
        int64_t fi = F->fnz[i];
        x[i] /= Li[i - fi];
        for (int64_t t = fi; t < i; t++) x[t] -= Li[t - fi] * x[i];
    }
}

typedef struct {
    or_part *p;
    or_factor *f;
    double *zport;  /* Z at each port (equal at both ends of a VTL) */
    or_coupling c;  /* coupled VTLs, or all NULL */
} or_solver;

static int factor_all(or_solver *s) {
    int rc = OR_OK;
    const or_part *p = s->p;
    s->f = calloc(p->nsub, sizeof(or_factor));
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t k = 0; k < p->nsub; k++) {
        int r = factor_local(p, k, s->zport, &s->c, &s->f[k]);
        if (r) {
#pragma omp critical
            rc = r;
        }
    }
    return rc;
}

int or_setup(or_part *p, const double *z_vtl, or_solver **out) {
    *out = NULL;
    int64_t np = 2 * p->nvtl;
    for (int64_t l = 0; l < p->nvtl; l++) if (!(z_vtl[l] > 0.0) || !isfinite(z_vtl[l])) return OR_ERR_INVALID;
    or_solver *s = calloc(1, sizeof(or_solver));
    s->p = p;
    s->zport = malloc(sizeof(double) * (np + 1));
    for (int64_t q = 0; q < np; q++) s->zport[q] = z_vtl[p->port_vtl[q]];
    int rc = factor_all(s);
    *out = s;
    return rc;
}

/* Union-find root with path halving. */
static int64_t uf_root(int64_t *par, int64_t x) {
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

/*
 * Coupled VTLs (Section 7.2, Theorem 7.1): the impedance is a symmetric matrix Z over the VTLs with
 * diagonal z_vtl and the off-diagonal entries Z[l1[e]][l2[e]] = Z[l2[e]][l1[e]] = zc[e] (each pair
 * given once).  Coupled VTLs must join the same two subgraphs; Z is then block diagonal over the
 * groups of coupled VTLs, and both subgraphs of a group use the group's block as their Z_j (in the
 * order of their own ports, so that the twins see the same matrix).  Every block must be SPD.  The
 * blocks are inverted here by a plain Cholesky factorisation and unit solves.
 */
int or_setup_coupled(or_part *p, const double *z_vtl, int64_t ncpl, const int64_t *l1, const int64_t *l2,
                     const double *zc, or_solver **out) {
    *out = NULL;
    const int64_t nl = p->nvtl, np = 2 * nl;
    for (int64_t l = 0; l < nl; l++) if (!(z_vtl[l] > 0.0) || !isfinite(z_vtl[l])) return OR_ERR_INVALID;
    for (int64_t e = 0; e < ncpl; e++) {
        if (l1[e] < 0 || l1[e] >= nl || l2[e] < 0 || l2[e] >= nl || l1[e] == l2[e] || !isfinite(zc[e]))
            return OR_ERR_INVALID;
        if (p->vtl_k[l1[e]] != p->vtl_k[l2[e]] || p->vtl_k2[l1[e]] != p->vtl_k2[l2[e]]) return OR_ERR_INVALID;
    }
    /* groups of coupled VTLs; member lists in ascending VTL order */
    int64_t *par = malloc(sizeof(int64_t) * (nl + 1));
    for (int64_t l = 0; l < nl; l++) par[l] = l;
    for (int64_t e = 0; e < ncpl; e++) {
        int64_t a = uf_root(par, l1[e]), b = uf_root(par, l2[e]);
        if (a != b) par[a < b ? b : a] = a < b ? a : b;
    }
    int64_t *root = malloc(sizeof(int64_t) * (nl + 1)), *gsz = calloc(nl + 1, sizeof(int64_t));
    int64_t *gpos = malloc(sizeof(int64_t) * (nl + 1));  /* index of a VTL inside its group */
    for (int64_t l = 0; l < nl; l++) { root[l] = uf_root(par, l); gpos[l] = gsz[root[l]]++; }
    int64_t *gptr = calloc(nl + 1, sizeof(int64_t)), *gmem = malloc(sizeof(int64_t) * (nl + 1));
    for (int64_t l = 0; l < nl; l++) gptr[l + 1] = gptr[l] + gsz[l];
    for (int64_t l = 0; l < nl; l++) gmem[gptr[root[l]] + gpos[l]] = l;
    /* the two ports of every VTL: end 0 in vtl_k, end 1 in vtl_k2 */
    int64_t *vport = malloc(sizeof(int64_t) * (np + 1));
    for (int32_t k = 0; k < p->nsub; k++)
        for (int64_t q = p->port_ptr[k]; q < p->port_ptr[k + 1]; q++) {
            int64_t l = p->port_vtl[q];
            vport[2 * l + (k == p->vtl_k[l] ? 0 : 1)] = q;
        }
    /* dense Z and Y = Z^{-1} per group (groups indexed by their root), entries kept per VTL pair */
    int64_t *yoff = calloc(nl + 1, sizeof(int64_t));
    int64_t tot = 0;
    for (int64_t r = 0; r < nl; r++) { yoff[r] = tot; tot += gsz[r] * gsz[r]; }
    double *Zd = calloc(tot + 1, sizeof(double)), *Yd = calloc(tot + 1, sizeof(double));
    for (int64_t l = 0; l < nl; l++) Zd[yoff[root[l]] + gpos[l] * gsz[root[l]] + gpos[l]] = z_vtl[l];
    for (int64_t e = 0; e < ncpl; e++) {
        int64_t r = root[l1[e]], m = gsz[r], i = gpos[l1[e]], j = gpos[l2[e]];
        Zd[yoff[r] + i * m + j] = zc[e];
        Zd[yoff[r] + j * m + i] = zc[e];
    }
    int rc = OR_OK;
    for (int64_t r = 0; r < nl && rc == OR_OK; r++) {
        int64_t m = gsz[r];
        if (m == 0) continue;
        double *Zg = Zd + yoff[r], *Yg = Yd + yoff[r];
        double *L = calloc(m * m, sizeof(double)), *col = malloc(sizeof(double) * m);
        for (int64_t i = 0; i < m && rc == OR_OK; i++)  /* Z = L L^T */
            for (int64_t j = 0; j <= i; j++) {
                double acc = Zg[i * m + j];
                for (int64_t t = 0; t < j; t++) acc -= L[i * m + t] * L[j * m + t];
                if (i == j) {
                    if (!(acc > 0.0)) { rc = OR_ERR_INVALID; break; }
                    L[i * m + i] = sqrt(acc);
                } else {
                    L[i * m + j] = acc / L[j * m + j];
                }
            }
        for (int64_t c = 0; c < m && rc == OR_OK; c++) {  /* column c of Z^{-1}: L L^T y = e_c */
            for (int64_t i = 0; i < m; i++) {
                double acc = i == c ? 1.0 : 0.0;
                for (int64_t t = 0; t < i; t++) acc -= L[i * m + t] * col[t];
                col[i] = acc / L[i * m + i];
            }
            for (int64_t i = m - 1; i >= 0; i--) {
                double acc = col[i];
                for (int64_t t = i + 1; t < m; t++) acc -= L[t * m + i] * col[t];
                col[i] = acc / L[i * m + i];
            }
            for (int64_t i = 0; i < m; i++) Yg[i * m + c] = col[i];
        }
        free(L);
        free(col);
    }
    or_solver *s = NULL;
    if (rc == OR_OK) {
        s = calloc(1, sizeof(or_solver));
        s->p = p;
        s->zport = malloc(sizeof(double) * (np + 1));
        for (int64_t q = 0; q < np; q++) s->zport[q] = z_vtl[p->port_vtl[q]];
        /* per port: the ports of its own subgraph on the VTLs of its group, in group order */
        s->c.cptr = calloc(np + 1, sizeof(int64_t));
        for (int64_t q = 0; q < np; q++) s->c.cptr[q + 1] = s->c.cptr[q] + gsz[root[p->port_vtl[q]]];
        s->c.cq = malloc(sizeof(int64_t) * (s->c.cptr[np] + 1));
        s->c.cy = malloc(sizeof(double) * (s->c.cptr[np] + 1));
        s->c.cz = malloc(sizeof(double) * (s->c.cptr[np] + 1));
        for (int64_t q = 0; q < np; q++) {
            int64_t l = p->port_vtl[q], r = root[l], m = gsz[r], i = gpos[l];
            int end = vport[2 * l] == q ? 0 : 1;
            for (int64_t j = 0; j < m; j++) {
                int64_t e = s->c.cptr[q] + j, lj = gmem[gptr[r] + j];
                s->c.cq[e] = vport[2 * lj + end];
                s->c.cy[e] = Yd[yoff[r] + i * m + j];
                s->c.cz[e] = Zd[yoff[r] + i * m + j];
            }
        }
        rc = factor_all(s);
    }
    free(par); free(root); free(gsz); free(gpos); free(gptr); free(gmem); free(vport); free(yoff); free(Zd); free(Yd);
    *out = s;
    return rc;
}

void or_solver_free(or_solver *s) {
    if (!s) return;
    if (s->f)
        for (int32_t k = 0; k < s->p->nsub; k++) { free(s->f[k].fnz); free(s->f[k].eptr); free(s->f[k].env); }
    free(s->f);
    free(s->zport);
    free(s->c.cptr); free(s->c.cq); free(s->c.cy); free(s->c.cz);
    free(s);
}

/* Merged potentials xbar_v = mean over the children of v, residual b - A xbar,
 * and the relative residual norm per system. */
static void merged_residual(const or_part *p, const double *xloc, const double *b, double *xbar,
                            int32_t nsys, const int64_t *sys_ptr, double *relres) {
    int64_t n = p->n;
    for (int64_t v = 0; v < n; v++) xbar[v] = 0.0;
    /* sum over children in subdomain order */
    for (int32_t k = 0; k < p->nsub; k++)
        for (int64_t li = p->loc_ptr[k]; li < p->loc_ptr[k + 1]; li++) xbar[p->loc_vtx[li]] += xloc[li];
    for (int64_t v = 0; v < n; v++) xbar[v] /= (double)(p->s_ptr[v + 1] - p->s_ptr[v]);
    for (int32_t s = 0; s < nsys; s++) {
        double rr = 0.0, bb = 0.0;
#pragma omp parallel for reduction(+ : rr, bb)
        for (int64_t v = sys_ptr[s]; v < sys_ptr[s + 1]; v++) {
            double r = b[v];
            for (int64_t e = p->rowptr[v]; e < p->rowptr[v + 1]; e++) r -= p->val[e] * xbar[p->col[e]];
            rr += r * r;
            bb += b[v] * b[v];
        }
        relres[s] = sqrt(rr) / sqrt(bb);
    }
}

/* One subgraph's part of a sweep: right side of (5.8), local solve, port currents and outgoing
 * waves (right side of (5.6)).  Diagonal Z:
 *   rhs += (a_p / Z_p) e_v(p);  w_p = (a_p - u_p) / Z_p;  o_p = u_p - Z_p w_p
 * coupled VTLs (Z_j a matrix over the subgraph's ports):
 *   rhs += R^T Z_j^{-1} a;  w = Z_j^{-1} (a - u);  o = u - Z_j w */
static void sweep_local(const or_solver *s, int32_t k, const double *b, const double *a, double *xk, double *o) {
    const or_part *p = s->p;
    int64_t base = p->loc_ptr[k], nk = p->loc_ptr[k + 1] - base;
    for (int64_t i = 0; i < nk; i++) {
        int64_t v = p->loc_vtx[base + i];
        xk[i] = b[v] / (double)(p->s_ptr[v + 1] - p->s_ptr[v]);  /* source split */
    }
    const int64_t q0 = p->port_ptr[k], q1 = p->port_ptr[k + 1];
    if (!s->c.cptr) {
        for (int64_t q = q0; q < q1; q++) xk[p->port_lidx[q]] += a[q] / s->zport[q];
        solve_local(&s->f[k], xk);
        for (int64_t q = q0; q < q1; q++) {
            double u = xk[p->port_lidx[q]];
            double w = (a[q] - u) / s->zport[q];
            o[q] = u - s->zport[q] * w;
        }
        return;
    }
    const or_coupling *c = &s->c;
    for (int64_t q = q0; q < q1; q++)
        for (int64_t e = c->cptr[q]; e < c->cptr[q + 1]; e++) xk[p->port_lidx[q]] += c->cy[e] * a[c->cq[e]];
    solve_local(&s->f[k], xk);
    double *w = malloc(sizeof(double) * (q1 - q0 + 1));
    for (int64_t q = q0; q < q1; q++) {
        double acc = 0.0;
        for (int64_t e = c->cptr[q]; e < c->cptr[q + 1]; e++) acc += c->cy[e] * (a[c->cq[e]] - xk[p->port_lidx[c->cq[e]]]);
        w[q - q0] = acc;
    }
    for (int64_t q = q0; q < q1; q++) {
        double acc = xk[p->port_lidx[q]];
        for (int64_t e = c->cptr[q]; e < c->cptr[q + 1]; e++) acc -= c->cz[e] * w[c->cq[e] - q0];
        o[q] = acc;
    }
    free(w);
}

/*
 * Run VTM for one right-hand side b (length n) from incoming waves a (length
 * nports; zeros = Example 5.1's start).  Every sweep:
 *   rhs_k = b~_k + sum_p (a_p / Z_p) e_v(p)          (right side of (5.8))
 *   x_k   = K_k^{-1} rhs_k
 *   u_p   = x_k[v(p)],  w_p = (a_p - u_p) / Z_p      (inflow current, below (5.8))
 *   o_p   = u_p - Z_p w_p                            (outgoing wave, right side of (5.6))
 *   a_p  <- o_twin(p)                                (delay of one iteration)
 * The test runs every `check_every` sweeps; the run stops when every system's
 * relative residual is <= tol or after max_sweeps.  On return x holds the
 * merged potentials of the last sweep, a the incoming waves for the next sweep,
 * iters[s] the first passing sweep (or -1) and relres[s] the last residual.
 * Returns the number of sweeps done.
 */
int64_t or_run(or_solver *s, const double *b, double *a, int64_t max_sweeps, int64_t check_every, double tol,
               int32_t nsys, const int64_t *sys_ptr, double *x, int64_t *iters, double *relres, double *hist,
               int64_t hist_cap) {
    const or_part *p = s->p;
    int64_t nsplit = p->loc_ptr[p->nsub], np = 2 * p->nvtl;
    double *xloc = calloc(nsplit + 1, sizeof(double));
    double *o = calloc(np + 1, sizeof(double));
    double *rr = calloc(nsys, sizeof(double));
    for (int32_t q = 0; q < nsys; q++) iters[q] = -1;
    int64_t sweep = 0, nh = 0;
    while (sweep < max_sweeps) {
        sweep++;
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t k = 0; k < p->nsub; k++) sweep_local(s, k, b, a, xloc + p->loc_ptr[k], o);
        for (int64_t q = 0; q < np; q++) a[q] = o[p->port_twin[q]];
        if (check_every > 0 && (sweep % check_every == 0 || sweep == max_sweeps)) {
            merged_residual(p, xloc, b, x, nsys, sys_ptr, rr);
            int done = 1;
            for (int32_t q = 0; q < nsys; q++) {
                relres[q] = rr[q];
                if (iters[q] < 0 && rr[q] <= tol) iters[q] = sweep;
                if (iters[q] < 0) done = 0;
            }
            if (hist && nh < hist_cap) hist[nh++] = rr[0];
            if (done) break;
        }
    }
    if (check_every <= 0) {
        merged_residual(p, xloc, b, x, nsys, sys_ptr, rr);
        for (int32_t q = 0; q < nsys; q++) relres[q] = rr[q];
    }
    free(xloc);
    free(o);
    free(rr);
    return sweep;
}

/* Local solution of the last sweep, for tests that look at twin agreement. */
int64_t or_run_local(or_solver *s, const double *b, double *a, int64_t nsweeps, double *xloc_out) {
    const or_part *p = s->p;
    int64_t np = 2 * p->nvtl;
    double *o = calloc(np + 1, sizeof(double));
    for (int64_t sweep = 0; sweep < nsweeps; sweep++) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int32_t k = 0; k < p->nsub; k++) sweep_local(s, k, b, a, xloc_out + p->loc_ptr[k], o);
        for (int64_t q = 0; q < np; q++) a[q] = o[p->port_twin[q]];
    }
    free(o);
    return nsweeps;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* First n outputs of splitmix64 from a seed (exposed so tests can pin the generator). */
void or_splitmix64_seq(uint64_t seed, int32_t n, uint64_t *out) {
    uint64_t st = seed;
    for (int32_t i = 0; i < n; i++) out[i] = splitmix64(&st);
}
