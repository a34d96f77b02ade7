/*
 * oracle.c -- plain CPU FP64 reference for the decomposed-TV min-cut method of
 * Kumar, Barbero, Jegelka, Sra and Bach, "Convex Optimization for Parallel
 * Energy Minimization" (arXiv:1503.01563).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the GPU library is
 * compared against; it is deliberately plain, slow and written for reading.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Conventions (public API of the project):
 *   grid [D][H][W], W contiguous; 2D grids have D = 1.
 *   axis 0 = W (stride 1), axis 1 = H (stride W), axis 2 = D (stride H*W).
 *   a[j][i] is the weight of the edge (i, i + stride_j); it is ignored on
 *   the last slice along axis j.
 *   Cut energy  E(S) = sum_{i in S} w_i + sum_edges a_e [edge crosses S].
 *   The paper minimises f(x) - w^T x (Sec. 2, eq. (D)); with our sign the
 *   paper's w is u = -w, and the TV problem is min_x f(x) + 1/2 |x - u|^2
 *   (Sec. 2.3, eq. (TV)).
 *
 * Parity status of each function is listed in its comment.
 *
 * Threads.  Built plainly (liborc.so) everything runs on one thread.  Built
 * with -fopenmp (liborc_omp.so, the benchmark's all-core baseline) the chains
 * of a family, the elementwise updates and the nine threshold energies of a
 * certificate are spread over threads; every sum keeps its serial order, so
 * both builds return identical bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_NOMEM (-2)

/* ------------------------------------------------------------------------ */
/* grid helpers                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    long D, H, W, n;
    int ndim;
} orc_grid;

static int orc_grid_make(int ndim, const long *dims, orc_grid *g)
{
    if (ndim == 2) {
        g->D = 1; g->H = dims[0]; g->W = dims[1];
    } else if (ndim == 3) {
        g->D = dims[0]; g->H = dims[1]; g->W = dims[2];
    } else {
        return ORC_ERR_ARG;
    }
    if (g->D <= 0 || g->H <= 0 || g->W <= 0) return ORC_ERR_ARG;
    g->ndim = ndim;
    g->n = g->D * g->H * g->W;
    return ORC_OK;
}

static long orc_stride(const orc_grid *g, int axis)
{
    return axis == 0 ? 1 : (axis == 1 ? g->W : g->W * g->H);
}

static long orc_extent(const orc_grid *g, int axis)
{
    return axis == 0 ? g->W : (axis == 1 ? g->H : g->D);
}

/* coordinate of voxel i along the axis */
static long orc_coord(const orc_grid *g, long i, int axis)
{
    if (axis == 0) return i % g->W;
    if (axis == 1) return (i / g->W) % g->H;
    return i / (g->W * g->H);
}

/* number of chains (lines) along an axis and the first voxel of chain c */
static long orc_nchains(const orc_grid *g, int axis)
{
    return g->n / orc_extent(g, axis);
}

static long orc_chain_base(const orc_grid *g, int axis, long c)
{
    if (axis == 0) return c * g->W;                          /* c = d*H + h */
    if (axis == 1) return (c / g->W) * g->H * g->W + c % g->W; /* c = d*W + w */
    return c;                                                 /* c = h*W + w */
}

/* ------------------------------------------------------------------------ */
/* Weighted 1D total-variation prox by the taut string.                      */
/*                                                                            */
/* Sec. 3.2 ("Efficient 1D TV") solves the chain subproblems with the        */
/* taut-string view of the weighted 1D-TV problem                            */
/*     x = argmin_x 1/2 |x - v|^2 + sum_e a_e |x_{e+1} - x_e| .               */
/* With cumulative sums r_k = v_0 + ... + v_{k-1} the solution's cumulative  */
/* sums s_k form the shortest path from (0,0) to (m, r_m) through the tube   */
/* |s_k - r_k| <= a_{k-1} (k = 1..m-1); x_i = s_{i+1} - s_i and the edge     */
/* dual is p_{k-1} = s_k - r_k (so that x = v - D^T p, |p| <= a).            */
/*                                                                            */
/* The path is built segment by segment: from the current anchor, keep the   */
/* steepest slope to a lower tube point and the flattest slope to an upper   */
/* tube point; when they cross, the string bends at the tube point that set  */
/* the violated bound (the last one, on ties), which becomes the new anchor. */
/* Worst case O(m^2), which is fine for a checker.                           */
/*                                                                            */
/* Parity: pinned in tests by KKT, brute force over jump patterns (m <= 8),  */
/* bounded least squares on the dual, and closed forms.                      */
/* ------------------------------------------------------------------------ */
int orc_tv1d(long m, const double *v, const double *a, double *x, double *p)
{
    if (m <= 0 || !v || !x) return ORC_ERR_ARG;
    double *r = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *s = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    if (!r || !s) { free(r); free(s); return ORC_ERR_NOMEM; }
    r[0] = 0.0;
    for (long k = 1; k <= m; ++k) r[k] = r[k - 1] + v[k - 1];

    long k0 = 0;      /* anchor knot */
    double s0 = 0.0;  /* string height at the anchor */
    s[0] = 0.0;
    while (k0 < m) {
        double mu_lo = -INFINITY, mu_hi = INFINITY;
        long j_lo = k0, j_hi = k0;
        int bent = 0;
        for (long j = k0 + 1; j <= m; ++j) {
            double lo, hi;
            if (j == m) {
                lo = hi = r[m];
            } else {
                lo = r[j] - a[j - 1];
                hi = r[j] + a[j - 1];
            }
            double sl = (lo - s0) / (double)(j - k0);
            double sh = (hi - s0) / (double)(j - k0);
            if (sh < mu_lo) {
                /* string must bend down at the last lower touch point */
                for (long i = k0; i < j_lo; ++i) {
                    x[i] = mu_lo;
                    s[i + 1] = s0 + (double)(i + 1 - k0) * mu_lo;
                }
                s[j_lo] = r[j_lo] - a[j_lo - 1];
                s0 = s[j_lo];
                k0 = j_lo;
                bent = 1;
                break;
            }
            if (sl > mu_hi) {
                /* string must bend up at the last upper touch point */
                for (long i = k0; i < j_hi; ++i) {
                    x[i] = mu_hi;
                    s[i + 1] = s0 + (double)(i + 1 - k0) * mu_hi;
                }
                s[j_hi] = r[j_hi] + a[j_hi - 1];
                s0 = s[j_hi];
                k0 = j_hi;
                bent = 1;
                break;
            }
            if (sl >= mu_lo) { mu_lo = sl; j_lo = j; }
            if (sh <= mu_hi) { mu_hi = sh; j_hi = j; }
        }
        if (!bent) {
            /* no bend until the pinned end point (m, r_m) */
            double mu = (r[m] - s0) / (double)(m - k0);
            for (long i = k0; i < m; ++i) {
                x[i] = mu;
                s[i + 1] = s0 + (double)(i + 1 - k0) * mu;
            }
            s[m] = r[m];
            k0 = m;
        }
    }
    if (p) {
        for (long k = 1; k < m; ++k) p[k - 1] = s[k] - r[k];
    }
    free(r);
    free(s);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Cut energy (Sec. 2, eq. (4) with one weight per undirected grid edge).     */
/* Exact for integer and dyadic data.  Parity: hand-computed fixtures.        */
/* ------------------------------------------------------------------------ */
double orc_cut_energy(int ndim, const long *dims, const double *w,
                      const double *const *a, const uint8_t *lab)
{
    orc_grid g;
    if (orc_grid_make(ndim, dims, &g) != ORC_OK) return NAN;
    double e = 0.0;
    for (long i = 0; i < g.n; ++i) {
        if (lab[i]) e += w[i];
        for (int j = 0; j < ndim; ++j) {
            if (orc_coord(&g, i, j) + 1 < orc_extent(&g, j)) {
                long nb = i + orc_stride(&g, j);
                if ((lab[i] != 0) != (lab[nb] != 0)) e += a[j][i];
            }
        }
    }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Brute force over all 2^n labellings (n <= 22).  Returns E*, the number of  */
/* minimisers, their intersection (minimal set) and union (maximal set).      */
/* ------------------------------------------------------------------------ */
double orc_bruteforce(int ndim, const long *dims, const double *w,
                      const double *const *a, uint8_t *min_set,
                      uint8_t *max_set, long *count)
{
    orc_grid g;
    if (orc_grid_make(ndim, dims, &g) != ORC_OK || g.n > 22) return NAN;
    long n = g.n;
    uint8_t *lab = (uint8_t *)calloc((size_t)n, 1);
    double best = INFINITY;
    long cnt = 0;
    for (long i = 0; i < n; ++i) { min_set[i] = 1; max_set[i] = 0; }
    for (uint64_t mask = 0; mask < (1ull << n); ++mask) {
        for (long i = 0; i < n; ++i) lab[i] = (uint8_t)((mask >> i) & 1u);
        double e = orc_cut_energy(ndim, dims, w, a, lab);
        if (e < best) {
            best = e;
            cnt = 0;
            for (long i = 0; i < n; ++i) { min_set[i] = 1; max_set[i] = 0; }
        }
        if (e == best) {
            ++cnt;
            for (long i = 0; i < n; ++i) {
                min_set[i] = (uint8_t)(min_set[i] && lab[i]);
                max_set[i] = (uint8_t)(max_set[i] || lab[i]);
            }
        }
    }
    free(lab);
    if (count) *count = cnt;
    return best;
}

/* ------------------------------------------------------------------------ */
/* s-t max-flow on the grid graph (the traditional min-cut/max-flow view the  */
/* paper's certificate corresponds to, Sec. 2.2).                             */
/*   w_i > 0: arc i -> t, capacity w_i;  w_i < 0: arc s -> i, capacity -w_i;  */
/*   each grid edge: arcs i -> j and j -> i, capacity a_e.                    */
/*   E* = maxflow + sum_i min(w_i, 0).                                        */
/* Minimal optimal set = nodes reachable from s in the residual graph;        */
/* maximal optimal set = nodes that cannot reach t.                           */
/* ------------------------------------------------------------------------ */
typedef struct {
    long nv, na, cap_arcs;
    long *head;   /* first arc of each vertex, -1 terminated lists */
    long *next;
    long *to;
    double *cap;  /* residual capacity; arc k and k^1 are a pair */
} orc_graph;

static int orc_graph_init(orc_graph *G, long nv, long max_arcs)
{
    G->nv = nv; G->na = 0; G->cap_arcs = max_arcs;
    G->head = (long *)malloc(sizeof(long) * (size_t)nv);
    G->next = (long *)malloc(sizeof(long) * (size_t)max_arcs);
    G->to = (long *)malloc(sizeof(long) * (size_t)max_arcs);
    G->cap = (double *)malloc(sizeof(double) * (size_t)max_arcs);
    if (!G->head || !G->next || !G->to || !G->cap) return ORC_ERR_NOMEM;
    for (long i = 0; i < nv; ++i) G->head[i] = -1;
    return ORC_OK;
}

static void orc_graph_free(orc_graph *G)
{
    free(G->head); free(G->next); free(G->to); free(G->cap);
}

/* one pair of arcs u->v (capacity c_uv) and v->u (capacity c_vu) */
static void orc_add_pair(orc_graph *G, long u, long v, double c_uv, double c_vu)
{
    long k = G->na;
    G->to[k] = v; G->cap[k] = c_uv; G->next[k] = G->head[u]; G->head[u] = k;
    G->to[k + 1] = u; G->cap[k + 1] = c_vu; G->next[k + 1] = G->head[v]; G->head[v] = k + 1;
    G->na += 2;
}

static int orc_build_grid_graph(const orc_grid *g, const double *w,
                                const double *const *a, orc_graph *G)
{
    long n = g->n;
    long max_arcs = 2 * (n + (long)g->ndim * n);
    if (orc_graph_init(G, n + 2, max_arcs) != ORC_OK) return ORC_ERR_NOMEM;
    long s = n, t = n + 1;
    for (long i = 0; i < n; ++i) {
        if (w[i] > 0) orc_add_pair(G, i, t, w[i], 0.0);
        else if (w[i] < 0) orc_add_pair(G, s, i, -w[i], 0.0);
    }
    for (long i = 0; i < n; ++i) {
        for (int j = 0; j < g->ndim; ++j) {
            if (orc_coord(g, i, j) + 1 < orc_extent(g, j)) {
                double c = a[j][i];
                if (c > 0) orc_add_pair(G, i, i + orc_stride(g, j), c, c);
            }
        }
    }
    return ORC_OK;
}

/* Edmonds-Karp: repeatedly augment along a BFS-shortest residual path. */
static double orc_maxflow_ek(orc_graph *G, long s, long t)
{
    long nv = G->nv;
    long *pred_arc = (long *)malloc(sizeof(long) * (size_t)nv);
    long *queue = (long *)malloc(sizeof(long) * (size_t)nv);
    double flow = 0.0;
    for (;;) {
        for (long i = 0; i < nv; ++i) pred_arc[i] = -2;
        pred_arc[s] = -1;
        long qh = 0, qt = 0;
        queue[qt++] = s;
        while (qh < qt && pred_arc[t] == -2) {
            long u = queue[qh++];
            for (long k = G->head[u]; k >= 0; k = G->next[k]) {
                long v = G->to[k];
                if (G->cap[k] > 0 && pred_arc[v] == -2) {
                    pred_arc[v] = k;
                    queue[qt++] = v;
                }
            }
        }
        if (pred_arc[t] == -2) break;
        double b = INFINITY;
        for (long v = t; v != s; v = G->to[pred_arc[v] ^ 1]) {
            double c = G->cap[pred_arc[v]];
            if (c < b) b = c;
        }
        for (long v = t; v != s; v = G->to[pred_arc[v] ^ 1]) {
            G->cap[pred_arc[v]] -= b;
            G->cap[pred_arc[v] ^ 1] += b;
        }
        flow += b;
    }
    free(pred_arc);
    free(queue);
    return flow;
}

/* Dinic: BFS level graph, then blocking flow by (iterative) DFS with
 * current-arc pointers. */
static double orc_maxflow_dinic(orc_graph *G, long s, long t)
{
    long nv = G->nv;
    long *level = (long *)malloc(sizeof(long) * (size_t)nv);
    long *cur = (long *)malloc(sizeof(long) * (size_t)nv);
    long *queue = (long *)malloc(sizeof(long) * (size_t)nv);
    long *stack_arc = (long *)malloc(sizeof(long) * (size_t)nv);
    double flow = 0.0;
    for (;;) {
        for (long i = 0; i < nv; ++i) level[i] = -1;
        level[s] = 0;
        long qh = 0, qt = 0;
        queue[qt++] = s;
        while (qh < qt) {
            long u = queue[qh++];
            for (long k = G->head[u]; k >= 0; k = G->next[k]) {
                long v = G->to[k];
                if (G->cap[k] > 0 && level[v] < 0) {
                    level[v] = level[u] + 1;
                    queue[qt++] = v;
                }
            }
        }
        if (level[t] < 0) break;
        for (long i = 0; i < nv; ++i) cur[i] = G->head[i];
        /* iterative DFS: stack_arc[d] is the arc taken at depth d */
        long depth = 0;
        long u = s;
        for (;;) {
            if (u == t) {
                double b = INFINITY;
                for (long d = 0; d < depth; ++d)
                    if (G->cap[stack_arc[d]] < b) b = G->cap[stack_arc[d]];
                for (long d = 0; d < depth; ++d) {
                    G->cap[stack_arc[d]] -= b;
                    G->cap[stack_arc[d] ^ 1] += b;
                }
                flow += b;
                /* restart from the source; saturated arcs are skipped below */
                depth = 0;
                u = s;
                continue;
            }
            long k = cur[u];
            while (k >= 0 && !(G->cap[k] > 0 && level[G->to[k]] == level[u] + 1))
                k = G->next[k];
            cur[u] = k;
            if (k >= 0) {
                stack_arc[depth++] = k;
                u = G->to[k];
            } else {
                /* dead end: retreat and drop the arc that led here */
                if (depth == 0) break;
                level[u] = -1;
                --depth;
                u = G->to[stack_arc[depth] ^ 1];
                cur[u] = G->next[cur[u]];
            }
        }
    }
    free(level); free(cur); free(queue); free(stack_arc);
    return flow;
}

/* method: 0 = Edmonds-Karp, 1 = Dinic.  Returns E* (NaN on error). */
double orc_mincut(int method, int ndim, const long *dims, const double *w,
                  const double *const *a, uint8_t *min_set, uint8_t *max_set,
                  double *flow_out)
{
    orc_grid g;
    if (orc_grid_make(ndim, dims, &g) != ORC_OK) return NAN;
    orc_graph G;
    if (orc_build_grid_graph(&g, w, a, &G) != ORC_OK) { orc_graph_free(&G); return NAN; }
    long s = g.n, t = g.n + 1;
    double flow = method == 0 ? orc_maxflow_ek(&G, s, t) : orc_maxflow_dinic(&G, s, t);
    double base = 0.0;
    for (long i = 0; i < g.n; ++i) if (w[i] < 0) base += w[i];

    long nv = G.nv;
    long *queue = (long *)malloc(sizeof(long) * (size_t)nv);
    uint8_t *seen = (uint8_t *)calloc((size_t)nv, 1);
    if (min_set) {
        long qh = 0, qt = 0;
        queue[qt++] = s; seen[s] = 1;
        while (qh < qt) {
            long u = queue[qh++];
            for (long k = G.head[u]; k >= 0; k = G.next[k]) {
                long v = G.to[k];
                if (G.cap[k] > 0 && !seen[v]) { seen[v] = 1; queue[qt++] = v; }
            }
        }
        for (long i = 0; i < g.n; ++i) min_set[i] = seen[i];
    }
    if (max_set) {
        memset(seen, 0, (size_t)nv);
        long qh = 0, qt = 0;
        queue[qt++] = t; seen[t] = 1;
        while (qh < qt) {
            long v = queue[qh++];
            /* u can reach v if the residual arc u->v (the pair of v->u) has capacity */
            for (long k = G.head[v]; k >= 0; k = G.next[k]) {
                long u = G.to[k];
                if (G.cap[k ^ 1] > 0 && !seen[u]) { seen[u] = 1; queue[qt++] = u; }
            }
        }
        for (long i = 0; i < g.n; ++i) max_set[i] = (uint8_t)!seen[i];
    }
    free(queue);
    free(seen);
    orc_graph_free(&G);
    if (flow_out) *flow_out = flow;
    return flow + base;
}

/* ------------------------------------------------------------------------ */
/* Projection onto K_j for one chain family (Sec. 3.3; Moreau: Pi_K(v) =      */
/* v - prox(v), with the dual x = w - y of Sec. 2.3 applied per chain).       */
/* y receives Pi_{K_j}(v), p the edge duals (p[i] for edge (i, i+stride)).    */
/* ------------------------------------------------------------------------ */
static int orc_project_family(const orc_grid *g, int axis, const double *a_axis,
                              const double *v, double *y, double *p)
{
    long L = orc_extent(g, axis), st = orc_stride(g, axis);
    long nc = orc_nchains(g, axis);
    int rc = ORC_OK;
#pragma omp parallel
    {
        /* one set of chain buffers per thread */
        double *cv = (double *)malloc(sizeof(double) * (size_t)L);
        double *ca = (double *)malloc(sizeof(double) * (size_t)(L > 1 ? L - 1 : 1));
        double *cx = (double *)malloc(sizeof(double) * (size_t)L);
        double *cp = (double *)malloc(sizeof(double) * (size_t)(L > 1 ? L - 1 : 1));
        int ok = cv && ca && cx && cp;
        if (!ok) {
#pragma omp atomic write
            rc = ORC_ERR_NOMEM;
        }
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            if (!ok) continue;
            long b = orc_chain_base(g, axis, c);
            for (long k = 0; k < L; ++k) cv[k] = v[b + k * st];
            for (long k = 0; k + 1 < L; ++k) ca[k] = a_axis[b + k * st];
            orc_tv1d(L, cv, ca, cx, cp);
            for (long k = 0; k < L; ++k) y[b + k * st] = cv[k] - cx[k];
            if (p) {
                for (long k = 0; k + 1 < L; ++k) p[b + k * st] = cp[k];
                p[b + (L - 1) * st] = 0.0;
            }
        }
        free(cv); free(ca); free(cx); free(cp);
    }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Certificate of Sec. 2.2: for y in K and any S,                             */
/*   E(S) >= sum_{i in S} (y_i + w_i) >= LB(y) = sum_i min(y_i + w_i, 0).     */
/* y is rebuilt from edge duals clipped to [-a, a], so it lies in K exactly.  */
/* Also returns the TV duality gap sum_e (a_e |Dx_e| - p_e Dx_e) at           */
/* x = u - y, a non-negative diagnostic (eq. (TV) against its dual).          */
/* ------------------------------------------------------------------------ */
static void orc_certificate(const orc_grid *g, const double *w,
                            const double *const *a, double *const *p,
                            double *lb_out, double *tvgap_out)
{
    long n = g->n;
    double *y = (double *)calloc((size_t)n, sizeof(double));
    for (int j = 0; j < g->ndim; ++j) {
        long st = orc_stride(g, j), L = orc_extent(g, j);
        for (long i = 0; i < n; ++i) {
            if (orc_coord(g, i, j) + 1 < L) {
                double pe = p[j][i], ae = a[j][i];
                if (pe > ae) pe = ae;
                if (pe < -ae) pe = -ae;
                /* (D^T p)_i = p_{i-1} - p_i along the chain */
                y[i] -= pe;
                y[i + st] += pe;
            }
        }
    }
    double lb = 0.0;
    for (long i = 0; i < n; ++i) {
        double t = y[i] + w[i];
        if (t < 0) lb += t;
    }
    double gap = 0.0;
    for (int j = 0; j < g->ndim; ++j) {
        long st = orc_stride(g, j), L = orc_extent(g, j);
        for (long i = 0; i < n; ++i) {
            if (orc_coord(g, i, j) + 1 < L) {
                double pe = p[j][i], ae = a[j][i];
                if (pe > ae) pe = ae;
                if (pe < -ae) pe = -ae;
                double x0 = -w[i] - y[i], x1 = -w[i + st] - y[i + st];
                double dx = x1 - x0;
                gap += ae * fabs(dx) - pe * dx;
            }
        }
    }
    free(y);
    *lb_out = lb;
    if (tvgap_out) *tvgap_out = gap;
}

/* ------------------------------------------------------------------------ */
/* Douglas-Rachford / averaged alternating reflections (Sec. 4.3, eq. (3)).  */
/*                                                                            */
/* variant 0 (2D only, r = 2, Sec. 3.3 "Special case r = 2"): the distance    */
/*   between A = K_1 (rows) and B = {u - y_2 : y_2 in K_2} (columns);         */
/*   z <- 1/2 (z + R_B R_A z), R = 2 Pi - I, Pi_B(v) = u - Pi_{K_2}(u - v);   */
/*   shadow y_1 = Pi_A(z), y_2 from Pi_B; state z has n entries.              */
/* variant 1 (product space, any r = ndim, Sec. 3.3 first dual and eq.        */
/*   (dualA)): z = (z_1..z_r), Pi_K acts per family, Pi_L(v)_j = v_j +        */
/*   (u - sum_k v_k)/r; z <- 1/2 (z + R_L R_K z); state has r*n entries.      */
/* In both, the primal estimate is x = u - sum_j y_j (Sec. 2.3: x = w - y).   */
/*                                                                            */
/* Rounding readout (reading of Sec. 2.1's level sets and Sec. 2.3's         */
/* threshold at 0 for an approximate x): S_tau = {x > tau} for the ladder    */
/* tau = +tau0, +tau0/10, +tau0/100, +tau0/1000, 0, -tau0/1000, ..., -tau0;  */
/* the first of minimal energy is kept; cert = E(S) - LB(y).                 */
/* Stop when (gap_tol <= 0 or cert < gap_tol) and (tv_tol <= 0 or           */
/* tvgap < tv_tol), with at least one of them positive; else run max_iters. */
/* ------------------------------------------------------------------------ */
#define ORC_NTAU 9

/* thresholds tau0 * (1, 1e-1, 1e-2, 1e-3, 0, -1e-3, -1e-2, -1e-1, -1) */
void orc_tau_ladder(double tau0, double *taus)
{
    const double f[ORC_NTAU] = {1.0, 1e-1, 1e-2, 1e-3, 0.0, -1e-3, -1e-2, -1e-1, -1.0};
    for (int t = 0; t < ORC_NTAU; ++t) taus[t] = tau0 * f[t];
}

typedef struct {
    int32_t iters;
    int32_t status;   /* 0 converged, 1 max_iters reached */
    double cert;
    double energy;
    double lower_bound;
    double tv_gap;
    double tau_used;
} orc_stats;

int orc_dr_solve(int ndim, const long *dims, const double *w,
                 const double *const *a, int variant, int max_iters,
                 double gap_tol, double tv_tol, double tau0,
                 const double *z0, double *x_out, uint8_t *labels_out,
                 double *z_out, double *cert_hist, double *tvgap_hist,
                 orc_stats *st)
{
    orc_grid g;
    if (orc_grid_make(ndim, dims, &g) != ORC_OK) return ORC_ERR_ARG;
    if (variant == 0 && ndim != 2) return ORC_ERR_ARG;
    long n = g.n;
    int r = ndim;
    long nz = variant == 0 ? n : (long)r * n;

    double *u = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)calloc((size_t)nz, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * (size_t)r * (size_t)n);
    double *pd = (double *)malloc(sizeof(double) * (size_t)r * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)nz);
    double *tmp2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    uint8_t *best_lab = (uint8_t *)malloc((size_t)n);
    if (!u || !z || !y || !pd || !tmp || !tmp2 || !x || !best_lab) return ORC_ERR_NOMEM;
    for (long i = 0; i < n; ++i) u[i] = -w[i];
    if (z0) memcpy(z, z0, sizeof(double) * (size_t)nz);
    double *pj[3] = {pd, pd + n, pd + 2 * n};
    double taus[ORC_NTAU];
    orc_tau_ladder(tau0, taus);

    int it = 0, done = 0;
    double cert = INFINITY, energy = INFINITY, lb = -INFINITY, tvgap = INFINITY, tau_used = 0;
    while (it < max_iters && !done) {
        ++it;
        if (variant == 0) {
            double *y1 = y, *y2 = y + n;
            orc_project_family(&g, 0, a[0], z, y1, pj[0]);            /* Pi_A(z) */
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) tmp[i] = 2.0 * y1[i] - z[i]; /* R_A z */
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) tmp2[i] = u[i] - tmp[i];
            orc_project_family(&g, 1, a[1], tmp2, y2, pj[1]);         /* Pi_{K2}(u - R_A z) */
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                double pib = u[i] - y2[i];                             /* Pi_B(R_A z) */
                double rb = 2.0 * pib - tmp[i];                        /* R_B R_A z */
                z[i] = 0.5 * (z[i] + rb);
                x[i] = u[i] - y1[i] - y2[i];
            }
        } else {
            for (int j = 0; j < r; ++j)
                orc_project_family(&g, j, a[j], z + (long)j * n, y + (long)j * n, pj[j]);
#pragma omp parallel for schedule(static)
            for (long i = 0; i < n; ++i) {
                double srk = 0.0;
                for (int j = 0; j < r; ++j) {
                    double rk = 2.0 * y[(long)j * n + i] - z[(long)j * n + i]; /* R_K z */
                    tmp[(long)j * n + i] = rk;
                    srk += rk;
                }
                double ysum = 0.0;
                for (int j = 0; j < r; ++j) {
                    double rk = tmp[(long)j * n + i];
                    double pl = rk + (u[i] - srk) / (double)r;          /* Pi_L(R_K z) */
                    double rl = 2.0 * pl - rk;                          /* R_L R_K z */
                    z[(long)j * n + i] = 0.5 * (z[(long)j * n + i] + rl);
                    ysum += y[(long)j * n + i];
                }
                x[i] = u[i] - ysum;
            }
        }
        orc_certificate(&g, w, a, pj, &lb, &tvgap);
        /* E(S_t) for every threshold (independent), then the first of least energy */
        double e_t[ORC_NTAU];
#pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < ORC_NTAU; ++t) {
            uint8_t *lt = (uint8_t *)malloc((size_t)n);
            if (!lt) { e_t[t] = NAN; continue; }
            for (long i = 0; i < n; ++i) lt[i] = (uint8_t)(x[i] > taus[t]);
            e_t[t] = orc_cut_energy(ndim, dims, w, a, lt);
            free(lt);
        }
        energy = INFINITY;
        int t_best = 0;
        for (int t = 0; t < ORC_NTAU; ++t) {
            if (e_t[t] < energy) {
                energy = e_t[t];
                tau_used = taus[t];
                t_best = t;
            }
        }
        for (long i = 0; i < n; ++i) best_lab[i] = (uint8_t)(x[i] > taus[t_best]);
        cert = energy - lb;
        if (cert_hist) cert_hist[it - 1] = cert;
        if (tvgap_hist) tvgap_hist[it - 1] = tvgap;
        int ok_cert = gap_tol <= 0 || cert < gap_tol;
        int ok_tv = tv_tol <= 0 || tvgap < tv_tol;
        if ((gap_tol > 0 || tv_tol > 0) && ok_cert && ok_tv) done = 1;
    }
    if (x_out) memcpy(x_out, x, sizeof(double) * (size_t)n);
    if (labels_out) memcpy(labels_out, best_lab, (size_t)n);
    if (z_out) memcpy(z_out, z, sizeof(double) * (size_t)nz);
    if (st) {
        st->iters = it;
        st->status = done ? 0 : 1;
        st->cert = cert;
        st->energy = energy;
        st->lower_bound = lb;
        st->tv_gap = tvgap;
        st->tau_used = tau_used;
    }
    free(u); free(z); free(y); free(pd); free(tmp); free(tmp2); free(x);
    free(best_lab);
    return ORC_OK;
}

#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads of the OpenMP build (no effect in the plain build); returns the
 * number the next parallel region will use. */
int orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
    return omp_get_max_threads();
#else
    (void)k;
    return 1;
#endif
}

/* Projection onto one family, exposed for tests (x = prox, p = edge duals). */
int orc_prox_family(int ndim, const long *dims, int axis, const double *v,
                    const double *a_axis, double *x, double *p)
{
    orc_grid g;
    if (orc_grid_make(ndim, dims, &g) != ORC_OK || axis < 0 || axis >= ndim) return ORC_ERR_ARG;
    double *y = (double *)malloc(sizeof(double) * (size_t)g.n);
    if (!y) return ORC_ERR_NOMEM;
    int rc = orc_project_family(&g, axis, a_axis, v, y, p);
    for (long i = 0; i < g.n; ++i) x[i] = v[i] - y[i];
    free(y);
    return rc;
}

/* Lower bound LB(y) and TV gap from given edge duals, exposed for tests. */
int orc_lower_bound(int ndim, const long *dims, const double *w,
                    const double *const *a, double *const *p, double *lb,
                    double *tvgap)
{
    orc_grid g;
    if (orc_grid_make(ndim, dims, &g) != ORC_OK) return ORC_ERR_ARG;
    orc_certificate(&g, w, a, p, lb, tvgap);
    return ORC_OK;
}
