/*
 * ORACLE — test infrastructure only.  Nothing in the product library links, loads or calls this file;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg do.
 *
 * Plain CPU solvers for one binary sub-problem of DOPE:
 *
 *     minimise  F(x) = sum_i un_i x_i + sum_e cap_e |x_a(e) - x_b(e)|   over x in {0,1}^n
 *
 * which is the block problem of the paper's Eq. (8) once the unary vector and the block pairwise weights of
 * Theorem 1 are fixed (label 1 = foreground).  Two solvers:
 *
 *   oracle_mincut      s-t max-flow by Dinic's blocking-flow algorithm (textbook form: BFS level graph,
 *                      then augmenting DFS along level-increasing residual arcs).  Source arc s->i carries
 *                      max(-un_i, 0), sink arc i->t carries max(un_i, 0), every edge is a pair of arcs of
 *                      capacity cap_e.  With label 1 = source side, cut(x) = F(x) + sum_i max(-un_i, 0).
 *                      Returned labelling: the nodes reachable from s in the final residual graph, i.e. the
 *                      minimal source set, which is the unique minimiser contained in every other one.
 *                      Requires cap_e >= 0 (the submodularity condition of the footnote in Sec. 1).
 *   oracle_enumerate   all 2^n labellings in increasing code order (bit p of the code = node p); keeps the
 *                      first strict minimum, i.e. the smallest-code minimiser.  Any sign of cap_e.
 *
 * Both are thread-safe (per-call allocation) so the Python driver may run blocks concurrently.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n_nodes;
    int *start;      /* CSR row start, size n_nodes + 1 */
    int *to;         /* arc head */
    int *rev;        /* index of the reverse arc */
    int64_t *res;    /* residual capacity */
} graph_t;

/* Build the s-t graph.  s = n, t = n + 1.  Returns 0 on success. */
static int build_graph(graph_t *g, int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb,
                       const int64_t *cap) {
    int N = n + 2, s = n, t = n + 1;
    int *deg = (int *)calloc((size_t)N, sizeof(int));
    if (!deg) return -1;
    for (int i = 0; i < n; ++i) {
        if (un[i] < 0) { deg[s]++; deg[i]++; }
        if (un[i] > 0) { deg[i]++; deg[t]++; }
    }
    for (int e = 0; e < m; ++e) { deg[ea[e]]++; deg[eb[e]]++; }
    g->n_nodes = N;
    g->start = (int *)malloc(sizeof(int) * (size_t)(N + 1));
    int total = 0;
    for (int v = 0; v < N; ++v) total += deg[v];
    g->to = (int *)malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
    g->rev = (int *)malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
    g->res = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    int *fill = (int *)malloc(sizeof(int) * (size_t)N);
    if (!g->start || !g->to || !g->rev || !g->res || !fill) { free(deg); free(fill); return -1; }
    g->start[0] = 0;
    for (int v = 0; v < N; ++v) g->start[v + 1] = g->start[v] + deg[v];
    for (int v = 0; v < N; ++v) fill[v] = g->start[v];
#define ADD_PAIR(a, b, cab, cba)                                      \
    do {                                                              \
        int ia = fill[(a)]++, ib = fill[(b)]++;                       \
        g->to[ia] = (b); g->rev[ia] = ib; g->res[ia] = (cab);         \
        g->to[ib] = (a); g->rev[ib] = ia; g->res[ib] = (cba);         \
    } while (0)
    for (int i = 0; i < n; ++i) {
        if (un[i] < 0) ADD_PAIR(s, i, -un[i], 0);
        if (un[i] > 0) ADD_PAIR(i, t, un[i], 0);
    }
    for (int e = 0; e < m; ++e) ADD_PAIR(ea[e], eb[e], cap[e], cap[e]);
#undef ADD_PAIR
    free(deg);
    free(fill);
    return 0;
}

static void free_graph(graph_t *g) {
    free(g->start); free(g->to); free(g->rev); free(g->res);
}

/* BFS from s over arcs with positive residual; level[v] = -1 if unreached.  Returns level[t] >= 0. */
static int bfs_levels(const graph_t *g, int s, int t, int *level, int *queue) {
    for (int v = 0; v < g->n_nodes; ++v) level[v] = -1;
    int head = 0, tail = 0;
    level[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int v = queue[head++];
        for (int a = g->start[v]; a < g->start[v + 1]; ++a) {
            int w = g->to[a];
            if (g->res[a] > 0 && level[w] < 0) {
                level[w] = level[v] + 1;
                queue[tail++] = w;
            }
        }
    }
    return level[t] >= 0;
}

/* Dinic max-flow; returns the flow value, or -1 on allocation failure. */
static int64_t dinic(graph_t *g, int s, int t) {
    int N = g->n_nodes;
    int *level = (int *)malloc(sizeof(int) * (size_t)N);
    int *queue = (int *)malloc(sizeof(int) * (size_t)N);
    int *it = (int *)malloc(sizeof(int) * (size_t)N);
    int *path_arc = (int *)malloc(sizeof(int) * (size_t)N);
    int *path_node = (int *)malloc(sizeof(int) * (size_t)N);
    if (!level || !queue || !it || !path_arc || !path_node) {
        free(level); free(queue); free(it); free(path_arc); free(path_node);
        return -1;
    }
    int64_t total = 0;
    while (bfs_levels(g, s, t, level, queue)) {
        for (int v = 0; v < N; ++v) it[v] = g->start[v];
        for (;;) {
            /* search one level-increasing path s -> t, pruning dead ends */
            int top = 0, v = s;
            while (v != t) {
                int found = -1;
                for (; it[v] < g->start[v + 1]; ++it[v]) {
                    int a = it[v];
                    if (g->res[a] > 0 && level[g->to[a]] == level[v] + 1) { found = a; break; }
                }
                if (found >= 0) {
                    path_node[top] = v;
                    path_arc[top] = found;
                    ++top;
                    v = g->to[found];
                } else {
                    level[v] = -1;           /* dead end for this phase */
                    if (top == 0) break;
                    --top;
                    v = path_node[top];
                    ++it[v];
                }
            }
            if (v != t) break;                /* no more paths in this level graph */
            int64_t b = INT64_MAX;
            for (int k = 0; k < top; ++k) if (g->res[path_arc[k]] < b) b = g->res[path_arc[k]];
            for (int k = 0; k < top; ++k) {
                g->res[path_arc[k]] -= b;
                g->res[g->rev[path_arc[k]]] += b;
            }
            total += b;
        }
    }
    free(level); free(queue); free(it); free(path_arc); free(path_node);
    return total;
}

int oracle_mincut(int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb, const int64_t *cap,
                  uint8_t *x, int64_t *flow_out) {
    for (int e = 0; e < m; ++e) if (cap[e] < 0) return -4;   /* not submodular */
    graph_t g;
    memset(&g, 0, sizeof(g));
    if (build_graph(&g, n, un, m, ea, eb, cap) != 0) { free_graph(&g); return -2; }
    int s = n, t = n + 1;
    int64_t f = dinic(&g, s, t);
    if (f < 0) { free_graph(&g); return -2; }
    /* minimal source set: reachable from s in the residual graph */
    int *level = (int *)malloc(sizeof(int) * (size_t)g.n_nodes);
    int *queue = (int *)malloc(sizeof(int) * (size_t)g.n_nodes);
    if (!level || !queue) { free(level); free(queue); free_graph(&g); return -2; }
    bfs_levels(&g, s, t, level, queue);
    for (int i = 0; i < n; ++i) x[i] = (uint8_t)(level[i] >= 0);
    if (flow_out) *flow_out = f;
    free(level); free(queue);
    free_graph(&g);
    return 0;
}

int oracle_enumerate(int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb, const int64_t *cap,
                     uint8_t *x, int64_t *emin_out) {
    if (n < 0 || n > 24) return -1;
    int64_t best = INT64_MAX;
    uint32_t best_code = 0;
    uint32_t ncodes = 1u << n;
    for (uint32_t code = 0; code < ncodes; ++code) {
        int64_t e = 0;
        for (int i = 0; i < n; ++i) if ((code >> i) & 1u) e += un[i];
        for (int k = 0; k < m; ++k) {
            uint32_t a = (code >> ea[k]) & 1u, b = (code >> eb[k]) & 1u;
            if (a != b) e += cap[k];
        }
        if (e < best) { best = e; best_code = code; }
    }
    for (int i = 0; i < n; ++i) x[i] = (uint8_t)((best_code >> i) & 1u);
    if (emin_out) *emin_out = best;
    return 0;
}

/* Energy of a given labelling under the same objective (used for duality checks). */
int64_t oracle_objective(int n, const int64_t *un, int m, const int32_t *ea, const int32_t *eb,
                         const int64_t *cap, const uint8_t *x) {
    int64_t e = 0;
    for (int i = 0; i < n; ++i) if (x[i]) e += un[i];
    for (int k = 0; k < m; ++k) if (x[ea[k]] != x[eb[k]]) e += cap[k];
    return e;
}
