/*
 * CPU oracle for exact max-flow / minimum s-t cut on image grid graphs.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP path and the product never calls it.
 *
 * What it computes (Sec. 2 of the paper): for a grid whose pixels are linked to
 * a source s and a sink t (data terms) and to their 4 or 8 neighbours
 * (smoothness terms), the value F of a maximum s-t flow, which by the
 * Ford-Fulkerson theorem equals the minimum cut cost, and the minimum cut
 * itself.  Because several cuts can be optimal, the cut reported is the
 * inclusion-minimal source side S_min: the pixels reachable from s in the
 * residual graph of a maximum flow (every maximum flow gives the same set).
 *
 * Two independent algorithms, both in 64-bit integers:
 *   - oracle_fifo_pr: Goldberg-Tarjan push-relabel with FIFO selection of
 *     active vertices and periodic exact relabelling by breadth-first search
 *     (first from t, then from s), run until no vertex other than s, t holds
 *     excess, i.e. to a genuine maximum flow.  Built on a CSR arc list.
 *   - oracle_ek: Edmonds-Karp (shortest augmenting paths by BFS), working on
 *     per-direction residual planes of the grid, with no arc list.
 * Both finish with a BFS from s over arcs of positive residual capacity.
 *
 * Capacities of a pixel p at parameter value lambda (the monotone parametric
 * case of Sec. 2.1, seeds frozen to a label as in Sec. 2.1):
 *   seed[p] == 1 (foreground): cs = INF, ct = 0
 *   seed[p] == 2 (background): cs = 0,   ct = INF
 *   seed[p] == 0 (free):       cs = cap_src[p], ct = cap_snk0[p] + slope[p]*lambda
 * with INF = 2^30.  nlink[k*n + p] is the capacity of the arc p -> p + d_k.
 *
 * A rational parameter value lambda = num / den (den >= 1) is solved on the
 * network with every capacity multiplied by den (INF included): there the
 * sink capacity of a free pixel is cap_snk0*den + slope*num, an integer.
 * Scaling all capacities by den scales every cut by den, so the minimum cuts
 * are the same sets and the flow value is den * F(num / den)
 * (oracle_fifo_pr_rational).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_INF ((int64_t)1 << 30)

static const int ODX[8] = {1, -1, 0, 0, 1, -1, -1, 1};
static const int ODY[8] = {0, 0, 1, -1, 1, -1, 1, -1};

typedef struct {
    int W, H, K;
    const int32_t *nlink, *cap_src, *cap_snk0, *slope;
    const uint8_t *seed;
    int64_t den; /* every capacity is multiplied by den; lambda is then the numerator */
} orc_grid;

static void terminal_caps(const orc_grid *g, int64_t lambda, int p, int64_t *cs, int64_t *ct) {
    uint8_t s = g->seed[p];
    if (s == 1) {
        *cs = ORC_INF * g->den;
        *ct = 0;
    } else if (s == 2) {
        *cs = 0;
        *ct = ORC_INF * g->den;
    } else {
        *cs = (int64_t)g->cap_src[p] * g->den;
        *ct = (int64_t)g->cap_snk0[p] * g->den + (int64_t)g->slope[p] * lambda;
    }
}

static int neighbour(const orc_grid *g, int p, int k) {
    int x = p % g->W, y = p / g->W;
    int qx = x + ODX[k], qy = y + ODY[k];
    if (qx < 0 || qy < 0 || qx >= g->W || qy >= g->H) return -1;
    return qy * g->W + qx;
}

/* ------------------------------------------------------------------------ */
/* CSR residual graph: arc a goes tail -> head[a]; rev[a] is its partner.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    int N;        /* vertices: pixels 0..n-1, s = n, t = n+1 */
    int M;        /* arcs */
    int *first;   /* [N+1] */
    int *head;    /* [M] */
    int *rev;     /* [M] */
    int64_t *res; /* [M] */
} orc_graph;

static void graph_free(orc_graph *G) {
    free(G->first);
    free(G->head);
    free(G->rev);
    free(G->res);
}

static int graph_build(const orc_grid *g, int64_t lambda, orc_graph *G) {
    int n = g->W * g->H, N = n + 2, s = n, t = n + 1;
    int *deg = (int *)calloc((size_t)N, sizeof(int));
    if (!deg) return -1;
    /* every unordered neighbour pair once (even directions), plus s->p, p->t */
    for (int p = 0; p < n; ++p) {
        for (int k = 0; k < g->K; k += 2) {
            int q = neighbour(g, p, k);
            if (q < 0) continue;
            deg[p]++;
            deg[q]++;
        }
        deg[p] += 2;
        deg[s]++;
        deg[t]++;
    }
    G->N = N;
    G->first = (int *)malloc(sizeof(int) * (size_t)(N + 1));
    G->first[0] = 0;
    for (int v = 0; v < N; ++v) G->first[v + 1] = G->first[v] + deg[v];
    G->M = G->first[N];
    G->head = (int *)malloc(sizeof(int) * (size_t)G->M);
    G->rev = (int *)malloc(sizeof(int) * (size_t)G->M);
    G->res = (int64_t *)malloc(sizeof(int64_t) * (size_t)G->M);
    int *fill = (int *)malloc(sizeof(int) * (size_t)N);
    if (!G->head || !G->rev || !G->res || !fill) {
        free(deg);
        free(fill);
        return -1;
    }
    memcpy(fill, G->first, sizeof(int) * (size_t)N);
#define ADD_PAIR(u, v, cuv, cvu)                                         \
    do {                                                                 \
        int a_ = fill[u]++, b_ = fill[v]++;                              \
        G->head[a_] = (v); G->rev[a_] = b_; G->res[a_] = (cuv);          \
        G->head[b_] = (u); G->rev[b_] = a_; G->res[b_] = (cvu);          \
    } while (0)
    for (int p = 0; p < n; ++p) {
        for (int k = 0; k < g->K; k += 2) {
            int q = neighbour(g, p, k);
            if (q < 0) continue;
            /* opposite of direction k is k^1 */
            ADD_PAIR(p, q, (int64_t)g->nlink[(size_t)k * n + p] * g->den,
                     (int64_t)g->nlink[(size_t)(k ^ 1) * n + q] * g->den);
        }
        int64_t cs, ct;
        terminal_caps(g, lambda, p, &cs, &ct);
        ADD_PAIR(s, p, cs, 0);
        ADD_PAIR(p, t, ct, 0);
    }
#undef ADD_PAIR
    free(fill);
    free(deg);
    return 0;
}

/* Exact distance labels: d = BFS distance to t in the residual graph; vertices
 * that cannot reach t get N + distance to s; the rest 2N.  These labels are
 * valid (d(u) <= d(v) + 1 for every residual arc u->v). */
static void global_relabel(const orc_graph *G, int s, int t, int *d, int *queue) {
    int N = G->N;
    for (int v = 0; v < N; ++v) d[v] = 2 * N;
    int roots[2] = {t, s};
    int base[2] = {0, N};
    for (int r = 0; r < 2; ++r) {
        int qh = 0, qt = 0;
        d[roots[r]] = base[r];
        queue[qt++] = roots[r];
        while (qh < qt) {
            int u = queue[qh++];
            for (int a = G->first[u]; a < G->first[u + 1]; ++a) {
                int v = G->head[a];
                /* v can reach u if the arc v->u (the partner of a) has residual */
                if (d[v] == 2 * N && v != s && v != t && G->res[G->rev[a]] > 0) {
                    d[v] = d[u] + 1;
                    queue[qt++] = v;
                }
            }
        }
    }
}

/* Residual reachability from s; writes mask[p] = 1 for reached pixels. */
static int csr_source_side(const orc_graph *G, int s, int t, int n, uint8_t *mask, int *queue) {
    uint8_t *seen = (uint8_t *)calloc((size_t)G->N, 1);
    if (!seen) return -1;
    int qh = 0, qt = 0;
    seen[s] = 1;
    queue[qt++] = s;
    while (qh < qt) {
        int u = queue[qh++];
        for (int a = G->first[u]; a < G->first[u + 1]; ++a) {
            int v = G->head[a];
            if (!seen[v] && G->res[a] > 0) {
                seen[v] = 1;
                queue[qt++] = v;
            }
        }
    }
    int reached_t = seen[t];
    for (int p = 0; p < n; ++p) mask[p] = seen[p];
    free(seen);
    return reached_t ? -2 : 0;
}

/*
 * Returns 0 on success, -1 out of memory, -2 internal check failed (the final
 * state is not a flow, or t is still reachable from s).
 */
static int fifo_pr(const orc_grid *gp, int64_t lambda, int64_t *flow_out, uint8_t *mask_out, int64_t *stats);

int oracle_fifo_pr(int W, int H, int K, const int32_t *nlink, const int32_t *cap_src,
                   const int32_t *cap_snk0, const int32_t *slope, const uint8_t *seed,
                   int64_t lambda, int64_t *flow_out, uint8_t *mask_out, int64_t *stats) {
    orc_grid g = {W, H, K, nlink, cap_src, cap_snk0, slope, seed, 1};
    return fifo_pr(&g, lambda, flow_out, mask_out, stats);
}

/* lambda = num / den: *flow_out = den * F(num / den); the mask is S_min there.
 * Returns -3 for den < 1. */
int oracle_fifo_pr_rational(int W, int H, int K, const int32_t *nlink, const int32_t *cap_src,
                            const int32_t *cap_snk0, const int32_t *slope, const uint8_t *seed,
                            int64_t num, int64_t den, int64_t *flow_out, uint8_t *mask_out, int64_t *stats) {
    if (den < 1) return -3;
    orc_grid g = {W, H, K, nlink, cap_src, cap_snk0, slope, seed, den};
    return fifo_pr(&g, num, flow_out, mask_out, stats);
}

static int fifo_pr(const orc_grid *gp, int64_t lambda, int64_t *flow_out, uint8_t *mask_out, int64_t *stats) {
    const orc_grid g = *gp;
    const int W = g.W, H = g.H;
    orc_graph G;
    memset(&G, 0, sizeof(G));
    if (graph_build(&g, lambda, &G)) {
        graph_free(&G);
        return -1;
    }
    int n = W * H, N = G.N, s = n, t = n + 1;
    int64_t *e = (int64_t *)calloc((size_t)N, sizeof(int64_t));
    int *d = (int *)malloc(sizeof(int) * (size_t)N);
    int *cur = (int *)malloc(sizeof(int) * (size_t)N);
    int *queue = (int *)malloc(sizeof(int) * (size_t)(N + 1));
    int *fifo = (int *)malloc(sizeof(int) * (size_t)(N + 1));
    uint8_t *inq = (uint8_t *)calloc((size_t)N, 1);
    int rc = 0;
    if (!e || !d || !cur || !queue || !fifo || !inq) {
        rc = -1;
        goto done;
    }
    /* saturate every arc out of s */
    for (int a = G.first[s]; a < G.first[s + 1]; ++a) {
        int64_t c = G.res[a];
        if (c <= 0) continue;
        G.res[a] = 0;
        G.res[G.rev[a]] += c;
        e[G.head[a]] += c;
        e[s] -= c;
    }
    global_relabel(&G, s, t, d, queue);
    for (int v = 0; v < N; ++v) cur[v] = G.first[v];
    /* circular FIFO of active vertices (excess > 0, not s or t) */
    int fh = 0, ft = 0, cap = N + 1;
    for (int v = 0; v < n; ++v)
        if (e[v] > 0) {
            fifo[ft] = v;
            ft = (ft + 1) % cap;
            inq[v] = 1;
        }
    int64_t relabels = 0, pushes = 0, grs = 1, since_gr = 0;
    while (fh != ft) {
        int v = fifo[fh];
        fh = (fh + 1) % cap;
        inq[v] = 0;
        /* discharge v */
        while (e[v] > 0) {
            int a = cur[v];
            if (a == G.first[v + 1]) {
                /* relabel: one above the lowest residual neighbour */
                int m = 2 * N;
                for (int b = G.first[v]; b < G.first[v + 1]; ++b)
                    if (G.res[b] > 0 && d[G.head[b]] + 1 < m) m = d[G.head[b]] + 1;
                d[v] = m;
                cur[v] = G.first[v];
                relabels++;
                since_gr++;
                continue;
            }
            int w = G.head[a];
            if (G.res[a] > 0 && d[v] == d[w] + 1) {
                int64_t delta = e[v] < G.res[a] ? e[v] : G.res[a];
                G.res[a] -= delta;
                G.res[G.rev[a]] += delta;
                e[v] -= delta;
                e[w] += delta;
                pushes++;
                if (w != s && w != t && !inq[w] && e[w] > 0) {
                    fifo[ft] = w;
                    ft = (ft + 1) % cap;
                    inq[w] = 1;
                }
            } else {
                cur[v]++;
            }
        }
        if (since_gr >= N) {
            global_relabel(&G, s, t, d, queue);
            for (int u = 0; u < N; ++u) cur[u] = G.first[u];
            since_gr = 0;
            grs++;
        }
    }
    /* the final state must be a flow: no excess left on any pixel */
    for (int v = 0; v < n; ++v)
        if (e[v] != 0) {
            rc = -2;
            goto done;
        }
    *flow_out = e[t];
    rc = csr_source_side(&G, s, t, n, mask_out, queue);
    if (stats) {
        stats[0] = pushes;
        stats[1] = relabels;
        stats[2] = grs;
    }
done:
    free(e);
    free(d);
    free(cur);
    free(queue);
    free(fifo);
    free(inq);
    graph_free(&G);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Edmonds-Karp on per-direction residual planes (no arc list).             */
/* ------------------------------------------------------------------------ */
int oracle_ek(int W, int H, int K, const int32_t *nlink, const int32_t *cap_src,
              const int32_t *cap_snk0, const int32_t *slope, const uint8_t *seed,
              int64_t lambda, int64_t *flow_out, uint8_t *mask_out, int64_t *stats) {
    orc_grid g = {W, H, K, nlink, cap_src, cap_snk0, slope, seed, 1};
    int n = W * H;
    /* residual of p->p+d_k, of s->p, of p->s, of p->t (t->p is never useful
     * for an s-t path: t is the target and is never left) */
    int64_t *rk = (int64_t *)malloc(sizeof(int64_t) * (size_t)K * n);
    int64_t *rs = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *rsback = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t *rt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int *par = (int *)malloc(sizeof(int) * (size_t)n);     /* predecessor pixel, -1 = s */
    int8_t *pdir = (int8_t *)malloc((size_t)n);            /* direction used into p    */
    int *queue = (int *)malloc(sizeof(int) * (size_t)n);
    uint8_t *seen = (uint8_t *)malloc((size_t)n);
    int rc = 0;
    if (!rk || !rs || !rsback || !rt || !par || !pdir || !queue || !seen) {
        rc = -1;
        goto done;
    }
    for (int k = 0; k < K; ++k)
        for (int p = 0; p < n; ++p)
            rk[(size_t)k * n + p] = neighbour(&g, p, k) >= 0 ? nlink[(size_t)k * n + p] : 0;
    for (int p = 0; p < n; ++p) terminal_caps(&g, lambda, p, &rs[p], &rt[p]);
    int64_t flow = 0, augments = 0;
    for (;;) {
        memset(seen, 0, (size_t)n);
        int qh = 0, qt = 0, last = -1;
        for (int p = 0; p < n; ++p)
            if (rs[p] > 0) {
                seen[p] = 1;
                par[p] = -1;
                pdir[p] = -1;
                queue[qt++] = p;
            }
        while (qh < qt && last < 0) {
            int u = queue[qh++];
            if (rt[u] > 0) {
                last = u;
                break;
            }
            for (int k = 0; k < K; ++k) {
                if (rk[(size_t)k * n + u] <= 0) continue;
                int v = neighbour(&g, u, k);
                if (v < 0 || seen[v]) continue;
                seen[v] = 1;
                par[v] = u;
                pdir[v] = (int8_t)k;
                queue[qt++] = v;
            }
        }
        if (last < 0) break;
        /* bottleneck along s -> ... -> last -> t */
        int64_t b = rt[last];
        int v = last;
        while (par[v] >= 0) {
            int64_t c = rk[(size_t)pdir[v] * n + par[v]];
            if (c < b) b = c;
            v = par[v];
        }
        if (rs[v] < b) b = rs[v];
        rt[last] -= b;
        v = last;
        while (par[v] >= 0) {
            int u = par[v], k = pdir[v];
            rk[(size_t)k * n + u] -= b;
            rk[(size_t)(k ^ 1) * n + v] += b;
            v = u;
        }
        rs[v] -= b;
        rsback[v] += b;
        flow += b;
        augments++;
    }
    /* residual reach from s: pixels with rs > 0, then along rk > 0.  The arc
     * p->s (rsback) leads back to s and t is unreachable, so neither matters. */
    memset(seen, 0, (size_t)n);
    {
        int qh = 0, qt = 0;
        for (int p = 0; p < n; ++p)
            if (rs[p] > 0) {
                seen[p] = 1;
                queue[qt++] = p;
            }
        while (qh < qt) {
            int u = queue[qh++];
            if (rt[u] > 0) rc = -2; /* would mean the flow is not maximum */
            for (int k = 0; k < K; ++k) {
                if (rk[(size_t)k * n + u] <= 0) continue;
                int v = neighbour(&g, u, k);
                if (v < 0 || seen[v]) continue;
                seen[v] = 1;
                queue[qt++] = v;
            }
        }
    }
    for (int p = 0; p < n; ++p) mask_out[p] = seen[p];
    *flow_out = flow;
    if (stats) stats[0] = augments;
done:
    free(rk);
    free(rs);
    free(rsback);
    free(rt);
    free(par);
    free(pdir);
    free(queue);
    free(seen);
    return rc;
}

/* Cost of the cut whose source side is mask (1 = with s), from the original
 * capacities: sum over p outside of cs(p) + sum over p inside of ct(p) + sum of
 * n-link capacities of arcs leaving the source side. */
int64_t oracle_cut_cost(int W, int H, int K, const int32_t *nlink, const int32_t *cap_src,
                        const int32_t *cap_snk0, const int32_t *slope, const uint8_t *seed,
                        int64_t lambda, const uint8_t *mask) {
    orc_grid g = {W, H, K, nlink, cap_src, cap_snk0, slope, seed, 1};
    int n = W * H;
    int64_t cost = 0;
    for (int p = 0; p < n; ++p) {
        int64_t cs, ct;
        terminal_caps(&g, lambda, p, &cs, &ct);
        if (mask[p]) {
            cost += ct;
            for (int k = 0; k < K; ++k) {
                int q = neighbour(&g, p, k);
                if (q >= 0 && !mask[q]) cost += nlink[(size_t)k * n + p];
            }
        } else {
            cost += cs;
        }
    }
    return cost;
}
