/*
 * CPU oracle for the s-t maximum-flow value -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the package smoke check and the benchmark's CPU
 * baseline load this file's library.  It shares no code, header, table or
 * data layout with the HIP library; it is plain sequential C with int64
 * arithmetic throughout, written for obviousness rather than speed.
 *
 * Problem (paper, Section 2.1): a directed graph with non-negative capacities
 * c(u,v), a source s and a sink t; a flow obeys 0 <= f(u,v) <= c(u,v) and
 * conservation at every vertex other than s and t; the maximum flow value F*
 * equals the minimum capacity of an s-t cut (max-flow min-cut theorem, cited
 * in the paper's Section 3.1 proof).
 *
 * Parts
 *   or_brute_min_cut  the plain min-cut definition: enumerate every vertex
 *                     subset S with s in S, t not in S (tiny graphs only)
 *   or_edmonds_karp   shortest augmenting paths (Edmonds-Karp, cited in the
 *                     paper's Section 2.2) on the raw, unmerged edge list
 *   og_*              a residual network over MERGED capacities (parallel
 *                     edges summed) with sequential FIFO push-relabel
 *                     (Goldberg-Tarjan, Section 2.2) using the gap heuristic
 *                     and the global-relabel heuristic (Section 2.2); the
 *                     sinks are t plus every deficient vertex, which is what
 *                     the dynamic algorithm of Section 4.2 (Algorithms 5 and 6)
 *                     needs, so the same solver gives the static value (from
 *                     zero flow, Algorithm 1's initialisation) and the value
 *                     after an update batch (Algorithm 5's steps, in order)
 *   or_cert_check     solver-independent certificate: flow feasibility,
 *                     conservation, flow value, and a cut of equal capacity
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_ERR_INPUT 1
#define OR_ERR_NOMEM 2

static void* xmalloc(size_t bytes) {
    void* p = malloc(bytes ? bytes : 1);
    if (!p) {
        fprintf(stderr, "oracle: out of memory (%zu bytes)\n", bytes);
        abort();
    }
    return p;
}

static void* xcalloc(size_t count, size_t size) {
    void* p = calloc(count ? count : 1, size ? size : 1);
    if (!p) {
        fprintf(stderr, "oracle: out of memory\n");
        abort();
    }
    return p;
}

/* ------------------------------------------------------------------------ */
/* Brute force: F* = min over S (s in S, t not in S) of sum_{u in S, v not  */
/* in S} c(u,v).  Raw edge list, duplicates counted as they come.           */
/* ------------------------------------------------------------------------ */
int64_t or_brute_min_cut(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         const int32_t* cap, int32_t s, int32_t t) {
    if (n < 2 || n > 22 || s == t) return -1;
    int32_t others[32];
    int k = 0;
    for (int32_t v = 0; v < n; ++v)
        if (v != s && v != t) others[k++] = v;
    uint8_t in_s[32];
    int64_t best = -1;
    for (uint64_t mask = 0; mask < (1ull << k); ++mask) {
        memset(in_s, 0, sizeof(in_s));
        in_s[s] = 1;
        for (int i = 0; i < k; ++i)
            if (mask >> i & 1) in_s[others[i]] = 1;
        int64_t c = 0;
        for (int64_t i = 0; i < m; ++i)
            if (in_s[src[i]] && !in_s[dst[i]]) c += cap[i];
        if (best < 0 || c < best) best = c;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Edmonds-Karp on the raw edge list.  Edge i becomes arc 2i (u->v, c) and  */
/* arc 2i+1 (v->u, 0).  Repeatedly augment along a BFS-shortest path in the */
/* residual network until t is unreachable.                                 */
/* flow_out[i] (optional) = flow on input edge i; side_out[v] (optional) =  */
/* 1 when v is reachable from s in the final residual network.              */
/* ------------------------------------------------------------------------ */
int64_t or_edmonds_karp(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        const int32_t* cap, int32_t s, int32_t t, int64_t* flow_out,
                        uint8_t* side_out) {
    int64_t na = 2 * m;
    int32_t* head = xmalloc(sizeof(int32_t) * (size_t)na);
    int64_t* res = xmalloc(sizeof(int64_t) * (size_t)na);
    int64_t* first = xcalloc((size_t)n + 1, sizeof(int64_t));
    int64_t* list = xmalloc(sizeof(int64_t) * (size_t)na);
    for (int64_t i = 0; i < m; ++i) {
        head[2 * i] = dst[i];
        res[2 * i] = cap[i];
        head[2 * i + 1] = src[i];
        res[2 * i + 1] = 0;
        first[src[i] + 1]++;
        first[dst[i] + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) first[v + 1] += first[v];
    int64_t* fill = xmalloc(sizeof(int64_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) fill[v] = first[v];
    for (int64_t i = 0; i < m; ++i) {
        list[fill[src[i]]++] = 2 * i;
        list[fill[dst[i]]++] = 2 * i + 1;
    }
    int64_t* parent = xmalloc(sizeof(int64_t) * (size_t)n);
    int32_t* queue = xmalloc(sizeof(int32_t) * (size_t)n);
    int64_t value = 0;
    for (;;) {
        for (int32_t v = 0; v < n; ++v) parent[v] = -2;
        parent[s] = -1;
        int32_t qh = 0, qt = 0;
        queue[qt++] = s;
        while (qh < qt && parent[t] == -2) {
            int32_t u = queue[qh++];
            for (int64_t k = first[u]; k < first[u + 1]; ++k) {
                int64_t a = list[k];
                int32_t w = head[a];
                if (res[a] > 0 && parent[w] == -2) {
                    parent[w] = a;
                    queue[qt++] = w;
                }
            }
        }
        if (parent[t] == -2) break;
        int64_t bottleneck = INT64_MAX;
        for (int32_t v = t; v != s; v = head[parent[v] ^ 1])
            if (res[parent[v]] < bottleneck) bottleneck = res[parent[v]];
        for (int32_t v = t; v != s; v = head[parent[v] ^ 1]) {
            res[parent[v]] -= bottleneck;
            res[parent[v] ^ 1] += bottleneck;
        }
        value += bottleneck;
    }
    if (flow_out)
        for (int64_t i = 0; i < m; ++i) flow_out[i] = res[2 * i + 1];
    if (side_out)
        for (int32_t v = 0; v < n; ++v) side_out[v] = parent[v] != -2;
    free(head); free(res); free(first); free(list); free(fill); free(parent); free(queue);
    return value;
}

/* ------------------------------------------------------------------------ */
/* Merged residual network with sequential push-relabel.                    */
/* Each distinct directed pair (u,v) with u != v owns an arc pair: a = u->v */
/* carries c(u,v), a^1 = v->u carries capacity 0 (its residual is the flow  */
/* on a).  The pair (v,u), if present, owns a separate arc pair.            */
/* ------------------------------------------------------------------------ */
typedef struct og {
    int32_t n, s, t;
    int64_t na, na_cap;          /* arcs in use / allocated */
    int32_t* head;               /* arc -> head vertex */
    int32_t* tail;               /* arc -> tail vertex */
    int64_t* cap;                /* arc -> capacity (0 on odd arcs) */
    int64_t* res;                /* arc -> residual capacity */
    /* per-vertex adjacency lists (arc ids) in a growable pool */
    int64_t* vbeg;
    int32_t* vdeg;
    int32_t* vroom;
    int64_t* pool;
    int64_t pool_len, pool_cap;
    /* (u,v) -> even arc id, open addressing */
    uint64_t* hkey;
    int64_t* hval;
    int64_t hcap, hcount;
    /* solver state */
    int64_t* e;
    int32_t* h;
    int32_t* cur;                /* current-arc position per vertex */
    /* FIFO of active vertices */
    int32_t* q;
    int64_t qhead, qcount;
    uint8_t* inq;
    /* height buckets (doubly linked) for the gap heuristic */
    int32_t* bhead;
    int32_t* bnext;
    int32_t* bprev;
    int32_t maxh;
    int64_t work;
    /* statistics */
    int64_t n_push, n_relabel, n_gap, n_global;
} og_t;

static const uint64_t HEMPTY = ~0ull;

static uint64_t pair_key(int32_t u, int32_t v) { return ((uint64_t)(uint32_t)u << 32) | (uint32_t)v; }

static uint64_t mix64(uint64_t x) {
    x ^= x >> 33; x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33; x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return x;
}

static int64_t map_find(const og_t* g, int32_t u, int32_t v) {
    uint64_t k = pair_key(u, v);
    uint64_t i = mix64(k) & (uint64_t)(g->hcap - 1);
    for (;;) {
        if (g->hkey[i] == HEMPTY) return -1;
        if (g->hkey[i] == k) return g->hval[i];
        i = (i + 1) & (uint64_t)(g->hcap - 1);
    }
}

static void map_put_raw(uint64_t* keys, int64_t* vals, int64_t cap, uint64_t k, int64_t val) {
    uint64_t i = mix64(k) & (uint64_t)(cap - 1);
    while (keys[i] != HEMPTY && keys[i] != k) i = (i + 1) & (uint64_t)(cap - 1);
    keys[i] = k;
    vals[i] = val;
}

static void map_put(og_t* g, int32_t u, int32_t v, int64_t a) {
    if (2 * (g->hcount + 1) > g->hcap) {
        int64_t ncap = g->hcap * 2;
        uint64_t* nk = xmalloc(sizeof(uint64_t) * (size_t)ncap);
        int64_t* nv = xmalloc(sizeof(int64_t) * (size_t)ncap);
        for (int64_t i = 0; i < ncap; ++i) nk[i] = HEMPTY;
        for (int64_t i = 0; i < g->hcap; ++i)
            if (g->hkey[i] != HEMPTY) map_put_raw(nk, nv, ncap, g->hkey[i], g->hval[i]);
        free(g->hkey); free(g->hval);
        g->hkey = nk; g->hval = nv; g->hcap = ncap;
    }
    map_put_raw(g->hkey, g->hval, g->hcap, pair_key(u, v), a);
    g->hcount++;
}

static void adj_push(og_t* g, int32_t v, int64_t a) {
    if (g->vdeg[v] == g->vroom[v]) {
        int32_t room = g->vroom[v] * 2 + 4;
        if (g->pool_len + room > g->pool_cap) {
            int64_t ncap = (g->pool_len + room) * 3 / 2 + 16;
            int64_t* np = xmalloc(sizeof(int64_t) * (size_t)ncap);
            memcpy(np, g->pool, sizeof(int64_t) * (size_t)g->pool_len);
            free(g->pool);
            g->pool = np;
            g->pool_cap = ncap;
        }
        memcpy(g->pool + g->pool_len, g->pool + g->vbeg[v], sizeof(int64_t) * (size_t)g->vdeg[v]);
        g->vbeg[v] = g->pool_len;
        g->vroom[v] = room;
        g->pool_len += room;
    }
    g->pool[g->vbeg[v] + g->vdeg[v]++] = a;
}

static int64_t new_arc_pair(og_t* g, int32_t u, int32_t v) {
    if (g->na + 2 > g->na_cap) {
        int64_t nc = g->na_cap * 3 / 2 + 64;
        g->head = realloc(g->head, sizeof(int32_t) * (size_t)nc);
        g->tail = realloc(g->tail, sizeof(int32_t) * (size_t)nc);
        g->cap = realloc(g->cap, sizeof(int64_t) * (size_t)nc);
        g->res = realloc(g->res, sizeof(int64_t) * (size_t)nc);
        if (!g->head || !g->tail || !g->cap || !g->res) abort();
        g->na_cap = nc;
    }
    int64_t a = g->na;
    g->na += 2;
    g->head[a] = v; g->tail[a] = u; g->cap[a] = 0; g->res[a] = 0;
    g->head[a + 1] = u; g->tail[a + 1] = v; g->cap[a + 1] = 0; g->res[a + 1] = 0;
    adj_push(g, u, a);
    adj_push(g, v, a + 1);
    map_put(g, u, v, a);
    return a;
}

void og_free(og_t* g) {
    if (!g) return;
    free(g->head); free(g->tail); free(g->cap); free(g->res);
    free(g->vbeg); free(g->vdeg); free(g->vroom); free(g->pool);
    free(g->hkey); free(g->hval);
    free(g->e); free(g->h); free(g->cur); free(g->q); free(g->inq);
    free(g->bhead); free(g->bnext); free(g->bprev);
    free(g);
}

/* Build the merged network.  Inputs: validated by the caller (u != v, ids in */
/* range, capacities >= 0).  Parallel (u,v) edges are summed.               */
og_t* og_create(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const int32_t* cap,
                int32_t s, int32_t t) {
    if (n < 2 || s < 0 || t < 0 || s >= n || t >= n || s == t) return NULL;
    for (int64_t i = 0; i < m; ++i)
        if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n || src[i] == dst[i] || cap[i] < 0)
            return NULL;
    og_t* g = xcalloc(1, sizeof(og_t));
    g->n = n; g->s = s; g->t = t;
    g->na_cap = 2 * m + 64;
    g->head = xmalloc(sizeof(int32_t) * (size_t)g->na_cap);
    g->tail = xmalloc(sizeof(int32_t) * (size_t)g->na_cap);
    g->cap = xmalloc(sizeof(int64_t) * (size_t)g->na_cap);
    g->res = xmalloc(sizeof(int64_t) * (size_t)g->na_cap);
    g->vbeg = xcalloc((size_t)n, sizeof(int64_t));
    g->vdeg = xcalloc((size_t)n, sizeof(int32_t));
    g->vroom = xcalloc((size_t)n, sizeof(int32_t));
    /* pre-size each adjacency list with its raw degree so loading does not move lists */
    for (int64_t i = 0; i < m; ++i) { g->vroom[src[i]]++; g->vroom[dst[i]]++; }
    int64_t total = 0;
    for (int32_t v = 0; v < n; ++v) { g->vbeg[v] = total; total += g->vroom[v]; }
    g->pool_cap = total + 64;
    g->pool = xmalloc(sizeof(int64_t) * (size_t)g->pool_cap);
    g->pool_len = total;
    g->hcap = 64;
    while (g->hcap < 2 * (m + 16)) g->hcap *= 2;
    g->hkey = xmalloc(sizeof(uint64_t) * (size_t)g->hcap);
    g->hval = xmalloc(sizeof(int64_t) * (size_t)g->hcap);
    for (int64_t i = 0; i < g->hcap; ++i) g->hkey[i] = HEMPTY;
    for (int64_t i = 0; i < m; ++i) {
        int64_t a = map_find(g, src[i], dst[i]);
        if (a < 0) a = new_arc_pair(g, src[i], dst[i]);
        g->cap[a] += cap[i];
    }
    for (int64_t a = 0; a < g->na; ++a) g->res[a] = g->cap[a];
    g->e = xcalloc((size_t)n, sizeof(int64_t));
    g->h = xcalloc((size_t)n, sizeof(int32_t));
    g->cur = xcalloc((size_t)n, sizeof(int32_t));
    g->q = xmalloc(sizeof(int32_t) * (size_t)n);
    g->inq = xcalloc((size_t)n, 1);
    g->bhead = xmalloc(sizeof(int32_t) * (size_t)n);
    g->bnext = xmalloc(sizeof(int32_t) * (size_t)n);
    g->bprev = xmalloc(sizeof(int32_t) * (size_t)n);
    return g;
}

int64_t og_num_pairs(const og_t* g) { return g->na / 2; }

/* --- FIFO of active vertices ------------------------------------------- */
static void q_push(og_t* g, int32_t v) {
    if (g->inq[v]) return;
    g->inq[v] = 1;
    g->q[(g->qhead + g->qcount) % g->n] = v;
    g->qcount++;
}

static int32_t q_pop(og_t* g) {
    int32_t v = g->q[g->qhead];
    g->qhead = (g->qhead + 1) % g->n;
    g->qcount--;
    g->inq[v] = 0;
    return v;
}

/* --- height buckets ----------------------------------------------------- */
static void b_insert(og_t* g, int32_t v) {
    int32_t k = g->h[v];
    g->bprev[v] = -1;
    g->bnext[v] = g->bhead[k];
    if (g->bhead[k] >= 0) g->bprev[g->bhead[k]] = v;
    g->bhead[k] = v;
    if (k > g->maxh) g->maxh = k;
}

static void b_remove(og_t* g, int32_t v) {
    int32_t k = g->h[v];
    if (g->bprev[v] >= 0) g->bnext[g->bprev[v]] = g->bnext[v];
    else g->bhead[k] = g->bnext[v];
    if (g->bnext[v] >= 0) g->bprev[g->bnext[v]] = g->bprev[v];
}

static int is_active(const og_t* g, int32_t v) {
    return v != g->s && v != g->t && g->e[v] > 0 && g->h[v] < g->n;
}

/* Global relabel (backward BFS, Algorithm 6): h(t) = 0, h(s) = |V|, every */
/* deficient vertex gets 0, every other vertex the residual hop distance to */
/* the nearest of those, |V| when none is reachable.                        */
static void global_relabel(og_t* g) {
    int32_t n = g->n;
    int32_t* bfs = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t qh = 0, qt = 0;
    for (int32_t v = 0; v < n; ++v) g->h[v] = n;
    g->h[g->t] = 0;
    bfs[qt++] = g->t;
    for (int32_t v = 0; v < n; ++v)
        if (v != g->s && v != g->t && g->e[v] < 0) {
            g->h[v] = 0;
            bfs[qt++] = v;
        }
    while (qh < qt) {
        int32_t u = bfs[qh++];
        const int64_t* adj = g->pool + g->vbeg[u];
        for (int32_t k = 0; k < g->vdeg[u]; ++k) {
            int64_t a = adj[k];          /* a: u -> w, so a^1 is w -> u */
            int32_t w = g->head[a];
            if (w != g->s && g->h[w] == n && g->res[a ^ 1] > 0) {
                g->h[w] = g->h[u] + 1;
                bfs[qt++] = w;
            }
        }
    }
    free(bfs);
    for (int32_t k = 0; k < n; ++k) g->bhead[k] = -1;
    g->maxh = 0;
    for (int32_t v = 0; v < n; ++v) {
        g->cur[v] = 0;
        if (v != g->s && g->h[v] < n) b_insert(g, v);
    }
    g->qhead = 0; g->qcount = 0;
    memset(g->inq, 0, (size_t)n);
    for (int32_t v = 0; v < n; ++v)
        if (is_active(g, v)) q_push(g, v);
    g->work = 0;
    g->n_global++;
}

static void relabel(og_t* g, int32_t u) {
    int32_t n = g->n;
    int32_t old = g->h[u];
    int32_t nh = n;
    const int64_t* adj = g->pool + g->vbeg[u];
    for (int32_t k = 0; k < g->vdeg[u]; ++k) {
        int64_t a = adj[k];
        if (g->res[a] > 0 && g->h[g->head[a]] + 1 < nh) nh = g->h[g->head[a]] + 1;
    }
    b_remove(g, u);
    g->n_relabel++;
    g->work += 12 + g->vdeg[u];
    if (g->bhead[old] < 0) {
        /* gap: no vertex is left at height `old`, so nothing above it can
         * reach a height-0 vertex any more */
        for (int32_t k = old + 1; k <= g->maxh; ++k) {
            for (int32_t v = g->bhead[k]; v >= 0; v = g->bnext[v]) g->h[v] = n;
            g->bhead[k] = -1;
        }
        g->maxh = old > 0 ? old - 1 : 0;
        g->h[u] = n;
        g->n_gap++;
    } else {
        g->h[u] = nh;
        if (nh < n) b_insert(g, u);
    }
    g->cur[u] = 0;
}

static void discharge(og_t* g, int32_t u) {
    int32_t n = g->n;
    while (g->e[u] > 0 && g->h[u] < n) {
        if (g->cur[u] == g->vdeg[u]) {
            relabel(g, u);
            continue;
        }
        int64_t a = g->pool[g->vbeg[u] + g->cur[u]];
        int32_t w = g->head[a];
        if (g->res[a] > 0 && g->h[u] == g->h[w] + 1) {
            int64_t d = g->e[u] < g->res[a] ? g->e[u] : g->res[a];
            int64_t before = g->e[w];
            g->res[a] -= d;
            g->res[a ^ 1] += d;
            g->e[u] -= d;
            g->e[w] += d;
            g->n_push++;
            if (before <= 0 && g->e[w] > 0 && is_active(g, w)) q_push(g, w);
        } else {
            g->cur[u]++;
        }
    }
}

/* Run push-relabel from the current preflow until no vertex outside {s,t} */
/* has positive excess below height |V|; return e(t) + sum of deficits.     */
static int64_t solve(og_t* g) {
    int64_t period = (6 * (int64_t)g->n + g->na) / 2;
    global_relabel(g);
    while (g->qcount > 0) {
        int32_t u = q_pop(g);
        if (!is_active(g, u)) continue;
        discharge(g, u);
        if (g->work > period) global_relabel(g);
    }
    int64_t value = g->e[g->t];
    for (int32_t v = 0; v < g->n; ++v)
        if (v != g->s && v != g->t && g->e[v] < 0) value += g->e[v];
    return value;
}

/* Push every unit of residual capacity out of s (Algorithm 1's saturation, */
/* and its re-application after a batch in Algorithm 5).                    */
static void saturate_source(og_t* g) {
    int32_t s = g->s;
    const int64_t* adj = g->pool + g->vbeg[s];
    for (int32_t k = 0; k < g->vdeg[s]; ++k) {
        int64_t a = adj[k];
        int64_t x = g->res[a];
        if (x > 0) {
            g->res[a] = 0;
            g->res[a ^ 1] += x;
            g->e[g->head[a]] += x;
            g->e[s] -= x;
        }
    }
}

/* Static max flow (Algorithm 1): zero flow, saturate s, push-relabel. */
int64_t og_static(og_t* g) {
    for (int64_t a = 0; a < g->na; ++a) g->res[a] = g->cap[a];
    memset(g->e, 0, sizeof(int64_t) * (size_t)g->n);
    saturate_source(g);
    return solve(g);
}

/* Dynamic max flow (Algorithm 5) after a batch of k updates "c(u,v) := c'". */
/* Returns the new value, or -1 on invalid input (nothing is changed then).  */
int64_t og_apply(og_t* g, int64_t k, const int32_t* uu, const int32_t* vv, const int32_t* cc) {
    for (int64_t i = 0; i < k; ++i)
        if (uu[i] < 0 || uu[i] >= g->n || vv[i] < 0 || vv[i] >= g->n || uu[i] == vv[i] || cc[i] < 0)
            return -1;
    int64_t* touched = xmalloc(sizeof(int64_t) * (size_t)(k ? k : 1));
    /* 1. add the change of every capacity to its residual (later updates of */
    /*    the same pair overwrite earlier ones, so the last one wins)         */
    for (int64_t i = 0; i < k; ++i) {
        int64_t a = map_find(g, uu[i], vv[i]);
        if (a < 0) a = new_arc_pair(g, uu[i], vv[i]);
        g->res[a] += (int64_t)cc[i] - g->cap[a];
        g->cap[a] = cc[i];
        touched[i] = a;
    }
    /* 2. an over-full arc sends its surplus flow back */
    for (int64_t i = 0; i < k; ++i) {
        int64_t a = touched[i];
        if (g->res[a] < 0) {
            g->res[a ^ 1] += g->res[a];
            g->res[a] = 0;
        }
    }
    free(touched);
    /* 3. excess of every vertex = flow in - flow out (flow on an even arc is */
    /*    the residual of its odd partner)                                    */
    memset(g->e, 0, sizeof(int64_t) * (size_t)g->n);
    for (int64_t a = 0; a < g->na; a += 2) {
        int64_t f = g->res[a + 1];
        g->e[g->head[a]] += f;
        g->e[g->tail[a]] -= f;
    }
    /* 4. the source saturates its out-arcs again */
    saturate_source(g);
    /* 5. push-relabel with t and the deficient vertices as sinks */
    return solve(g);
}

/* Source side of the cut certified by the final heights: the vertices that */
/* cannot reach t or a deficient vertex in the residual network.  Returns   */
/* the capacity of that cut over the current (merged) capacities.          */
int64_t og_min_cut(og_t* g, uint8_t* side) {
    global_relabel(g);
    int64_t c = 0;
    for (int32_t v = 0; v < g->n; ++v) side[v] = g->h[v] == g->n;
    for (int64_t a = 0; a < g->na; a += 2)
        if (side[g->tail[a]] && !side[g->head[a]]) c += g->cap[a];
    return c;
}

/* Heights and excess right after Algorithm 1's initialisation and the first */
/* backward BFS (zero flow, s saturated).  Leaves the network in that state. */
void og_initial_labels(og_t* g, int32_t* h_out, int64_t* e_out) {
    for (int64_t a = 0; a < g->na; ++a) g->res[a] = g->cap[a];
    memset(g->e, 0, sizeof(int64_t) * (size_t)g->n);
    saturate_source(g);
    global_relabel(g);
    memcpy(h_out, g->h, sizeof(int32_t) * (size_t)g->n);
    memcpy(e_out, g->e, sizeof(int64_t) * (size_t)g->n);
}

/* Current state, for invariant tests: per vertex e and h. */
void og_state(const og_t* g, int64_t* e_out, int32_t* h_out) {
    if (e_out) memcpy(e_out, g->e, sizeof(int64_t) * (size_t)g->n);
    if (h_out) memcpy(h_out, g->h, sizeof(int32_t) * (size_t)g->n);
}

/* Current merged capacities and flows: one entry per pair with an arc pair */
/* (including pairs whose capacity went to 0).  Arrays sized og_num_pairs.  */
void og_pairs(const og_t* g, int32_t* u, int32_t* v, int64_t* c, int64_t* flow) {
    for (int64_t a = 0, i = 0; a < g->na; a += 2, ++i) {
        if (u) u[i] = g->tail[a];
        if (v) v[i] = g->head[a];
        if (c) c[i] = g->cap[a];
        if (flow) flow[i] = g->res[a + 1];
    }
}

void og_stats(const og_t* g, int64_t* out4) {
    out4[0] = g->n_push; out4[1] = g->n_relabel; out4[2] = g->n_gap; out4[3] = g->n_global;
}

/* ------------------------------------------------------------------------ */
/* Certificate.  Given an edge list (duplicates allowed), a flow per edge,  */
/* a vertex side (1 = source side) and a claimed value, check:              */
/*   1. 0 <= f <= c on every edge                                           */
/*   2. conservation at every vertex other than s and t                     */
/*   3. net flow into t == value == net flow out of s                        */
/*   4. side[s] = 1, side[t] = 0 and the cut capacity == value              */
/* Either of flow / side may be NULL to skip its checks.  Returns 0 when    */
/* all requested checks pass, else the number of the first failed check,   */
/* with a message in msg.                                                   */
/* ------------------------------------------------------------------------ */
int or_cert_check(int32_t n, int64_t m, const int32_t* src, const int32_t* dst, const int32_t* cap,
                  int32_t s, int32_t t, const int64_t* flow, const uint8_t* side, int64_t value,
                  char* msg, int32_t msg_len) {
    int rc = 0;
    if (flow) {
        int64_t* net = xcalloc((size_t)n, sizeof(int64_t));
        for (int64_t i = 0; i < m; ++i) {
            if (flow[i] < 0 || flow[i] > cap[i]) {
                snprintf(msg, (size_t)msg_len, "edge %lld (%d->%d): flow %lld outside [0,%d]",
                         (long long)i, src[i], dst[i], (long long)flow[i], cap[i]);
                free(net);
                return 1;
            }
            net[dst[i]] += flow[i];
            net[src[i]] -= flow[i];
        }
        for (int32_t v = 0; v < n && !rc; ++v)
            if (v != s && v != t && net[v] != 0) {
                snprintf(msg, (size_t)msg_len, "vertex %d: net inflow %lld != 0", v, (long long)net[v]);
                rc = 2;
            }
        if (!rc && (net[t] != value || -net[s] != value)) {
            snprintf(msg, (size_t)msg_len, "flow value: into t %lld, out of s %lld, claimed %lld",
                     (long long)net[t], (long long)-net[s], (long long)value);
            rc = 3;
        }
        free(net);
        if (rc) return rc;
    }
    if (side) {
        if (!side[s] || side[t]) {
            snprintf(msg, (size_t)msg_len, "cut does not separate s from t");
            return 4;
        }
        int64_t c = 0;
        for (int64_t i = 0; i < m; ++i)
            if (side[src[i]] && !side[dst[i]]) c += cap[i];
        if (c != value) {
            snprintf(msg, (size_t)msg_len, "cut capacity %lld != value %lld", (long long)c,
                     (long long)value);
            return 4;
        }
    }
    if (msg_len > 0) msg[0] = 0;
    return 0;
}
