/*
 * rn_oracle.c -- plain CPU oracle for the network-distance theta-join and the
 * k-closest-pairs join.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  The GPU library
 * never links, calls or includes anything from here, and this file includes
 * nothing from it.
 *
 * What is computed (the paper's problem statement):
 *   theta-join  (Abstract; Section 1; Section 4, opening paragraph):
 *       every (u, v, dist(u,v)) with u in R, v in S and dist(u,v) <= theta,
 *       where dist is the shortest-path length over the weighted arcs of the
 *       road network (network distance, not Euclidean; Section 1).
 *   k closest pairs (Abstract; Section 1; Section 6):
 *       the k pairs (u,v), u in R, v in S, whose distance is no larger than that
 *       of any pair left out.  Ties are broken by (dist, u, v) ascending so the
 *       answer is unique; with fewer than k reachable pairs, all are returned.
 *   Both results are returned sorted by (dist, u, v).
 *
 * How: textbook Dijkstra from each u in R with a binary heap (lazy deletion),
 * cut off at theta (an arc whose tentative length exceeds theta is not
 * followed, and the search ends when the smallest tentative length exceeds
 * theta).  Every settled v that is in S gives a pair.  Lengths are summed in
 * 64 bits; a path of length >= 2^32 - 1 counts as unreachable.
 *
 * k-closest pairs: the same per-source search, with a bound tau taken from a
 * size-k max-heap of the best (dist,u,v) triples found so far (tau = the heap's
 * largest dist once it holds k triples, else unbounded).  A tentative length
 * above tau cannot belong to the answer, so it is not followed; a length equal
 * to tau still can (ties are decided on (u,v)).  This is the paper's shared
 * k-th-best distance threshold (Section 4, Algorithm 3 and the text after it),
 * kept here by a single thread.
 *
 * The search also counts, per source, the out-degrees of its settled vertices:
 * the number of arcs a work-efficient expansion must scan.  That count is the
 * numerator of the traversed-edges-per-second figure.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_UNREACH 0xFFFFFFFFu

typedef struct { int32_t u, v; uint32_t dist; } orc_pair;

/* ---------------- binary min-heap of (dist, vertex) ---------------- */
typedef struct { uint64_t d; int32_t x; } hitem;
typedef struct { hitem *a; int64_t n, cap; } minheap;

static int mh_push(minheap *h, uint64_t d, int32_t x) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hitem *na = (hitem *)realloc(h->a, (size_t)nc * sizeof(hitem));
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    int64_t i = h->n++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].d <= d) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].d = d; h->a[i].x = x;
    return 0;
}

static hitem mh_pop(minheap *h) {
    hitem top = h->a[0], last = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= h->n) break;
        if (c + 1 < h->n && h->a[c + 1].d < h->a[c].d) c++;
        if (h->a[c].d >= last.d) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* ---------------- pair order (dist, u, v) ---------------- */
static int pair_less(const orc_pair *a, const orc_pair *b) {
    if (a->dist != b->dist) return a->dist < b->dist;
    if (a->u != b->u) return a->u < b->u;
    return a->v < b->v;
}

static int pair_cmp(const void *pa, const void *pb) {
    const orc_pair *a = (const orc_pair *)pa, *b = (const orc_pair *)pb;
    return pair_less(a, b) ? -1 : (pair_less(b, a) ? 1 : 0);
}

/* ---------------- growable pair list ---------------- */
typedef struct { orc_pair *a; int64_t n, cap; } pairvec;

static int pv_push(pairvec *p, int32_t u, int32_t v, uint32_t d) {
    if (p->n == p->cap) {
        int64_t nc = p->cap ? 2 * p->cap : 1024;
        orc_pair *na = (orc_pair *)realloc(p->a, (size_t)nc * sizeof(orc_pair));
        if (!na) return -1;
        p->a = na; p->cap = nc;
    }
    p->a[p->n].u = u; p->a[p->n].v = v; p->a[p->n].dist = d;
    p->n++;
    return 0;
}

/* ---------------- one bounded Dijkstra ---------------- */
typedef struct {
    int32_t V;
    const int32_t *row_ptr, *col;
    const uint32_t *w;
    uint64_t *dist;      /* [V], ORC_UNREACH-filled between searches */
    int32_t *touched;    /* vertices whose dist was set, for the sparse reset */
    int64_t ntouched;
    minheap heap;
} search_ws;

static int ws_init(search_ws *s, int32_t V, const int32_t *rp, const int32_t *col, const uint32_t *w) {
    s->V = V; s->row_ptr = rp; s->col = col; s->w = w;
    s->dist = (uint64_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(uint64_t));
    s->touched = (int32_t *)malloc((size_t)(V > 0 ? V : 1) * sizeof(int32_t));
    s->ntouched = 0;
    s->heap.a = NULL; s->heap.n = 0; s->heap.cap = 0;
    if (!s->dist || !s->touched) return -1;
    for (int32_t i = 0; i < V; i++) s->dist[i] = ORC_UNREACH;
    return 0;
}

static void ws_free(search_ws *s) {
    free(s->dist); free(s->touched); free(s->heap.a);
}

static void ws_reset(search_ws *s) {
    for (int64_t i = 0; i < s->ntouched; i++) s->dist[s->touched[i]] = ORC_UNREACH;
    s->ntouched = 0;
    s->heap.n = 0;
}

/* Bounded search for the theta-join: settled vertices in S become pairs. */
static int search_join(search_ws *s, int32_t u, uint64_t theta, const uint8_t *inS,
                       pairvec *out, int64_t *arcs, int64_t *settled) {
    s->dist[u] = 0;
    s->touched[s->ntouched++] = u;
    if (mh_push(&s->heap, 0, u)) return -1;
    while (s->heap.n > 0) {
        hitem it = mh_pop(&s->heap);
        if (it.d != s->dist[it.x]) continue;          /* stale heap entry */
        if (it.d > theta) break;
        int32_t x = it.x;
        *settled += 1;
        *arcs += s->row_ptr[x + 1] - s->row_ptr[x];
        if (inS[x] && pv_push(out, u, x, (uint32_t)it.d)) return -1;
        for (int32_t a = s->row_ptr[x]; a < s->row_ptr[x + 1]; a++) {
            int32_t y = s->col[a];
            uint64_t nd = it.d + s->w[a];
            if (nd > theta || nd >= s->dist[y]) continue;
            if (s->dist[y] == ORC_UNREACH) s->touched[s->ntouched++] = y;
            s->dist[y] = nd;
            if (mh_push(&s->heap, nd, y)) return -1;
        }
    }
    ws_reset(s);
    return 0;
}

/* ---------------- theta-join, parallel over sources ---------------- */
typedef struct {
    int32_t V;
    const int32_t *row_ptr, *col;
    const uint32_t *w;
    const int32_t *R;
    int32_t nR;
    const uint8_t *inS;
    uint64_t theta;
    int64_t next;          /* next source index, taken under the lock */
    pthread_mutex_t lock;
    int failed;
} join_job;

typedef struct { join_job *job; pairvec out; int64_t arcs, settled; int rc; } join_thread;

static void *join_worker(void *arg) {
    join_thread *t = (join_thread *)arg;
    join_job *j = t->job;
    search_ws ws;
    t->rc = ws_init(&ws, j->V, j->row_ptr, j->col, j->w);
    for (;;) {
        if (t->rc) break;
        pthread_mutex_lock(&j->lock);
        int64_t i = j->next++;
        int stop = j->failed;
        pthread_mutex_unlock(&j->lock);
        if (stop || i >= j->nR) break;
        t->rc = search_join(&ws, j->R[i], j->theta, j->inS, &t->out, &t->arcs, &t->settled);
    }
    if (t->rc) { pthread_mutex_lock(&j->lock); j->failed = 1; pthread_mutex_unlock(&j->lock); }
    ws_free(&ws);
    return NULL;
}

static int check_ids(int32_t V, const int32_t *ids, int32_t n) {
    for (int32_t i = 0; i < n; i++)
        if (ids[i] < 0 || ids[i] >= V) return -1;
    return 0;
}

int orc_num_cores(void) {
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

/* Theta-join.  *out is malloc'd (free with orc_free), sorted by (dist,u,v).
 * arcs / settled receive the scanned-arc and settled-vertex totals.
 * nthreads <= 0 uses every online core.  Returns 0, or -1 on bad ids / no memory. */
int orc_dist_join(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                  const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, uint32_t theta,
                  int nthreads, orc_pair **out, int64_t *n_out, int64_t *arcs, int64_t *settled) {
    *out = NULL; *n_out = 0; *arcs = 0; *settled = 0;
    if (V < 0 || nR < 0 || nS < 0 || check_ids(V, R, nR) || check_ids(V, S, nS)) return -1;
    uint8_t *inS = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    if (!inS) return -1;
    for (int32_t i = 0; i < nS; i++) inS[S[i]] = 1;
    if (theta > ORC_UNREACH - 1u) theta = ORC_UNREACH - 1u;
    if (nthreads <= 0) nthreads = orc_num_cores();
    if (nthreads > nR) nthreads = nR > 0 ? nR : 1;
    join_job job = {V, row_ptr, col, w, R, nR, inS, theta, 0, PTHREAD_MUTEX_INITIALIZER, 0};
    join_thread *th = (join_thread *)calloc((size_t)nthreads, sizeof(join_thread));
    pthread_t *tid = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    int rc = (th && tid) ? 0 : -1;
    int started = 0;
    for (int t = 0; t < nthreads && !rc; t++) {
        th[t].job = &job;
        if (pthread_create(&tid[t], NULL, join_worker, &th[t])) { rc = -1; break; }
        started++;
    }
    int64_t total = 0;
    for (int t = 0; t < started; t++) {
        pthread_join(tid[t], NULL);
        if (th[t].rc) rc = -1;
        total += th[t].out.n;
        *arcs += th[t].arcs;
        *settled += th[t].settled;
    }
    orc_pair *all = NULL;
    if (!rc) {
        all = (orc_pair *)malloc((size_t)(total > 0 ? total : 1) * sizeof(orc_pair));
        if (!all) rc = -1;
    }
    int64_t pos = 0;
    for (int t = 0; t < started; t++) {
        if (!rc && th[t].out.n)
            memcpy(all + pos, th[t].out.a, (size_t)th[t].out.n * sizeof(orc_pair));
        pos += th[t].out.n;
        free(th[t].out.a);
    }
    free(th); free(tid); free(inS);
    if (rc) { free(all); *arcs = 0; *settled = 0; return -1; }
    qsort(all, (size_t)total, sizeof(orc_pair), pair_cmp);
    *out = all; *n_out = total;
    return 0;
}

/* ---------------- k closest pairs ---------------- */
/* Max-heap of pairs under (dist,u,v). */
typedef struct { orc_pair *a; int64_t n, k; } pairheap;

static void ph_sift_down(pairheap *h, int64_t i) {
    for (;;) {
        int64_t c = 2 * i + 1, m = i;
        if (c < h->n && pair_less(&h->a[m], &h->a[c])) m = c;
        if (c + 1 < h->n && pair_less(&h->a[m], &h->a[c + 1])) m = c + 1;
        if (m == i) return;
        orc_pair t = h->a[i]; h->a[i] = h->a[m]; h->a[m] = t;
        i = m;
    }
}

static void ph_offer(pairheap *h, orc_pair p) {
    if (h->n < h->k) {
        int64_t i = h->n++;
        while (i > 0) {
            int64_t q = (i - 1) / 2;
            if (!pair_less(&h->a[q], &p)) break;
            h->a[i] = h->a[q];
            i = q;
        }
        h->a[i] = p;
    } else if (pair_less(&p, &h->a[0])) {
        h->a[0] = p;
        ph_sift_down(h, 0);
    }
}

static uint64_t ph_bound(const pairheap *h) {
    return h->n == h->k ? (uint64_t)h->a[0].dist : (uint64_t)(ORC_UNREACH - 1u);
}

/* k-closest pairs under (dist,u,v); *out holds min(k, #reachable pairs) sorted. */
int orc_kcp_join(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                 const int32_t *R, int32_t nR, const int32_t *S, int32_t nS, int32_t k,
                 orc_pair **out, int64_t *n_out) {
    *out = NULL; *n_out = 0;
    if (V < 0 || nR < 0 || nS < 0 || k < 1 || check_ids(V, R, nR) || check_ids(V, S, nS)) return -1;
    uint8_t *inS = (uint8_t *)calloc((size_t)(V > 0 ? V : 1), 1);
    pairheap h = {(orc_pair *)malloc((size_t)k * sizeof(orc_pair)), 0, k};
    search_ws ws;
    int rc = (inS && h.a) ? ws_init(&ws, V, row_ptr, col, w) : -1;
    if (rc) { free(inS); free(h.a); return -1; }
    for (int32_t i = 0; i < nS; i++) inS[S[i]] = 1;
    for (int32_t i = 0; i < nR && !rc; i++) {
        int32_t u = R[i];
        ws.dist[u] = 0;
        ws.touched[ws.ntouched++] = u;
        if (mh_push(&ws.heap, 0, u)) { rc = -1; break; }
        while (ws.heap.n > 0) {
            hitem it = mh_pop(&ws.heap);
            if (it.d != ws.dist[it.x]) continue;
            if (it.d > ph_bound(&h)) break;
            int32_t x = it.x;
            if (inS[x]) { orc_pair p = {u, x, (uint32_t)it.d}; ph_offer(&h, p); }
            for (int32_t a = row_ptr[x]; a < row_ptr[x + 1]; a++) {
                int32_t y = col[a];
                uint64_t nd = it.d + w[a];
                if (nd > ph_bound(&h) || nd >= ws.dist[y]) continue;
                if (ws.dist[y] == ORC_UNREACH) ws.touched[ws.ntouched++] = y;
                ws.dist[y] = nd;
                if (mh_push(&ws.heap, nd, y)) { rc = -1; break; }
            }
            if (rc) break;
        }
        ws_reset(&ws);
    }
    ws_free(&ws);
    free(inS);
    if (rc) { free(h.a); return -1; }
    qsort(h.a, (size_t)h.n, sizeof(orc_pair), pair_cmp);
    *out = h.a; *n_out = h.n;
    return 0;
}

/* Single-source distances, cut off at `cutoff`: dist_out[x] = dist(src,x), or
 * ORC_UNREACH when it exceeds the cutoff.  Returns 0 or -1. */
int orc_sssp(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
             int32_t src, uint32_t cutoff, uint32_t *dist_out) {
    if (src < 0 || src >= V) return -1;
    if (cutoff > ORC_UNREACH - 1u) cutoff = ORC_UNREACH - 1u;
    search_ws ws;
    if (ws_init(&ws, V, row_ptr, col, w)) { ws_free(&ws); return -1; }
    int rc = 0;
    ws.dist[src] = 0;
    if (mh_push(&ws.heap, 0, src)) rc = -1;
    while (!rc && ws.heap.n > 0) {
        hitem it = mh_pop(&ws.heap);
        if (it.d != ws.dist[it.x]) continue;
        if (it.d > cutoff) break;
        for (int32_t a = row_ptr[it.x]; a < row_ptr[it.x + 1]; a++) {
            int32_t y = col[a];
            uint64_t nd = it.d + w[a];
            if (nd > cutoff || nd >= ws.dist[y]) continue;
            ws.dist[y] = nd;
            if (mh_push(&ws.heap, nd, y)) { rc = -1; break; }
        }
    }
    for (int32_t x = 0; x < V; x++)
        dist_out[x] = ws.dist[x] <= cutoff ? (uint32_t)ws.dist[x] : ORC_UNREACH;
    ws_free(&ws);
    return rc;
}

/* ---------------- objects on edges ----------------
 * Section 1: objects that move along the road network's edges, each given by
 * its distances from the two ends of the edge it is on, may form R or S.
 * Reading taken here (the paper gives no formula):
 *   - An object is named by an arc e = (a -> b, weight w) and its distance o
 *     from a along that arc, 0 <= o <= w.  Parallel arcs of equal tail, head
 *     and weight are one road: the object is on the first of them.
 *   - The road is two-way when an arc b -> a of the same weight exists (its
 *     twin: the first such arc other than the road's own, for a loop).  A road and its twin are one edge; an
 *     object on either is placed on the one with the smaller arc index, f,
 *     at distance s from f's tail (s = o, or w - o when it named the twin).
 *   - From an object on f = (a -> b, w) at s, b is reached at s' = w - s, and
 *     a at s when the road is two-way.  An object q on f_q = (c -> d, w_q) at
 *     s_q is reached from c by s_q more and, two-way, from d by w_q - s_q.
 *     Two objects on the same edge are also s_q - s_p apart along it when
 *     that is >= 0, and |s_p - s_q| apart on a two-way road.
 * dist(p, q) is the least of these: a path leaves p's edge at one of its
 * ends, follows the network (dist between vertices as for the vertex joins)
 * and enters q's edge at one of its ends, or stays on a shared edge.  The
 * object theta-join returns (i, j, dist) for R object i and S object j with
 * dist <= theta, sorted by (dist, i, j).
 */
typedef struct { int32_t f; uint32_t s, w; int32_t tail, head; int two_way; } orc_obj;

/* Place object (arc e, offset o); returns -1 for a bad arc or offset. */
static int obj_place(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                     int64_t A, int32_t e, uint32_t o, orc_obj *ob) {
    if (e < 0 || (int64_t)e >= A || o > w[e]) return -1;
    /* tail of e: the row holding it (binary search over row_ptr) */
    int32_t lo = 0, hi = V;
    while (hi - lo > 1) { int32_t mid = lo + (hi - lo) / 2; if (row_ptr[mid] <= e) lo = mid; else hi = mid; }
    int32_t a = lo, b = col[e];
    uint32_t wt = w[e];
    int32_t ec = e;                              /* first parallel arc of equal weight */
    for (int32_t x = row_ptr[a]; x < row_ptr[a + 1]; x++)
        if (col[x] == b && w[x] == wt) { ec = x; break; }
    int32_t tw = -1;                             /* first b -> a arc of the same weight, */
    for (int32_t x = row_ptr[b]; x < row_ptr[b + 1]; x++)   /* not the road's own arc (a loop) */
        if (col[x] == a && w[x] == wt && x != ec) { tw = x; break; }
    ob->w = wt;
    ob->two_way = tw >= 0;
    if (tw >= 0 && tw < ec) {                    /* the twin names the edge */
        ob->f = tw; ob->s = wt - o; ob->tail = b; ob->head = a;
    } else {
        ob->f = ec; ob->s = o; ob->tail = a; ob->head = b;
    }
    return 0;
}

int orc_object_join(int32_t V, const int32_t *row_ptr, const int32_t *col, const uint32_t *w,
                    const int32_t *Rarc, const uint32_t *Roff, int32_t nR,
                    const int32_t *Sarc, const uint32_t *Soff, int32_t nS, uint32_t theta,
                    orc_pair **out, int64_t *n_out) {
    *out = NULL; *n_out = 0;
    if (V < 1 || nR < 0 || nS < 0) return -1;
    const int64_t A = row_ptr[V];
    orc_obj *ro = (orc_obj *)malloc((size_t)(nR > 0 ? nR : 1) * sizeof(orc_obj));
    orc_obj *so = (orc_obj *)malloc((size_t)(nS > 0 ? nS : 1) * sizeof(orc_obj));
    search_ws ws;
    int rc = (ro && so) ? ws_init(&ws, V, row_ptr, col, w) : -1;
    if (rc) { free(ro); free(so); return -1; }
    for (int32_t i = 0; i < nR && !rc; i++) rc = obj_place(V, row_ptr, col, w, A, Rarc[i], Roff[i], &ro[i]);
    for (int32_t j = 0; j < nS && !rc; j++) rc = obj_place(V, row_ptr, col, w, A, Sarc[j], Soff[j], &so[j]);
    pairvec pv = {NULL, 0, 0};
    const uint64_t th = theta;
    for (int32_t i = 0; i < nR && !rc; i++) {
        const orc_obj *p = &ro[i];
        /* Dijkstra from the object's exits: its edge's head at w - s, and its
         * tail at s on a two-way road; cut off at theta */
        const uint64_t eh = (uint64_t)p->w - p->s, et = p->s;
        if (eh <= th) {
            ws.dist[p->head] = eh;
            ws.touched[ws.ntouched++] = p->head;
            if (mh_push(&ws.heap, eh, p->head)) rc = -1;
        }
        if (!rc && p->two_way && et <= th && et < ws.dist[p->tail]) {
            if (ws.dist[p->tail] == ORC_UNREACH) ws.touched[ws.ntouched++] = p->tail;
            ws.dist[p->tail] = et;
            if (mh_push(&ws.heap, et, p->tail)) rc = -1;
        }
        while (!rc && ws.heap.n > 0) {
            hitem it = mh_pop(&ws.heap);
            if (it.d != ws.dist[it.x]) continue;
            if (it.d > th) break;
            for (int32_t a = row_ptr[it.x]; a < row_ptr[it.x + 1]; a++) {
                int32_t y = col[a];
                uint64_t nd = it.d + w[a];
                if (nd > th || nd >= ws.dist[y]) continue;
                if (ws.dist[y] == ORC_UNREACH) ws.touched[ws.ntouched++] = y;
                ws.dist[y] = nd;
                if (mh_push(&ws.heap, nd, y)) { rc = -1; break; }
            }
        }
        /* every S object: enter its edge at either end, or share p's edge */
        for (int32_t j = 0; j < nS && !rc; j++) {
            const orc_obj *q = &so[j];
            uint64_t best = ORC_UNREACH;
            if (ws.dist[q->tail] != ORC_UNREACH && ws.dist[q->tail] + q->s < best) best = ws.dist[q->tail] + q->s;
            if (q->two_way && ws.dist[q->head] != ORC_UNREACH && ws.dist[q->head] + (q->w - q->s) < best)
                best = ws.dist[q->head] + (q->w - q->s);
            if (q->f == p->f) {
                if (q->s >= p->s && (uint64_t)(q->s - p->s) < best) best = q->s - p->s;
                if (p->two_way && p->s >= q->s && (uint64_t)(p->s - q->s) < best) best = p->s - q->s;
            }
            if (best <= th && pv_push(&pv, i, j, (uint32_t)best)) rc = -1;
        }
        /* dist entries beyond theta were never set, so the reset covers all */
        ws_reset(&ws);
    }
    ws_free(&ws);
    free(ro);
    free(so);
    if (rc) { free(pv.a); return -1; }
    qsort(pv.a, (size_t)pv.n, sizeof(orc_pair), pair_cmp);
    *out = pv.a; *n_out = pv.n;
    return 0;
}

void orc_free(void *p) { free(p); }
