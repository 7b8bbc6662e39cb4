/*
 * CPU oracle for full-neighbourhood move evaluation in VRP local search.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use this file.  It shares no code, header, table or
 * helper with the device library.
 *
 * What it computes is the plain definition of the result (no blocking, no
 * incremental attributes, no concatenation algebra):
 *
 *   for every move m of the canonical move space N(S)
 *       build the touched routes of S' = m(S) explicitly (erase / insert /
 *       reverse / exchange on node lists),
 *       recompute each touched route from scratch:
 *         distance  = sum of c_ij over consecutive nodes, both depot edges
 *                     included (the objective with mu1 = 0, mu2 = 1; Section 2,
 *                     eq. objective),
 *         load      = the largest load carried: the sum of delivery demands
 *                     (the vehicle leaves with them and only unloads); with
 *                     pickups (VRPSPDTW) the largest load over the depot
 *                     departure and every customer after unloading its
 *                     delivery and loading its pickup; feasible iff <= capacity
 *                     (Section 2; Section 4.3.2 load attributes),
 *         windows   = forward simulation: leave the depot at e_0, wait when
 *                     early, infeasible when arriving after l_i, back at the
 *                     depot by l_0 (Section 2),
 *       delta(m) = sum of new distances - sum of old distances of the touched
 *                  route slots,
 *       feas(m)  = bit0 capacity of every touched route, bit1 windows of
 *                  every touched route (always 1 when windows are off),
 *   best = lexicographic minimum of (delta, id) over moves with feas == 3
 *          (Section 5.3.4, eq. scoring_tensor / eq. mask / eq. min_obj with
 *          the score equal to the distance delta and an infinite score for
 *          infeasible moves; lowest id breaks ties).
 *
 * Penalised mode (feasible and infeasible search, Alg. A2; the scoring
 * function of eq. scoring_tensor read as a weighted sum of the three
 * attribute deltas of Section 5.3.3): every move of N(S) is admissible and
 * scores
 *       score(m) = dD + w_L * dL_V + w_T * dT_V
 * over the touched route slots, where for one route
 *       L_V = max(load - capacity, 0)                      (load excess),
 *       T_V = time warp of the forward simulation: leave the depot at e_0,
 *             wait when early, and when arriving after l_i pay the lateness
 *             as warp and start service at l_i; arriving back after l_0 pays
 *             the lateness too (the time-warp technique of Section 4.3.3).
 * best = lexicographic minimum of (score, id) over all moves.
 *
 * Granular mode (edge-based neighbourhood reduction, Section 5.3.1 edge-based
 * extraction with the granularity threshold theta of the experiments): node
 * j is a neighbour of node i when it is among the theta nodes closest to i
 * (distance, then node id; the depot is node 0 and every start depot of a
 * route stands for it); the mask keeps the pairs {i, j} where either is a
 * neighbour of the other.  The inter-route moves (RELOCATE, SWAP of
 * customers in different routes, 2OPT*) are kept only when the nodes of
 * their two refs form such a pair; intra-route moves (2OPT, OR-OPT, SWAP
 * within a route) are all kept.
 *
 * Operators (Section 4.1, Fig. 2; the move space is the reading recorded in
 * the design notes):
 *   op 0 RELOCATE  k=1  a = customer u, b = any ref v of another route:
 *                       u leaves its route and is inserted right after v.
 *   op 1 SWAP      k=1  a < b customers (same or different routes):
 *                       u and v exchange places.
 *   op 2 2OPT*     k=0  a < b refs of different routes: the two tails after
 *                       them are exchanged; each head keeps its slot.
 *   op 3 2OPT      k=0  a < b customers of one route: the part between them
 *                       (inclusive) is reversed.
 *   op 4 OR-OPT    k=1..3  a = customer starting a k-node segment, b = ref of
 *                       the same route not inside [pred(a), last of segment]:
 *                       the segment is moved, in its orientation, to right
 *                       after b.
 * Operator variants (the extensions Section 4.1 and Section 7 name: segments
 * of N > 1 nodes in inter-route moves, reversed insertion, cross-exchange):
 *   op 5 SEGMENT RELOCATE   k=2,3  the k-node segment starting at customer a
 *                       moves, orientation kept, right after ref b of another
 *                       route.
 *   op 6 REVERSED RELOCATE  k=2,3  the same with the segment reversed.
 *   op 7..9 CROSS-EXCHANGE  the segment of op-6 nodes starting at customer a
 *                       and the segment of k = 1..3 nodes starting at customer
 *                       b (a < b, different routes) exchange places, each in
 *                       its orientation; op 7 with k = 1 is SWAP and is left
 *                       out.
 * Refs: customer c -> c - 1; start depot of route r -> n + r; Q = n + R.
 * Move id = ((op * 4 + k) * Q + a) * Q + b.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef struct {
    int n;
    const int32_t *D;     /* (n+1) x (n+1), row-major */
    const int32_t *node4; /* (n+1) x {demand, e, l, s} */
    int64_t cap;
    int has_tw;
    const int32_t *pick;  /* (n+1) pickup amounts (VRPSPDTW), or NULL */
} Inst;

typedef struct {
    int R;
    const int32_t *off;  /* R + 1 */
    const int32_t *cust; /* n */
} Sol;

typedef struct {
    int64_t delta;
    uint32_t id;
    int32_t feas;
    int32_t found;
} Best;

static inline int64_t dist(const Inst *I, int i, int j) {
    return I->D[(int64_t)i * (I->n + 1) + j];
}

/* Distance of the closed route 0, c[0], ..., c[L-1], 0. */
static int64_t route_distance(const Inst *I, const int32_t *c, int L) {
    int64_t d = 0;
    int prev = 0;
    for (int i = 0; i < L; i++) {
        d += dist(I, prev, c[i]);
        prev = c[i];
    }
    return d + dist(I, prev, 0);
}

/* The largest load the vehicle carries on the route.  Without pickups the
 * vehicle leaves the depot with all deliveries and only unloads, so this is
 * the sum of the demands.  With pickups (VRPSPDTW, Section 2) it leaves with
 * all deliveries, and at each customer unloads its delivery and loads its
 * pickup; every point of the route counts (Section 4.3.2). */
static int64_t route_load(const Inst *I, const int32_t *c, int L) {
    int64_t q = 0;
    for (int i = 0; i < L; i++) q += I->node4[4 * c[i] + 0];
    if (!I->pick) return q;
    int64_t peak = q;
    for (int i = 0; i < L; i++) {
        q += I->pick[c[i]] - I->node4[4 * c[i] + 0];
        if (q > peak) peak = q;
    }
    return peak;
}

/* Hard time windows, simulated forward (Section 2). */
static int route_windows_ok(const Inst *I, const int32_t *c, int L) {
    if (!I->has_tw) return 1;
    const int32_t *nd = I->node4;
    int64_t t = nd[1]; /* service start at the depot = e_0 */
    int prev = 0;
    for (int i = 0; i < L; i++) {
        int x = c[i];
        int64_t arrive = t + nd[4 * prev + 3] + dist(I, prev, x);
        if (arrive > nd[4 * x + 2]) return 0;
        t = arrive > nd[4 * x + 1] ? arrive : nd[4 * x + 1];
        prev = x;
    }
    int64_t back = t + nd[4 * prev + 3] + dist(I, prev, 0);
    return back <= nd[2];
}

/* Load excess of a route (penalised mode). */
static int64_t route_load_excess(const Inst *I, const int32_t *c, int L) {
    int64_t q = route_load(I, c, L);
    return q > I->cap ? q - I->cap : 0;
}

/* Time warp of a route, simulated forward (penalised mode; 0 without
 * windows). */
static int64_t route_time_warp(const Inst *I, const int32_t *c, int L) {
    if (!I->has_tw) return 0;
    const int32_t *nd = I->node4;
    int64_t t = nd[1], warp = 0;
    int prev = 0;
    for (int i = 0; i < L; i++) {
        int x = c[i];
        int64_t arrive = t + nd[4 * prev + 3] + dist(I, prev, x);
        if (arrive > nd[4 * x + 2]) {
            warp += arrive - nd[4 * x + 2];
            t = nd[4 * x + 2];
        } else {
            t = arrive > nd[4 * x + 1] ? arrive : nd[4 * x + 1];
        }
        prev = x;
    }
    int64_t back = t + nd[4 * prev + 3] + dist(I, prev, 0);
    if (back > nd[2]) warp += back - nd[2];
    return warp;
}

static int route_feas(const Inst *I, const int32_t *c, int L) {
    int f = 0;
    if (route_load(I, c, L) <= I->cap) f |= 1;
    if (route_windows_ok(I, c, L)) f |= 2;
    return f;
}

/* ------------------------------------------------------------------ moves */

typedef struct {
    int op, k, a, b;
} Move;

static uint32_t move_id(int Q, int op, int k, int a, int b) {
    return (uint32_t)((((uint64_t)(op * 4 + k) * Q + a) * Q) + b);
}

static Move move_decode(int Q, uint32_t id) {
    Move m;
    uint64_t qq = (uint64_t)Q * Q;
    uint64_t opk = id / qq, rem = id % qq;
    m.op = (int)(opk / 4);
    m.k = (int)(opk % 4);
    m.a = (int)(rem / Q);
    m.b = (int)(rem % Q);
    return m;
}

/* Where every node sits: route and 1-based position (0 = start depot). */
typedef struct {
    int n, R, Q;
    int32_t *route_of; /* by customer id, 1..n */
    int32_t *pos_of;
    int64_t *rdist;    /* current distance per route */
    int64_t *rlv;      /* current load excess per route */
    int64_t *rtv;      /* current time warp per route */
} Index;

static void index_build(const Inst *I, const Sol *S, Index *X) {
    X->n = I->n;
    X->R = S->R;
    X->Q = I->n + S->R;
    X->route_of = calloc((size_t)I->n + 1, sizeof(int32_t));
    X->pos_of = calloc((size_t)I->n + 1, sizeof(int32_t));
    X->rdist = calloc((size_t)S->R + 1, sizeof(int64_t));
    X->rlv = calloc((size_t)S->R + 1, sizeof(int64_t));
    X->rtv = calloc((size_t)S->R + 1, sizeof(int64_t));
    for (int r = 0; r < S->R; r++) {
        int L = S->off[r + 1] - S->off[r];
        for (int p = 0; p < L; p++) {
            int c = S->cust[S->off[r] + p];
            X->route_of[c] = r;
            X->pos_of[c] = p + 1;
        }
        X->rdist[r] = route_distance(I, S->cust + S->off[r], L);
        X->rlv[r] = route_load_excess(I, S->cust + S->off[r], L);
        X->rtv[r] = route_time_warp(I, S->cust + S->off[r], L);
    }
}

static void index_free(Index *X) {
    free(X->route_of);
    free(X->pos_of);
    free(X->rdist);
    free(X->rlv);
    free(X->rtv);
}

/* Route and position of a ref. */
static void ref_where(const Index *X, int ref, int *r, int *p) {
    if (ref < X->n) {
        *r = X->route_of[ref + 1];
        *p = X->pos_of[ref + 1];
    } else {
        *r = ref - X->n;
        *p = 0;
    }
}

/* Literal list edits.  Each writes the new customer list(s) of the touched
 * route slot(s) and returns how many slots it touched (1 or 2).  out1 gets
 * slot *r1, out2 gets slot *r2.  Buffers hold at least n entries. */
static int find_node(const int32_t *c, int L, int node) {
    for (int i = 0; i < L; i++)
        if (c[i] == node) return i;
    return -1;
}

static int edit_move(const Inst *I, const Sol *S, const Index *X, Move m,
                     int *r1, int32_t *out1, int *L1, int *r2, int32_t *out2, int *L2) {
    const int n = I->n;
    int ra, pa, rb, pb;
    ref_where(X, m.a, &ra, &pa);
    ref_where(X, m.b, &rb, &pb);
    const int32_t *A = S->cust + S->off[ra];
    const int LA = S->off[ra + 1] - S->off[ra];
    const int32_t *B = S->cust + S->off[rb];
    const int LB = S->off[rb + 1] - S->off[rb];
    *r1 = ra;
    *r2 = rb;
    if (m.op == 0) { /* RELOCATE u after v, other route */
        int u = m.a + 1;
        int l = 0;
        for (int i = 0; i < LA; i++)
            if (A[i] != u) out1[l++] = A[i];
        *L1 = l;
        l = 0;
        if (m.b >= n) out2[l++] = u; /* after the start depot */
        for (int i = 0; i < LB; i++) {
            out2[l++] = B[i];
            if (B[i] == m.b + 1) out2[l++] = u;
        }
        *L2 = l;
        return 2;
    }
    if (m.op == 1) { /* SWAP u and v */
        int u = m.a + 1, v = m.b + 1;
        if (ra == rb) {
            memcpy(out1, A, sizeof(int32_t) * LA);
            int iu = find_node(out1, LA, u), iv = find_node(out1, LA, v);
            out1[iu] = v;
            out1[iv] = u;
            *L1 = LA;
            return 1;
        }
        memcpy(out1, A, sizeof(int32_t) * LA);
        memcpy(out2, B, sizeof(int32_t) * LB);
        out1[find_node(out1, LA, u)] = v;
        out2[find_node(out2, LB, v)] = u;
        *L1 = LA;
        *L2 = LB;
        return 2;
    }
    if (m.op == 2) { /* 2OPT*: head(a) + tail after b ; head(b) + tail after a */
        int l = 0;
        for (int i = 0; i < pa; i++) out1[l++] = A[i];
        for (int i = pb; i < LB; i++) out1[l++] = B[i];
        *L1 = l;
        l = 0;
        for (int i = 0; i < pb; i++) out2[l++] = B[i];
        for (int i = pa; i < LA; i++) out2[l++] = A[i];
        *L2 = l;
        return 2;
    }
    if (m.op == 3) { /* 2OPT: reverse positions lo..hi */
        int lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
        memcpy(out1, A, sizeof(int32_t) * LA);
        for (int i = lo - 1, j = hi - 1; i < j; i++, j--) {
            int32_t t = out1[i];
            out1[i] = out1[j];
            out1[j] = t;
        }
        *L1 = LA;
        return 1;
    }
    if (m.op == 5 || m.op == 6) { /* segment of k from route A to right after b in route B */
        const int k = m.k;
        int32_t seg[3];
        for (int q = 0; q < k; q++) seg[q] = A[pa - 1 + (m.op == 5 ? q : k - 1 - q)];
        int l = 0;
        for (int i = 0; i < LA; i++)
            if (i < pa - 1 || i >= pa - 1 + k) out1[l++] = A[i];
        *L1 = l;
        l = 0;
        if (m.b >= n)
            for (int q = 0; q < k; q++) out2[l++] = seg[q];
        for (int i = 0; i < LB; i++) {
            out2[l++] = B[i];
            if (B[i] == m.b + 1)
                for (int q = 0; q < k; q++) out2[l++] = seg[q];
        }
        *L2 = l;
        return 2;
    }
    if (m.op >= 7) { /* cross-exchange: segment (a, op-6) <-> segment (b, k) */
        const int ka = m.op - 6, kb = m.k;
        int l = 0;
        for (int i = 0; i < pa - 1; i++) out1[l++] = A[i];
        for (int q = 0; q < kb; q++) out1[l++] = B[pb - 1 + q];
        for (int i = pa - 1 + ka; i < LA; i++) out1[l++] = A[i];
        *L1 = l;
        l = 0;
        for (int i = 0; i < pb - 1; i++) out2[l++] = B[i];
        for (int q = 0; q < ka; q++) out2[l++] = A[pa - 1 + q];
        for (int i = pb - 1 + kb; i < LB; i++) out2[l++] = B[i];
        *L2 = l;
        return 2;
    }
    /* op 4 OR-OPT: remove segment of k starting at a, reinsert after b */
    {
        int k = m.k;
        int32_t seg[3];
        for (int q = 0; q < k; q++) seg[q] = A[pa - 1 + q];
        int32_t rest[LA > 0 ? LA : 1];
        int l = 0;
        for (int i = 0; i < LA; i++)
            if (i < pa - 1 || i >= pa - 1 + k) rest[l++] = A[i];
        int o = 0;
        if (m.b >= n)
            for (int q = 0; q < k; q++) out1[o++] = seg[q];
        for (int i = 0; i < l; i++) {
            out1[o++] = rest[i];
            if (rest[i] == m.b + 1)
                for (int q = 0; q < k; q++) out1[o++] = seg[q];
        }
        *L1 = o;
        return 1;
    }
}

/* --------------------------------------------------------- enumeration --- */

typedef struct {
    const Inst *I;
    const Sol *S;
    const Index *X;
    uint32_t op_mask;
    const uint8_t *gran; /* (n+1) x (n+1) pair mask, or NULL for the full neighbourhood */
    int pen;             /* penalised mode */
    int64_t w_load, w_tw;
    int32_t *dump_delta;
    uint8_t *dump_feas;
    int64_t *count;      /* per-thread move counts */
    Best *best;          /* per-thread */
    Best *pair;          /* multi-move: per thread, R x R best improving move per route pair, or NULL */
    int ntasks;
    int next_task;       /* atomic */
    int nthreads;
} Ctx;

typedef struct {
    Ctx *C;
    int tid;
} Arg;

static void consider(Ctx *C, int tid, Move m, int32_t *b1, int32_t *b2) {
    const Inst *I = C->I;
    int r1, r2, L1, L2;
    int touched = edit_move(I, C->S, C->X, m, &r1, b1, &L1, &r2, b2, &L2);
    int64_t delta = route_distance(I, b1, L1) - C->X->rdist[r1];
    int feas = route_feas(I, b1, L1);
    if (touched == 2) {
        delta += route_distance(I, b2, L2) - C->X->rdist[r2];
        feas &= route_feas(I, b2, L2);
    }
    if (C->pen) {
        int64_t dlv = route_load_excess(I, b1, L1) - C->X->rlv[r1];
        int64_t dtv = route_time_warp(I, b1, L1) - C->X->rtv[r1];
        if (touched == 2) {
            dlv += route_load_excess(I, b2, L2) - C->X->rlv[r2];
            dtv += route_time_warp(I, b2, L2) - C->X->rtv[r2];
        }
        delta += C->w_load * dlv + C->w_tw * dtv;  /* the score */
    }
    uint32_t id = move_id(C->X->Q, m.op, m.k, m.a, m.b);
    if (C->dump_delta) C->dump_delta[id] = (int32_t)delta;
    if (C->dump_feas) C->dump_feas[id] = (uint8_t)feas;
    C->count[tid]++;
    if (C->pair && (feas == 3 || C->pen) && delta < 0) {
        int lo = touched == 2 && r2 < r1 ? r2 : r1, hi = touched == 2 && r2 > r1 ? r2 : r1;
        const int R = C->X->R;
        Best *pb = &C->pair[((size_t)tid * R + lo) * R + hi];
        if (!pb->found || delta < pb->delta || (delta == pb->delta && id < pb->id)) {
            pb->found = 1;
            pb->delta = delta;
            pb->id = id;
            pb->feas = feas;
        }
    }
    if (feas == 3 || C->pen) {
        Best *bt = &C->best[tid];
        if (!bt->found || delta < bt->delta || (delta == bt->delta && id < bt->id)) {
            bt->found = 1;
            bt->delta = delta;
            bt->id = id;
            bt->feas = feas;
        }
    }
}

static int ref_node(const Index *X, int ref) { return ref < X->n ? ref + 1 : 0; }

/* Granular mask test of an inter-route move's refs (1 without a mask). */
static int gran_ok(const Ctx *C, int a, int b) {
    if (!C->gran) return 1;
    const int n = C->I->n;
    return C->gran[(size_t)ref_node(C->X, a) * (n + 1) + ref_node(C->X, b)];
}

/* Task t covers operator op = t / n and first ref a = t % n (customers), or
 * for 2OPT* any first ref; OR-OPT tasks run over (k, a). */
static void run_task(Ctx *C, int tid, int t, int32_t *b1, int32_t *b2) {
    const int n = C->I->n, Q = C->X->Q, R = C->X->R;
    const Sol *S = C->S;
    const Index *X = C->X;
    int op = t / Q, a = t % Q;
    if (op > 11) return;
    if (op == 0 && (C->op_mask & 1) && a < n) {
        int ra = X->route_of[a + 1];
        for (int b = 0; b < Q; b++) {
            int rb, pb;
            ref_where(X, b, &rb, &pb);
            if (rb == ra || !gran_ok(C, a, b)) continue;
            consider(C, tid, (Move){0, 1, a, b}, b1, b2);
        }
    } else if (op == 1 && (C->op_mask & 2) && a < n) {
        for (int b = a + 1; b < n; b++) {
            if (X->route_of[a + 1] != X->route_of[b + 1] && !gran_ok(C, a, b)) continue;
            consider(C, tid, (Move){1, 1, a, b}, b1, b2);
        }
    } else if (op == 2 && (C->op_mask & 4)) {
        int ra, pa;
        ref_where(X, a, &ra, &pa);
        for (int b = a + 1; b < Q; b++) {
            int rb, pb;
            ref_where(X, b, &rb, &pb);
            if (rb == ra || !gran_ok(C, a, b)) continue;
            consider(C, tid, (Move){2, 0, a, b}, b1, b2);
        }
    } else if (op == 3 && (C->op_mask & 8) && a < n) {
        int ra = X->route_of[a + 1];
        for (int b = a + 1; b < n; b++)
            if (X->route_of[b + 1] == ra) consider(C, tid, (Move){3, 0, a, b}, b1, b2);
    } else if ((op == 7 || op == 8) && (C->op_mask & (32 | 64)) && a < n) {
        int k = op - 5; /* 2, 3 */
        int ra = X->route_of[a + 1], pa = X->pos_of[a + 1];
        if (pa + k - 1 > S->off[ra + 1] - S->off[ra]) return;
        for (int b = 0; b < Q; b++) {
            int rb, pb;
            ref_where(X, b, &rb, &pb);
            if (rb == ra) continue;
            if (C->op_mask & 32) consider(C, tid, (Move){5, k, a, b}, b1, b2);
            if (C->op_mask & 64) consider(C, tid, (Move){6, k, a, b}, b1, b2);
        }
    } else if (op >= 9 && (C->op_mask & 128) && a < n) {
        int ka = op - 8; /* 1..3 */
        int ra = X->route_of[a + 1], pa = X->pos_of[a + 1];
        if (pa + ka - 1 > S->off[ra + 1] - S->off[ra]) return;
        for (int b = a + 1; b < n; b++) {
            int rb = X->route_of[b + 1], pb = X->pos_of[b + 1];
            if (rb == ra) continue;
            int Lb = S->off[rb + 1] - S->off[rb];
            for (int kb = 1; kb <= 3; kb++) {
                if (ka == 1 && kb == 1) continue;
                if (pb + kb - 1 > Lb) break;
                consider(C, tid, (Move){6 + ka, kb, a, b}, b1, b2);
            }
        }
    } else if (op >= 4 && op <= 6 && (C->op_mask & 16) && a < n) {
        int k = op - 3; /* 1..3 */
        int r = X->route_of[a + 1], i = X->pos_of[a + 1];
        int L = S->off[r + 1] - S->off[r];
        if (i + k - 1 > L) return;
        for (int j = 0; j <= L; j++) {
            if (j >= i - 1 && j <= i + k - 1) continue;
            int b = j == 0 ? n + r : S->cust[S->off[r] + j - 1] - 1;
            consider(C, tid, (Move){4, k, a, b}, b1, b2);
        }
    }
    (void)R;
}

static void *worker(void *p) {
    Arg *A = (Arg *)p;
    Ctx *C = A->C;
    int32_t *b1 = malloc(sizeof(int32_t) * (C->I->n + 4));
    int32_t *b2 = malloc(sizeof(int32_t) * (C->I->n + 4));
    for (;;) {
        int t = __atomic_fetch_add(&C->next_task, 1, __ATOMIC_RELAXED);
        if (t >= C->ntasks) break;
        run_task(C, A->tid, t, b1, b2);
    }
    free(b1);
    free(b2);
    return NULL;
}

static int resolve_threads(int nthreads) {
    if (nthreads > 0) return nthreads;
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* ------------------------------------------------------------ exported --- */

/* Evaluate N(S) restricted to op_mask.  Returns 1 if an admissible move
 * exists (written to *best_*), 0 otherwise.  Optional dumps are indexed by
 * move id and must hold 20 * Q * Q entries (40 * Q * Q with ops 5..9); entries that are not moves are
 * left untouched.  *moves receives |N(S)| for the enabled operators. */
static int eval_core2(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                      int has_tw, int R, const int32_t *off, const int32_t *cust, uint32_t op_mask,
                      const uint8_t *gran, int pen, int64_t w_load, int64_t w_tw,
                      int nthreads, int32_t *dump_delta, uint8_t *dump_feas,
                      int64_t *best_delta, uint32_t *best_id, int64_t *moves, Best *pair_out);

static int eval_core(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                     int has_tw, int R, const int32_t *off, const int32_t *cust, uint32_t op_mask,
                     const uint8_t *gran, int pen, int64_t w_load, int64_t w_tw,
                     int nthreads, int32_t *dump_delta, uint8_t *dump_feas,
                     int64_t *best_delta, uint32_t *best_id, int64_t *moves) {
    return eval_core2(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, gran, pen, w_load, w_tw, nthreads,
                      dump_delta, dump_feas, best_delta, best_id, moves, NULL);
}

/* As eval_core; pair_out (R x R, nullable) receives for every pair of route
 * slots r1 <= r2 the best admissible improving move that touches exactly
 * those routes (r1 = r2: one route). */
static int eval_core2(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                      int has_tw, int R, const int32_t *off, const int32_t *cust, uint32_t op_mask,
                      const uint8_t *gran, int pen, int64_t w_load, int64_t w_tw,
                      int nthreads, int32_t *dump_delta, uint8_t *dump_feas,
                      int64_t *best_delta, uint32_t *best_id, int64_t *moves, Best *pair_out) {
    Inst I = {n, D, node4, cap, has_tw, pick};
    Sol S = {R, off, cust};
    Index X;
    index_build(&I, &S, &X);
    int T = resolve_threads(nthreads);
    Ctx C;
    memset(&C, 0, sizeof C);
    C.I = &I;
    C.S = &S;
    C.X = &X;
    C.op_mask = op_mask;
    C.gran = gran;
    C.pen = pen;
    C.w_load = w_load;
    C.w_tw = w_tw;
    C.dump_delta = dump_delta;
    C.dump_feas = dump_feas;
    C.nthreads = T;
    C.ntasks = 12 * X.Q;
    C.best = calloc((size_t)T, sizeof(Best));
    C.count = calloc((size_t)T, sizeof(int64_t));
    if (pair_out) C.pair = calloc((size_t)T * R * R, sizeof(Best));
    pthread_t *th = malloc(sizeof(pthread_t) * T);
    Arg *args = malloc(sizeof(Arg) * T);
    for (int t = 0; t < T; t++) {
        args[t].C = &C;
        args[t].tid = t;
        if (T == 1)
            worker(&args[0]);
        else
            pthread_create(&th[t], NULL, worker, &args[t]);
    }
    if (T > 1)
        for (int t = 0; t < T; t++) pthread_join(th[t], NULL);
    Best b = {0, 0, 0, 0};
    int64_t total = 0;
    for (int t = 0; t < T; t++) {
        total += C.count[t];
        Best *x = &C.best[t];
        if (!x->found) continue;
        if (!b.found || x->delta < b.delta || (x->delta == b.delta && x->id < b.id)) b = *x;
    }
    if (moves) *moves = total;
    if (b.found) {
        *best_delta = b.delta;
        *best_id = b.id;
    }
    if (pair_out) {
        for (size_t q = 0; q < (size_t)R * R; q++) {
            Best m = {0, 0, 0, 0};
            for (int t = 0; t < T; t++) {
                Best *x = &C.pair[(size_t)t * R * R + q];
                if (x->found && (!m.found || x->delta < m.delta || (x->delta == m.delta && x->id < m.id))) m = *x;
            }
            pair_out[q] = m;
        }
        free(C.pair);
    }
    free(th);
    free(args);
    free(C.best);
    free(C.count);
    index_free(&X);
    return b.found;
}

int oracle_eval(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                int R, const int32_t *off, const int32_t *cust, uint32_t op_mask,
                int nthreads, int32_t *dump_delta, uint8_t *dump_feas,
                int64_t *best_delta, uint32_t *best_id, int64_t *moves) {
    return eval_core(n, D, node4, NULL, cap, has_tw, R, off, cust, op_mask, NULL, 0, 0, 0, nthreads,
                     dump_delta, dump_feas, best_delta, best_id, moves);
}

/* Penalised mode: as oracle_eval, but every move is admissible, the dumped
 * and returned value is the score dD + w_load * dL_V + w_tw * dT_V, and
 * dump_feas still holds the hard capacity / window bits of the touched
 * routes.  Returns 1 when N(S) has a move. */
int oracle_eval_pen(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                    int R, const int32_t *off, const int32_t *cust, uint32_t op_mask,
                    int64_t w_load, int64_t w_tw, int nthreads, int32_t *dump_score,
                    uint8_t *dump_feas, int64_t *best_score, uint32_t *best_id, int64_t *moves) {
    return eval_core(n, D, node4, NULL, cap, has_tw, R, off, cust, op_mask, NULL, 1, w_load, w_tw, nthreads,
                     dump_score, dump_feas, best_score, best_id, moves);
}

/* Apply move `id` to (off, cust) in place.  Returns 0 on success, -1 if the
 * id does not name a move of N(S). */
int oracle_apply(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                 int R, int32_t *off, int32_t *cust, uint32_t id) {
    Inst I = {n, D, node4, cap, has_tw, NULL};
    Sol S = {R, off, cust};
    Index X;
    index_build(&I, &S, &X);
    int Q = X.Q;
    Move m = move_decode(Q, id);
    int ok = 1;
    if (m.a >= Q || m.b >= Q || m.op > 9) ok = 0;
    int ra = 0, pa = 0, rb = 0, pb = 0;
    if (ok) {
        ref_where(&X, m.a, &ra, &pa);
        ref_where(&X, m.b, &rb, &pb);
        int La = off[ra + 1] - off[ra];
        switch (m.op) {
        case 0: ok = m.k == 1 && m.a < n && rb != ra; break;
        case 1: ok = m.k == 1 && m.a < m.b && m.b < n; break;
        case 2: ok = m.k == 0 && m.a < m.b && ra != rb; break;
        case 3: ok = m.k == 0 && m.a < m.b && m.b < n && ra == rb; break;
        case 4:
            ok = m.k >= 1 && m.k <= 3 && m.a < n && ra == rb && pa + m.k - 1 <= La &&
                 !(pb >= pa - 1 && pb <= pa + m.k - 1);
            break;
        case 5:
        case 6: ok = m.k >= 2 && m.k <= 3 && m.a < n && ra != rb && pa + m.k - 1 <= La; break;
        default: {
            const int Lb = off[rb + 1] - off[rb];
            ok = m.k >= 1 && m.k <= 3 && m.a < m.b && m.b < n && ra != rb && pa + (m.op - 6) - 1 <= La &&
                 pb + m.k - 1 <= Lb && !(m.op == 7 && m.k == 1);
            break;
        }
        }
    }
    if (!ok) {
        index_free(&X);
        return -1;
    }
    int32_t *b1 = malloc(sizeof(int32_t) * (n + 4));
    int32_t *b2 = malloc(sizeof(int32_t) * (n + 4));
    int r1, r2, L1, L2;
    int touched = edit_move(&I, &S, &X, m, &r1, b1, &L1, &r2, b2, &L2);
    /* Rebuild the whole CSR with the touched slots replaced. */
    int32_t *noff = malloc(sizeof(int32_t) * (R + 1));
    int32_t *ncust = malloc(sizeof(int32_t) * (n + 1));
    int w = 0;
    for (int r = 0; r < R; r++) {
        noff[r] = w;
        if (r == r1) {
            memcpy(ncust + w, b1, sizeof(int32_t) * L1);
            w += L1;
        } else if (touched == 2 && r == r2) {
            memcpy(ncust + w, b2, sizeof(int32_t) * L2);
            w += L2;
        } else {
            int L = off[r + 1] - off[r];
            memcpy(ncust + w, cust + off[r], sizeof(int32_t) * L);
            w += L;
        }
    }
    noff[R] = w;
    memcpy(off, noff, sizeof(int32_t) * (R + 1));
    memcpy(cust, ncust, sizeof(int32_t) * n);
    free(noff);
    free(ncust);
    free(b1);
    free(b2);
    index_free(&X);
    return 0;
}

/* Total distance of S (eq. objective, mu1 = 0, mu2 = 1) and the number of
 * routes that violate capacity (*cap_bad) or windows (*tw_bad). */
int64_t oracle_cost(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                    int R, const int32_t *off, const int32_t *cust, int *cap_bad, int *tw_bad) {
    Inst I = {n, D, node4, cap, has_tw, NULL};
    int64_t c = 0;
    int cb = 0, tb = 0;
    for (int r = 0; r < R; r++) {
        int L = off[r + 1] - off[r];
        c += route_distance(&I, cust + off[r], L);
        int f = route_feas(&I, cust + off[r], L);
        if (!(f & 1)) cb++;
        if (!(f & 2)) tb++;
    }
    if (cap_bad) *cap_bad = cb;
    if (tw_bad) *tw_bad = tb;
    return c;
}

/* Check mode: for every move, build the whole S' and recompute its full
 * cost; count moves where cost(S') - cost(S) differs from the dumped delta.
 * dump_delta must come from oracle_eval on the same (S, op_mask). */
int64_t oracle_check_full(int n, const int32_t *D, const int32_t *node4, int64_t cap,
                          int has_tw, int R, const int32_t *off, const int32_t *cust,
                          const int32_t *dump_delta, const uint8_t *dump_feas,
                          uint32_t op_mask, int64_t sample_every) {
    Inst I = {n, D, node4, cap, has_tw, NULL};
    Sol S = {R, off, cust};
    Index X;
    index_build(&I, &S, &X);
    int64_t base = oracle_cost(n, D, node4, cap, has_tw, R, off, cust, NULL, NULL);
    int Q = X.Q;
    uint64_t total = 20ull * Q * Q;
    int32_t *o2 = malloc(sizeof(int32_t) * (R + 1));
    int32_t *c2 = malloc(sizeof(int32_t) * (n + 1));
    int64_t bad = 0, seen = 0;
    for (uint64_t id = 0; id < total; id++) {
        if (dump_feas[id] == 0xFF) continue; /* not a move */
        Move m = move_decode(Q, (uint32_t)id);
        if (!((op_mask >> m.op) & 1)) continue;
        if (sample_every > 1 && (seen++ % sample_every) != 0) continue;
        memcpy(o2, off, sizeof(int32_t) * (R + 1));
        memcpy(c2, cust, sizeof(int32_t) * n);
        if (oracle_apply(n, D, node4, cap, has_tw, R, o2, c2, (uint32_t)id) != 0) {
            bad++;
            continue;
        }
        int64_t after = oracle_cost(n, D, node4, cap, has_tw, R, o2, c2, NULL, NULL);
        if (after - base != dump_delta[id]) bad++;
    }
    free(o2);
    free(c2);
    index_free(&X);
    return bad;
}

typedef struct {
    uint32_t id;
    int32_t delta;
} Step;

/* Best-improvement local search (the loop of the feasible-and-infeasible
 * search, Appendix Alg. A2, with hard feasibility): evaluate, accept the best
 * move while its delta is negative, stop at a local optimum or after
 * max_steps.  Writes the accepted moves to `traj` (max_steps entries) and
 * updates (off, cust) in place.  Returns the number of accepted moves. */
static int ls_core(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                   int has_tw, int R, int32_t *off, int32_t *cust, uint32_t op_mask, const uint8_t *gran,
                   int pen, int64_t w_load,
                   int64_t w_tw, int max_steps, int nthreads, uint32_t *traj_id, int32_t *traj_delta,
                   int64_t *moves_total) {
    int steps = 0;
    int64_t mv_sum = 0;
    while (steps < max_steps) {
        int64_t bd = 0, mv = 0;
        uint32_t bid = 0;
        int found = eval_core(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, gran, pen, w_load, w_tw,
                              nthreads, NULL, NULL, &bd, &bid, &mv);
        mv_sum += mv;
        if (!found || bd >= 0) break;
        if (oracle_apply(n, D, node4, cap, has_tw, R, off, cust, bid) != 0) break;
        traj_id[steps] = bid;
        traj_delta[steps] = (int32_t)bd;
        steps++;
    }
    if (moves_total) *moves_total = mv_sum;
    return steps;
}

int oracle_ls(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
              int R, int32_t *off, int32_t *cust, uint32_t op_mask, int max_steps,
              int nthreads, uint32_t *traj_id, int32_t *traj_delta, int64_t *moves_total) {
    return ls_core(n, D, node4, NULL, cap, has_tw, R, off, cust, op_mask, NULL, 0, 0, 0, max_steps, nthreads,
                   traj_id, traj_delta, moves_total);
}

/* Penalised local search: repeat {best move by score; apply it if its score
 * is negative} (feasible and infeasible search, Alg. A2). */
int oracle_ls_pen(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                  int R, int32_t *off, int32_t *cust, uint32_t op_mask, int64_t w_load, int64_t w_tw,
                  int max_steps, int nthreads, uint32_t *traj_id, int32_t *traj_score,
                  int64_t *moves_total) {
    return ls_core(n, D, node4, NULL, cap, has_tw, R, off, cust, op_mask, NULL, 1, w_load, w_tw, max_steps,
                   nthreads, traj_id, traj_score, moves_total);
}

/* The granular pair mask: mask[i * (n+1) + j] = 1 when j is among the
 * theta nodes closest to i (distance, then id; i itself excluded) or i is
 * among the theta closest to j.  Plain selection by sorting each row. */
static int cmp_key(const void *x, const void *y) {
    const int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return a < b ? -1 : a > b;
}

void oracle_granular_mask(int n, const int32_t *D, int theta, uint8_t *mask) {
    const int N = n + 1;
    memset(mask, 0, (size_t)N * N);
    int64_t *key = malloc(sizeof(int64_t) * N);
    for (int i = 0; i < N; i++) {
        int m = 0;
        for (int j = 0; j < N; j++)
            if (j != i) key[m++] = ((int64_t)D[(int64_t)i * N + j] << 20) | j;
        qsort(key, m, sizeof(int64_t), cmp_key);
        for (int k = 0; k < theta && k < m; k++) {
            int j = (int)(key[k] & ((1 << 20) - 1));
            mask[(size_t)i * N + j] = 1;
            mask[(size_t)j * N + i] = 1;
        }
    }
    free(key);
}

/* Granular mode (hard feasibility): as oracle_eval over the reduced
 * neighbourhood of the mask built by oracle_granular_mask. */
int oracle_eval_gran(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                     int R, const int32_t *off, const int32_t *cust, uint32_t op_mask, const uint8_t *mask,
                     int nthreads, int32_t *dump_delta, uint8_t *dump_feas, int64_t *best_delta,
                     uint32_t *best_id, int64_t *moves) {
    return eval_core(n, D, node4, NULL, cap, has_tw, R, off, cust, op_mask, mask, 0, 0, 0, nthreads,
                     dump_delta, dump_feas, best_delta, best_id, moves);
}

int oracle_ls_gran(int n, const int32_t *D, const int32_t *node4, int64_t cap, int has_tw,
                   int R, int32_t *off, int32_t *cust, uint32_t op_mask, const uint8_t *mask, int max_steps,
                   int nthreads, uint32_t *traj_id, int32_t *traj_delta, int64_t *moves_total) {
    return ls_core(n, D, node4, NULL, cap, has_tw, R, off, cust, op_mask, mask, 0, 0, 0, max_steps, nthreads,
                   traj_id, traj_delta, moves_total);
}

/* General entry points: optional pickups (VRPSPDTW), optional granular
 * mask, hard or penalised scoring (pen = 0 / 1). */
int oracle_eval_ex(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap, int has_tw,
                   int R, const int32_t *off, const int32_t *cust, uint32_t op_mask, const uint8_t *mask,
                   int pen, int64_t w_load, int64_t w_tw, int nthreads, int32_t *dump_delta, uint8_t *dump_feas,
                   int64_t *best_delta, uint32_t *best_id, int64_t *moves) {
    return eval_core(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, mask, pen, w_load, w_tw, nthreads,
                     dump_delta, dump_feas, best_delta, best_id, moves);
}

int oracle_ls_ex(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap, int has_tw,
                 int R, int32_t *off, int32_t *cust, uint32_t op_mask, const uint8_t *mask, int pen,
                 int64_t w_load, int64_t w_tw, int max_steps, int nthreads, uint32_t *traj_id,
                 int32_t *traj_delta, int64_t *moves_total) {
    return ls_core(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, mask, pen, w_load, w_tw, max_steps,
                   nthreads, traj_id, traj_delta, moves_total);
}

/* ------------------------------------------------------- multi-move --- */

typedef struct {
    int64_t delta;
    uint32_t id;
    int r1, r2;
} Cand;

static int cmp_cand(const void *x, const void *y) {
    const Cand *a = x, *b = y;
    if (a->delta != b->delta) return a->delta < b->delta ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

/* Several independent moves per iteration (Section 7, after Dynasearch):
 * the candidates are, for every pair of route slots {r1, r2} (r1 = r2 for
 * moves inside one route), the best admissible improving move touching
 * exactly those routes; taken in (delta, id) order, a candidate is selected
 * when none of its routes is used by an earlier selection.  Moves on disjoint
 * routes are independent: each keeps its delta and its feasibility, so the
 * selected set improves the objective by the sum of their deltas.  Writes up
 * to max_out selections in order; returns how many were selected. */
static int multi_select(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                        int has_tw, int R, const int32_t *off, const int32_t *cust, uint32_t op_mask, int pen,
                        int64_t w_load, int64_t w_tw, int nthreads, int max_out, uint32_t *ids,
                        int64_t *deltas, int64_t *moves, int64_t *ncand) {
    Best *pair = calloc((size_t)R * R, sizeof(Best));
    int64_t bd = 0;
    uint32_t bid = 0;
    eval_core2(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, NULL, pen, w_load, w_tw, nthreads, NULL,
               NULL, &bd, &bid, moves, pair);
    Cand *c = malloc(sizeof(Cand) * (size_t)R * R);
    int nc = 0;
    for (int r1 = 0; r1 < R; r1++)
        for (int r2 = r1; r2 < R; r2++) {
            Best *b = &pair[(size_t)r1 * R + r2];
            if (b->found) c[nc++] = (Cand){b->delta, b->id, r1, r2};
        }
    if (ncand) *ncand = nc;
    qsort(c, (size_t)nc, sizeof(Cand), cmp_cand);
    char *used = calloc((size_t)R, 1);
    int cnt = 0;
    for (int q = 0; q < nc && cnt < max_out; q++) {
        if (used[c[q].r1] || used[c[q].r2]) continue;
        used[c[q].r1] = used[c[q].r2] = 1;
        ids[cnt] = c[q].id;
        deltas[cnt] = c[q].delta;
        cnt++;
    }
    free(used);
    free(c);
    free(pair);
    return cnt;
}

int oracle_multi_select(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                        int has_tw, int R, const int32_t *off, const int32_t *cust, uint32_t op_mask, int pen,
                        int64_t w_load, int64_t w_tw, int nthreads, int max_out, uint32_t *ids, int64_t *deltas,
                        int64_t *moves, int64_t *ncand) {
    return multi_select(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, pen, w_load, w_tw, nthreads,
                        max_out, ids, deltas, moves, ncand);
}

/* Multi-move local search: repeat {select; apply every selected move, in
 * selection order} until nothing improves or max_iters iterations.  Writes
 * the applied moves in order (up to max_moves) and the count per iteration;
 * updates (off, cust) in place; returns the number of iterations. */
int oracle_ls_multi(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                    int has_tw, int R, int32_t *off, int32_t *cust, uint32_t op_mask, int pen, int64_t w_load,
                    int64_t w_tw, int max_iters, int nthreads, int max_moves, uint32_t *traj_id,
                    int32_t *traj_delta, int32_t *per_iter, int64_t *moves_total) {
    uint32_t *ids = malloc(sizeof(uint32_t) * (size_t)R);
    int64_t *dl = malloc(sizeof(int64_t) * (size_t)R);
    int it = 0, nm = 0;
    int64_t mv_sum = 0;
    while (it < max_iters) {
        int64_t mv = 0;
        int cnt = multi_select(n, D, node4, pick, cap, has_tw, R, off, cust, op_mask, pen, w_load, w_tw,
                               nthreads, R, ids, dl, &mv, NULL);
        mv_sum += mv;
        if (cnt == 0) break;
        for (int q = 0; q < cnt; q++) {
            if (oracle_apply(n, D, node4, cap, has_tw, R, off, cust, ids[q]) != 0) {
                cnt = q;
                break;
            }
            if (nm < max_moves) {
                traj_id[nm] = ids[q];
                traj_delta[nm] = (int32_t)dl[q];
            }
            nm++;
        }
        per_iter[it++] = cnt;
    }
    free(ids);
    free(dl);
    if (moves_total) *moves_total = mv_sum;
    return it;
}

/* Penalty terms of S: total load excess and total time warp over the routes
 * (as in penalised mode). */
void oracle_violations(int n, const int32_t *D, const int32_t *node4, const int32_t *pick, int64_t cap,
                       int has_tw, int R, const int32_t *off, const int32_t *cust, int64_t *load_excess,
                       int64_t *time_warp) {
    Inst I = {n, D, node4, cap, has_tw, pick};
    int64_t lv = 0, tv = 0;
    for (int r = 0; r < R; r++) {
        int L = off[r + 1] - off[r];
        lv += route_load_excess(&I, cust + off[r], L);
        tv += route_time_warp(&I, cust + off[r], L);
    }
    *load_excess = lv;
    *time_warp = tv;
}
