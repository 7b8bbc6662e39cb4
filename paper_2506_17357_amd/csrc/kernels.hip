// HIP kernels (gfx950) for full-neighbourhood move evaluation, best-move
// reduction, move application and attribute rebuild.
//
// The paper evaluates moves by concatenating route subsequences whose
// attributes are precomputed (Section 4.1; distance: eq. dist; load: the
// zero-pickup form of the load concatenation; windows: Section 4.3.3), in
// five steps per operator (Section 5.1): extraction, concatenation,
// differencing, evaluation (argmin), update.  Here the five steps are fused
// per pair of positions: the attribute "tensor" is a set of per-slot arrays
// (route id and position, as the positional tensors of Section 5.3.1; prefix
// load; edge to the successor; earliest departure; latest feasible arrival
// at the successor), every concatenation is evaluated in registers, and the
// argmin is a running (delta, id) minimum per lane followed by a wavefront and
// workgroup reduction and one 64-bit atomicMin per solution.
//
// Time windows use the hard-window case of the time-warp algebra (Section
// 4.3.3: a concatenation is feasible exactly when its time-window violation
// T_V is zero): forward earliest service starts A, backward latest arrivals
// Z, and (duration, earliest finish, latest arrival) summaries for the middle
// segments of intra-route moves.

#include "tga_internal.h"
#include <type_traits>

namespace tga {

constexpr int kInterWaves = 8;      // wavefronts per inter-route workgroup
constexpr int kInterThreads = kInterWaves * 64;
constexpr int kColsPerWave = 62;    // lanes 1..62 own a column; 0 and 63 are halo
constexpr int kIntraThreads = 256;
constexpr int kApplyThreads = 1024;
constexpr int kTwOff = 1 << 28;     // due time standing for "no window" (CVRP)

// Loads through pointers kept in the solution descriptor: the pointee is
// global memory, so say so (global_load instead of a generic flat load).
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}

__device__ __forceinline__ int4 gld(const int4 *p) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = *(const __attribute__((address_space(1))) v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int2 gld(const int2 *p) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    const v2i v = *(const __attribute__((address_space(1))) v2i *)p;
    return make_int2(v.x, v.y);
}

// Load of a value every lane of the wavefront reads at the same address,
// through the constant address space so that it becomes a scalar load into
// SGPRs.  Only for data no kernel of the same launch writes.
__device__ __forceinline__ int4 sld(const int4 *p) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i v = *(const __attribute__((address_space(4))) v4i *)p;
    return make_int4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ int sld1(const int *p) { return *(const __attribute__((address_space(4))) int *)p; }

// The same at a byte offset from p (one scalar load with an offset register).
__device__ __forceinline__ int4 sld_at(const int4 *p, uint32_t byte_off) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const __attribute__((address_space(4))) char *b = (const __attribute__((address_space(4))) char *)p;
    const v4i v = *(const __attribute__((address_space(4))) v4i *)(b + byte_off);
    return make_int4(v.x, v.y, v.z, v.w);
}

template <class T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

__device__ __forceinline__ void gst(int4 *p, int4 v) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i x = {v.x, v.y, v.z, v.w};
    *(__attribute__((address_space(1))) v4i *)p = x;
}

__device__ __forceinline__ void gst(int2 *p, int2 v) {
    typedef int v2i __attribute__((ext_vector_type(2)));
    const v2i x = {v.x, v.y};
    *(__attribute__((address_space(1))) v2i *)p = x;
}

__device__ __forceinline__ int nodeof(int x) { return x & 0xFFFF; }
__device__ __forceinline__ int flagsof(int x) { return x >> 16; }

// Deltas at or above this are not admissible (inter-route moves carry a
// penalty of 2^30; every admissible delta is far below 2^29).
constexpr int kAdmissibleBound = 1 << 29;

// Internal operator-mask bit: the evaluation feeds a local-search step, which
// applies the best move only when its delta is negative.  Lanes then start
// from the bound (delta 0, no id): moves with a positive delta are never
// evaluated in full, and the best improving move — the only one the step can
// apply — is found exactly as before.
constexpr uint32_t kImprovingOnly = 1u << 31;
// Operator-mask modifier (TGA_OP_COUNT_FULL, batched form): the evaluation
// launch is the instantiation that also counts the pairs evaluated in full.
constexpr uint32_t kCountFull = 1u << 17;
// Operator-mask modifier (TGA_OP_MULTI, general path): the evaluation also
// keeps, per pair of route slots, the best improving move touching exactly
// those routes (S.pairkey), for the selection of independent moves.
constexpr uint32_t kMulti = 1u << 18;

// Operator-mask modifier (TGA_OP_GRANULAR): inter-route operators restricted
// to the granular pairs of the instance.
constexpr uint32_t kGranular = 1u << 16;

__device__ __forceinline__ int initial_bound(uint32_t op_mask) {
    return (op_mask & kImprovingOnly) ? 0 : kAdmissibleBound;
}

// A local-search evaluation skips a solution that has converged (or reached
// its step cap); any other evaluation covers every solution, converged or not.
__device__ __forceinline__ bool skip_solution(const SolDev &S, uint32_t op_mask) {
    return (op_mask & kImprovingOnly) && S.state[kStDone];
}

__device__ __forceinline__ unsigned long long pack_key(int delta, uint32_t id) {
    return ((unsigned long long)((uint32_t)delta ^ 0x80000000u) << 32) | id;
}

__device__ __forceinline__ bool better(int d, uint32_t id, int bd, uint32_t bid) {
    return d < bd || (d == bd && id < bid);
}

__device__ __forceinline__ void consider(int d, uint32_t id, int &bd, uint32_t &bid) {
    if (d < kAdmissibleBound && better(d, id, bd, bid)) {
        bd = d;
        bid = id;
    }
}

__device__ __forceinline__ void wave_argmin(int &bd, uint32_t &bid) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int od = __shfl_xor(bd, off);
        const uint32_t oid = (uint32_t)__shfl_xor((int)bid, off);
        if (better(od, oid, bd, bid)) {
            bd = od;
            bid = oid;
        }
    }
}

// Reduce the per-lane bests of a workgroup and fold the result into the
// solution's key.  Every thread of the block must call it.
__device__ __forceinline__ void block_argmin_commit(int bd, uint32_t bid, unsigned long long *key,
                                    unsigned long long *red) {
    wave_argmin(bd, bid);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = (bd >= kAdmissibleBound || bid == 0xFFFFFFFFu) ? ~0ull : pack_key(bd, bid);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = ~0ull;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = red[w] < m ? red[w] : m;
        if (m != ~0ull) atomicMin(key, m);
    }
    __syncthreads();
}

// Insert one node with window [e, l] and service s: arrive from a departure
// time `dep` over `cin`, leave over `cout` to a successor whose latest
// feasible arrival is `z`.
__device__ __forceinline__ bool tw_insert(int dep, int cin, int e, int l, int s, int cout, int z) {
    const int arr = dep + cin;
    const int st = arr > e ? arr : e;
    return (arr <= l) & (st + s + cout <= z);
}

// (duration, earliest finish, latest arrival) summary of a segment under hard
// windows: arriving at time a <= la, the segment is served and left at
// max(a + dur, ef).
struct Seg {
    int dur, ef, la;
    bool ok;
};

__device__ __forceinline__ Seg seg_node(int e, int l, int s) { return Seg{s, e + s, l, true}; }

// a then b, travelling c from the last node of a to the first node of b.
__device__ __forceinline__ Seg seg_cat(const Seg &a, int c, const Seg &b) {
    Seg r;
    r.dur = a.dur + c + b.dur;
    r.ef = max(a.ef + c + b.dur, b.ef);
    r.la = min(a.la, b.la - c - a.dur);
    r.ok = a.ok && b.ok && (a.ef + c <= b.la);
    return r;
}

// Arrive at `arr`; returns the departure time, or kInf when infeasible.
__device__ __forceinline__ int seg_pass(const Seg &g, int arr) {
    if (!g.ok || arr > g.la) return kInf;
    const int d = arr + g.dur;
    return d > g.ef ? d : g.ef;
}

// ------------------------------------------------------------ rebuild ------
// Segmented scans over the route-major slot array, one workgroup per
// solution.  Forward: prefix load and prefix distance (sums) and the earliest
// service start A (maps x -> x <= th ? max(x + al, be) : INF, closed under
// composition).  Backward: latest feasible arrival Z (maps
// y -> y >= th ? min(y + al, be) : NEG).  A reset flag marks a segment
// boundary (a route start for the forward scans, a route end for the
// backward scan).

struct FwdElem {
    int32_t rs;          // reset
    int32_t load, dist;  // additive parts
    int32_t th, al, be;  // A map
};

__device__ __forceinline__ FwdElem fwd_identity() { return FwdElem{0, 0, 0, kInf, 0, kNeg}; }

// apply a, then b
__device__ __forceinline__ FwdElem fwd_cat(const FwdElem &a, const FwdElem &b) {
    if (b.rs) return b;
    FwdElem r;
    r.rs = a.rs;
    r.load = a.load + b.load;
    r.dist = a.dist + b.dist;
    r.th = (a.be <= b.th) ? min(a.th, b.th - a.al) : -1;
    r.al = a.al + b.al;
    r.be = max(a.be + b.al, b.be);
    return r;
}

__device__ __forceinline__ int fwd_apply(const FwdElem &m, int x) {
    return (x <= m.th) ? max(x + m.al, m.be) : kInf;
}

struct BwdElem {
    int32_t rs, th, al, be;
};

__device__ __forceinline__ BwdElem bwd_identity() { return BwdElem{0, kNeg, 0, kInf}; }

// apply r (the part to the right) first, then l
__device__ __forceinline__ BwdElem bwd_cat(const BwdElem &l, const BwdElem &r) {
    if (l.rs) return l;
    BwdElem o;
    o.rs = r.rs;
    o.th = (r.be >= l.th) ? max(r.th, l.th - r.al) : kInf;
    o.al = r.al + l.al;
    o.be = min(r.be + l.al, l.be);
    return o;
}

__device__ __forceinline__ int bwd_apply(const BwdElem &m, int y) {
    return (y >= m.th) ? min(y + m.al, m.be) : kNeg;
}

struct ApplyShared {
    FwdElem fw[kApplyThreads / 64];
    BwdElem bw[kApplyThreads / 64];
    long long red[kApplyThreads / 64][5];
};

__device__ __forceinline__ FwdElem shfl_f(const FwdElem &e, int src) {
    return FwdElem{__shfl(e.rs, src), __shfl(e.load, src), __shfl(e.dist, src),
                   __shfl(e.th, src),  __shfl(e.al, src),   __shfl(e.be, src)};
}

__device__ __forceinline__ BwdElem shfl_b(const BwdElem &e, int src) {
    return BwdElem{__shfl(e.rs, src), __shfl(e.th, src), __shfl(e.al, src), __shfl(e.be, src)};
}

// Exclusive prefix (in thread order) of per-thread forward aggregates:
// wavefront shuffle scan, then a scan of the wavefront totals by wavefront 0.
__device__ __forceinline__ FwdElem block_prefix_fwd(FwdElem v, FwdElem *wtot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    FwdElem x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const FwdElem y = shfl_f(x, lane - d < 0 ? lane : lane - d);
        if (lane >= d) x = fwd_cat(y, x);
    }
    if (lane == 63) wtot[wave] = x;
    __syncthreads();
    if (wave == 0) {
        FwdElem w = lane < nw ? wtot[lane] : fwd_identity();
        for (int d = 1; d < 64; d <<= 1) {
            const FwdElem y = shfl_f(w, lane - d < 0 ? lane : lane - d);
            if (lane >= d) w = fwd_cat(y, w);
        }
        if (lane < nw) wtot[lane] = w;
    }
    __syncthreads();
    FwdElem ex = shfl_f(x, lane == 0 ? 0 : lane - 1);
    if (lane == 0) ex = fwd_identity();
    const FwdElem pre = wave > 0 ? wtot[wave - 1] : fwd_identity();
    const FwdElem r = fwd_cat(pre, ex);
    __syncthreads();
    return r;
}

// Exclusive suffix (aggregate of the threads after this one) of backward
// aggregates.
__device__ __forceinline__ BwdElem block_suffix_bwd(BwdElem v, BwdElem *wtot) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    BwdElem x = v;
    for (int d = 1; d < 64; d <<= 1) {
        const BwdElem y = shfl_b(x, lane + d > 63 ? lane : lane + d);
        if (lane + d < 64) x = bwd_cat(x, y);
    }
    if (lane == 0) wtot[wave] = x;
    __syncthreads();
    if (wave == 0) {
        BwdElem w = lane < nw ? wtot[lane] : bwd_identity();
        for (int d = 1; d < 64; d <<= 1) {
            const BwdElem y = shfl_b(w, lane + d > 63 ? lane : lane + d);
            if (lane + d < nw) w = bwd_cat(w, y);
        }
        if (lane < nw) wtot[lane] = w;
    }
    __syncthreads();
    BwdElem ex = shfl_b(x, lane == 63 ? 63 : lane + 1);
    if (lane == 63) ex = bwd_identity();
    const BwdElem post = wave < nw - 1 ? wtot[wave + 1] : bwd_identity();
    const BwdElem r = bwd_cat(ex, post);
    __syncthreads();
    return r;
}

// Forward element of slot s (reads what passes 1 and 2 wrote).
__device__ __forceinline__ FwdElem fwd_elem(const SolDev &S, const int32_t *roffn, int s) {
    const int4 a = gld(S.a4 + s);
    FwdElem e;
    if (s == gld(roffn + a.y)) {
        e = fwd_identity();
        e.rs = 1;
        return e;
    }
    const int4 ap = gld(S.a4 + s - 1);
    const int sp = gld(S.w4 + s - 1).z;
    const int4 w = gld(S.w4 + s);
    e.rs = 0;
    e.load = gld(S.b4 + s).x;
    e.dist = ap.z;
    e.al = sp + ap.z;
    e.th = w.y - e.al;
    e.be = w.x;
    return e;
}

__device__ __forceinline__ BwdElem bwd_elem(const SolDev &S, const int32_t *roffn, int s) {
    const int4 a = gld(S.a4 + s);
    const int4 w = gld(S.w4 + s);
    const int last = gld(roffn + a.y + 1) - 1;
    const int b = w.z + a.z;
    BwdElem e;
    e.rs = s == last;
    e.th = w.x + b;
    e.al = -b;
    e.be = w.y;
    return e;
}

// Cost (sum of route distances) and |N(S)| per operator from the route
// offsets and distances.  Every thread of the block calls it.
__device__ __forceinline__ void solution_totals(const SolDev &S, const int32_t *roffn, ApplyShared &sh) {
    const int Q = S.Q, R = S.R, n = S.n;
    const int tid = threadIdx.x, T = blockDim.x;
    // cost and |N(S)| per operator
    long long v[5] = {0, 0, 0, 0, 0};
    for (int r = tid; r < R; r += T) {
        const long long L = gld(roffn + r + 1) - gld(roffn + r) - 1;
        v[0] += gld(S.rdist + r);
        v[1] += L * (Q - L - 1);
        v[2] += (L + 1) * (L + 1);
        v[3] += L * (L - 1) / 2;
        for (int k = 1; k <= 3; ++k)
            if (k <= L) v[4] += (L - k + 1) * (L - k);
    }
    for (int i = 0; i < 5; ++i) {
        long long x = v[i];
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
        v[i] = x;
    }
    if ((tid & 63) == 0)
        for (int i = 0; i < 5; ++i) sh.red[tid >> 6][i] = v[i];
    __syncthreads();
    if (tid == 0) {
        long long t[5] = {0, 0, 0, 0, 0};
        for (int w = 0; w < T / 64; ++w)
            for (int i = 0; i < 5; ++i) t[i] += sh.red[w][i];
        const long long qq = (long long)Q * Q;
        S.acc[kAccCost] = t[0];
        S.acc[kAccCnt0 + 0] = t[1];
        S.acc[kAccCnt0 + 1] = (long long)n * (n - 1) / 2;
        S.acc[kAccCnt0 + 2] = (qq - t[2]) / 2;
        S.acc[kAccCnt0 + 3] = t[3];
        S.acc[kAccCnt0 + 4] = t[4];
    }
    __threadfence_block();
    __syncthreads();
}

// Attributes of the slots [lo, hi) of the layout (nr, roffn), a union of
// whole routes, from their nodes (nr[s] = {node, route}; nr is then reused
// as scratch for the scans' A and Z).  `full`: the whole layout (also the
// route offsets and the sentinel slot Q); otherwise the other slots are
// already right.  Route distances, cost and |N(S)| are refreshed either way.
// Requires blockDim.x == kApplyThreads.
__device__ __forceinline__ void rebuild_range(const SolDev &S, int2 *nr, const int32_t *roffn, int lo, int hi,
                                              bool full, ApplyShared &sh) {
    const int Q = S.Q, R = S.R, n = S.n, np1 = S.np1;
    const int tid = threadIdx.x, T = blockDim.x;
    const int32_t *D = S.D;
    const int4 *nd = S.node4;
    const bool tw = S.has_tw;

    if (full)
        for (int r = tid; r <= R; r += T) gst(S.roff + r, gld(roffn + r));
    // pass 1: node, route, edge, per-node data, ref map
    for (int s = lo + tid; s < hi; s += T) {
        const int2 x = gld(nr + s);
        const int node = x.x, r = x.y;
        const int first = gld(roffn + r), last = gld(roffn + r + 1) - 1;
        const int succ = s < last ? gld(nr + s + 1).x : 0;
        int4 q = gld(nd + node);
        if (!tw) q = make_int4(q.x, 0, kTwOff, 0);
        const int edge = gld(D + (size_t)node * np1 + succ);
        const bool cust = s != first;
        gst(S.a4 + s, make_int4(node | ((cust ? kFlagCustomer : 0) << 16), r, edge, 0));
        gst(S.w4 + s, make_int4(q.y, q.z, q.w, 0));
        gst(S.b4 + s, make_int4(cust ? q.x : 0, 0, 0, 0));
        gst(S.ref2slot + (cust ? node - 1 : n + r), s);
    }
    if (full && tid == 0) {
        gst(S.a4 + Q, make_int4(0, R, 0, 0));
        gst(S.b4 + Q, make_int4(0, 0, 0, 0));
        gst(S.w4 + Q, make_int4(tw ? gld(nd).y : 0, tw ? gld(nd).z : kTwOff, 0, 0));
        gst(S.t4 + Q, make_int4(kInf, kNeg, kInf, kNeg));
        gst(S.pdist + Q, 0);
    }
    __threadfence_block();
    __syncthreads();
    // pass 2: removal delta and incident-edge sums (customers)
    for (int s = lo + tid; s < hi; s += T) {
        int4 a = gld(S.a4 + s);
        if (s == gld(roffn + a.y)) continue;
        const int4 ap = gld(S.a4 + s - 1);
        const int succ = s + 1 < gld(roffn + a.y + 1) ? gld(nr + s + 1).x : 0;
        const int dpw = gld(D + (size_t)nodeof(ap.x) * np1 + succ);
        a.w = dpw - ap.z - a.z;
        gst(S.a4 + s, a);
        int4 b = gld(S.b4 + s);
        b.w = ap.z + a.z;
        gst(S.b4 + s, b);
    }
    __threadfence_block();
    __syncthreads();

    const int C = (hi - lo + T - 1) / T;
    const int beg = min(hi, lo + tid * C), end = min(hi, beg + C);
    // forward scans: prefix load, prefix distance, earliest service start A
    {
        FwdElem agg = fwd_identity();
        for (int s = beg; s < end; ++s) agg = fwd_cat(agg, fwd_elem(S, roffn, s));
        FwdElem run = block_prefix_fwd(agg, sh.fw);
        const int e0 = tw ? gld(nd).y : 0;
        for (int s = beg; s < end; ++s) {
            run = fwd_cat(run, fwd_elem(S, roffn, s));
            int4 b = gld(S.b4 + s);
            b.y = run.load;
            gst(S.b4 + s, b);
            gst(S.pdist + s, run.dist);
            int2 z = gld(nr + s);
            z.x = tw ? fwd_apply(run, e0) : 0;  // A[s]
            gst(nr + s, z);
        }
    }
    __threadfence_block();
    __syncthreads();
    // backward scan: latest feasible arrival Z (windows only)
    if (!tw) {
        for (int s = beg; s < end; ++s) {
            int2 z = gld(nr + s);
            z.y = kTwOff;
            gst(nr + s, z);
        }
    } else {
        BwdElem agg = bwd_identity();
        for (int s = end - 1; s >= beg; --s) agg = bwd_cat(bwd_elem(S, roffn, s), agg);
        BwdElem run = block_suffix_bwd(agg, sh.bw);
        const int l0 = gld(nd).z;
        for (int s = end - 1; s >= beg; --s) {
            run = bwd_cat(bwd_elem(S, roffn, s), run);
            int2 z = gld(nr + s);
            z.y = bwd_apply(run, l0);  // Z[s]
            gst(nr + s, z);
        }
    }
    __threadfence_block();
    __syncthreads();
    // pass 3: route totals (by the thread owning each route's last slot)
    for (int s = lo + tid; s < hi; s += T) {
        const int r = gld(S.a4 + s).y;
        if (s == gld(roffn + r + 1) - 1) gst(S.rdist + r, gld(S.pdist + s) + gld(S.a4 + s).z);
    }
    // pass 4: derived per-slot values and flags
    const int l0 = tw ? gld(nd).z : kTwOff;
    const int cap = S.cap;
    for (int s = lo + tid; s < hi; s += T) {
        int4 a = gld(S.a4 + s);
        const int first = gld(roffn + a.y), last = gld(roffn + a.y + 1) - 1;
        const int rload = gld(S.b4 + last).y;
        const int4 w = gld(S.w4 + s);
        const int2 az = gld(nr + s);
        const int A = az.x;
        const int dep = A >= kInf ? kInf : A + w.z;
        const int zn = s < last ? gld(nr + s + 1).y : l0;
        int adp = kInf;
        int flags = flagsof(a.x);
        int4 b = gld(S.b4 + s);
        if (s != first) {
            const int Ap = gld(nr + s - 1).x;
            adp = Ap >= kInf ? kInf : Ap + gld(S.w4 + s - 1).z;
            if (rload - b.x <= cap) flags |= kFlagRemCap;
            // without this node: predecessor departure + c(pred, succ) <= Z(succ)
            const int dpw = a.w + b.w;  // removal delta + incident edges = c(pred, succ)
            if (adp < kInf && adp + dpw <= zn) flags |= kFlagRemTw;
        }
        a.x = nodeof(a.x) | (flags << 16);
        gst(S.a4 + s, a);
        b.z = rload;
        gst(S.b4 + s, b);
        gst(S.t4 + s, make_int4(dep, zn, adp, az.y));
    }
    __threadfence_block();
    __syncthreads();
    solution_totals(S, roffn, sh);
}

// The same attributes for one route of at most 64 slots, by one wavefront
// entirely in registers: lane p holds position p (slot base + p; p = 0 is
// the start depot, L customers follow; nr[slot].x is the node).  The
// prefix load and distance and the two window maps are wavefront shuffle
// scans of the same elements the block scans use.  Writes the slot
// attributes, the reverse map and the route distance; no barrier.
__device__ __forceinline__ void rebuild_route_wave(const SolDev &S, const int2 *nr, int r, int base, int L) {
    const int lane = threadIdx.x & 63, np1 = S.np1;
    const int32_t *D = S.D;
    const bool tw = S.has_tw;
    const bool on = lane <= L;
    const int s = base + lane;
    const int node = on ? nr[s].x : 0;
    const int succ = __shfl(node, min(lane + 1, 63));
    const int nsucc = lane < L ? succ : 0;  // the route ends at the depot
    const int pred = __shfl(node, max(lane - 1, 0));
    int4 q = gld(S.node4 + node);
    if (!tw) q = make_int4(q.x, 0, kTwOff, 0);
    const int edge = on ? gld(D + (size_t)node * np1 + nsucc) : 0;
    const bool cust = lane >= 1 && on;
    const int demand = cust ? q.x : 0;
    const int epred = __shfl(edge, max(lane - 1, 0));
    const int spred = __shfl(q.w, max(lane - 1, 0));
    const int dpw = cust ? gld(D + (size_t)pred * np1 + nsucc) : 0;  // c(pred, succ)
    // forward elements (as fwd_elem): reset at the start depot
    FwdElem f;
    if (lane == 0 || !on) {
        f = fwd_identity();
        f.rs = lane == 0;
    } else {
        f.rs = 0;
        f.load = demand;
        f.dist = epred;
        f.al = spred + epred;
        f.th = q.z - f.al;
        f.be = q.y;
    }
    for (int d = 1; d < 64; d <<= 1) {
        const FwdElem y = shfl_f(f, lane - d < 0 ? lane : lane - d);
        if (lane >= d) f = fwd_cat(y, f);
    }
    // backward elements (as bwd_elem): reset at the last slot
    BwdElem g;
    if (on) {
        const int b = q.w + edge;
        g.rs = lane == L;
        g.th = q.y + b;
        g.al = -b;
        g.be = q.z;
    } else {
        g = bwd_identity();
    }
    for (int d = 1; d < 64; d <<= 1) {
        const BwdElem y = shfl_b(g, lane + d > 63 ? lane : lane + d);
        if (lane + d < 64) g = bwd_cat(g, y);
    }
    const int e0 = tw ? gld(S.node4).y : 0;
    const int l0 = tw ? gld(S.node4).z : kTwOff;
    const int A = tw ? fwd_apply(f, e0) : 0;
    const int Z = tw ? bwd_apply(g, l0) : kTwOff;
    const int rload = __shfl(f.load, L);
    const int Zn = __shfl(Z, min(lane + 1, 63));
    const int Ap = __shfl(A, max(lane - 1, 0));
    const int dep = A >= kInf ? kInf : A + q.w;
    const int zn = lane < L ? Zn : l0;
    int adp = kInf;
    int flags = cust ? kFlagCustomer : 0;
    if (cust) {
        adp = Ap >= kInf ? kInf : Ap + spred;
        if (rload - demand <= S.cap) flags |= kFlagRemCap;
        if (adp < kInf && adp + dpw <= zn) flags |= kFlagRemTw;
    }
    if (on) {
        const int rem = cust ? dpw - epred - edge : 0;
        const int inc = cust ? epred + edge : 0;
        gst(S.a4 + s, make_int4(node | (flags << 16), r, edge, rem));
        gst(S.b4 + s, make_int4(demand, f.load, rload, inc));
        gst(S.w4 + s, make_int4(q.y, q.z, q.w, 0));
        gst(S.t4 + s, make_int4(dep, zn, adp, Z));
        gst(S.pdist + s, f.dist);
        gst(S.ref2slot + (cust ? node - 1 : S.n + r), s);
        if (lane == L) gst(S.rdist + r, f.dist + edge);
    }
}

__device__ __forceinline__ void rebuild(const SolDev &S, int2 *nr, const int32_t *roffn, ApplyShared &sh) {
    rebuild_range(S, nr, roffn, 0, S.Q, true, sh);
}

// ------------------------------------------------------ penalised mode ---
// Time-warp summaries (Section 4.3.3): a subsequence sigma carries its
// duration T_D, earliest and latest start T_E / T_L and time warp T_V; a node
// is {s, e, l, 0}; two subsequences joined by an edge of travel time t
// concatenate as below (the garbled shift read as T_D(a) - T_V(a) + t).  A
// route's time warp is the T_V of depot, customers, depot.

struct Tw {
    int d, e, l, v;
};

__device__ __forceinline__ Tw tw_of(int4 x) { return Tw{x.x, x.y, x.z, x.w}; }
__device__ __forceinline__ int4 tw_pack(const Tw &x) { return make_int4(x.d, x.e, x.l, x.v); }
__device__ __forceinline__ Tw tw_node(int e, int l, int s) { return Tw{s, e, l, 0}; }

__device__ __forceinline__ Tw tw_cat(const Tw &a, int t, const Tw &b) {
    const int dt = a.d - a.v + t;
    const int dw = max(b.e - dt - a.l, 0);
    const int dv = max(a.e + dt - b.l, 0);
    return Tw{a.d + t + dw + b.d, max(a.e, b.e - dt) - dw, min(a.l, b.l - dt) + dv, a.v + dv + b.v};
}

__device__ __forceinline__ Tw tw_depot(const SolDev &S) {
    const int4 q = gld(S.node4);
    return tw_node(q.y, q.z, q.w);
}

// Prefix and suffix summaries of route r (one thread; TW instances only).
__device__ __forceinline__ void pen_route(const SolDev &S, int r) {
    const int off = gld(S.roff + r), L = gld(S.roff + r + 1) - off - 1;
    const Tw dep = tw_depot(S);
    Tw f = dep;
    gst(S.pf4 + off, tw_pack(f));
    for (int p = 1; p <= L; ++p) {
        const int4 w = gld(S.w4 + off + p);
        f = tw_cat(f, gld(S.a4 + off + p - 1).z, tw_node(w.x, w.y, w.z));
        gst(S.pf4 + off + p, tw_pack(f));
    }
    Tw b = dep;
    for (int p = L; p >= 1; --p) {
        const int4 w = gld(S.w4 + off + p);
        b = tw_cat(tw_node(w.x, w.y, w.z), gld(S.a4 + off + p).z, b);
        gst(S.pb4 + off + p, tw_pack(b));
    }
    gst(S.pb4 + off, tw_pack(tw_cat(dep, gld(S.a4 + off).z, b)));
}

// Load summaries (Section 4.3.2): {L_I delivered, L_O picked up, L_M the
// largest load on board}; a node is {d, p, max(d, p)}; concatenation keeps
// the later part's deliveries on board through the earlier part, and the
// earlier part's pickups through the later one.
struct Ld {
    int li, lo, lm;
};

__device__ __forceinline__ Ld ld_of(int4 x) { return Ld{x.x, x.y, x.z}; }
__device__ __forceinline__ int4 ld_pack(const Ld &x) { return make_int4(x.li, x.lo, x.lm, 0); }
__device__ __forceinline__ Ld ld_cat(const Ld &a, const Ld &b) {
    return Ld{a.li + b.li, a.lo + b.lo, max(a.lm + b.li, a.lo + b.lm)};
}
__device__ __forceinline__ Ld ld_node_at(const SolDev &S, int x) {
    const int node = nodeof(gld(S.a4 + x).x);
    const int d = gld(S.b4 + x).x, p = node ? gld(S.pick + node) : 0;
    return Ld{d, p, max(d, p)};
}

// Prefix and suffix load summaries of route r (one thread; pickups only).
__device__ __forceinline__ void pd_route(const SolDev &S, int r) {
    const int off = gld(S.roff + r), L = gld(S.roff + r + 1) - off - 1;
    Ld f{0, 0, 0};
    gst(S.pl4 + off, ld_pack(f));
    for (int p = 1; p <= L; ++p) {
        f = ld_cat(f, ld_node_at(S, off + p));
        gst(S.pl4 + off + p, ld_pack(f));
    }
    Ld b{0, 0, 0};
    for (int p = L; p >= 1; --p) {
        b = ld_cat(ld_node_at(S, off + p), b);
        gst(S.ql4 + off + p, ld_pack(b));
    }
    gst(S.ql4 + off, ld_pack(b));
}

// Largest load on route r: the route load without pickups (kept in every
// slot's b4.z), the suffix summary's L_M at the start depot with them.
__device__ __forceinline__ int route_peak(const SolDev &S, int r) {
    const int off = gld(S.roff + r);
    return S.pd ? gld(S.ql4 + off).z : gld(S.b4 + off).z;
}

// Load excess of route r.
__device__ __forceinline__ int route_excess(const SolDev &S, int r) { return max(route_peak(S, r) - S.cap, 0); }

// Summaries the general evaluation path reads (penalised mode or pickups).
__device__ __forceinline__ void gen_route(const SolDev &S, int r) {
    if (S.has_tw) pen_route(S, r);
    if (S.pd) pd_route(S, r);
}

// Time warp of route r (the suffix summary at its start depot).
__device__ __forceinline__ int route_warp(const SolDev &S, int r) {
    return S.has_tw ? gld(S.pb4 + gld(S.roff + r)).w : 0;
}

// Totals of load excess and time warp over the routes (every thread of the
// block calls it; the summaries must be current).
__device__ __forceinline__ void pen_totals(const SolDev &S, ApplyShared &sh) {
    long long lv = 0, tv = 0;
    for (int r = threadIdx.x; r < S.R; r += blockDim.x) {
        lv += route_excess(S, r);
        tv += route_warp(S, r);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        lv += __shfl_xor(lv, off);
        tv += __shfl_xor(tv, off);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        sh.red[threadIdx.x >> 6][0] = lv;
        sh.red[threadIdx.x >> 6][1] = tv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a += sh.red[w][0];
            b += sh.red[w][1];
        }
        S.acc[kAccLoadExcess] = a;
        S.acc[kAccTimeWarp] = b;
    }
    __syncthreads();
}

// Summaries of every route and the totals (one block).
__device__ __forceinline__ void pen_all(const SolDev &S, ApplyShared &sh) {
    for (int r = threadIdx.x; r < S.R; r += blockDim.x) gen_route(S, r);
    __threadfence_block();
    __syncthreads();
    pen_totals(S, sh);
}

// Build the attributes of a freshly uploaded layout (nr_alt, roff_alt).
__global__ __launch_bounds__(kApplyThreads) void k_build(const SolDev *__restrict__ sols) {
    __shared__ ApplyShared sh;
    const SolDev &S = sols[blockIdx.x];
    rebuild(S, S.nr_alt, S.roff_alt, sh);
    if (S.pen || S.pd || S.gen) pen_all(S, sh);
    if (threadIdx.x == 0) {
        *S.best_key = ~0ull;
        S.state[kStDone] = 0;
        S.state[kStStatus] = 0;
    }
}

// Switch penalised mode on for a solution whose descriptor now says so:
// summaries of every route and the totals.
__global__ __launch_bounds__(kApplyThreads) void k_pen_init(const SolDev *__restrict__ sols) {
    __shared__ ApplyShared sh;
    const SolDev &S = sols[blockIdx.x];
    if (S.pen || S.pd || S.gen) pen_all(S, sh);
}

// ------------------------------------------------------ inter-route eval ---
// One work item = rows [s0, s1) (slots, route-major) against every column
// slot of a later route.  For each unordered pair of slots (s, t) in
// different routes, route(s) < route(t), the fused pass evaluates
// RELOCATE s->after t, RELOCATE t->after s, SWAP s<->t and 2OPT*(s, t) (the
// node-based extraction of Section 5.3.1, eq. node_based1 and
// eq. node_based2, over the positional attributes).
//
// Rows stream through LDS in sub-blocks of S.tile_rows rows plus one halo row
// on each side, copied straight from HBM into LDS (global_load_lds).  A lane
// owns one column of a 62-column chunk and keeps its attributes in
// registers; per row it gathers D[row][node(t)] from LDS once and takes
// D[row][succ(t)] and D[row][pred(t)] from its neighbour lanes (DPP
// wavefront shifts), D[pred(s)][t] and D[succ(s)][t] from the previous and
// next row of a register window.

typedef __attribute__((address_space(3))) void *lds_void_ptr;
typedef __attribute__((address_space(1))) void *global_void_ptr;

// lane i receives lane i+1 (lane 63 receives 0)
__device__ __forceinline__ int from_next_lane(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
// lane i receives lane i-1 (lane 0 receives 0)
__device__ __forceinline__ int from_prev_lane(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }

// Column-side (lane) values of one chunk, kept in registers while the
// wavefront walks rows against it.  Every feasibility condition below is
// written as a difference that must be >= 0; "bad" values are 0 when a
// condition holds and negative otherwise, so OR-ing them keeps the sign of
// "any condition fails".
struct LaneCol {
    int4 ta, tb, tt, tw;
    int node;      // LDS gather index (node of slot t)
    int refT;
    int tyOwn;     // route(t) - 1 if the lane owns its column, else very negative
    int tInval;    // t is a start depot (cannot move): negative
    int tRemCap;   // t's route would exceed capacity without it... negative if not ok
    int tRemTw;    // t's route is late without it: negative
    int negTz, negTw;  // -edge(t), -(incident edges of t)
    int zx, zy;        // route load - demand, route load - prefix load of t
    // delta terms of the four moves with kPenalty added for a disabled
    // operator, for the delta-only pass
    int cRel, cRel2, cSwap, c2s;
};

// Raw column attributes of the chunk whose first owned column is slot cb
// (lanes 1..kColsPerWave own cb..cb+61; lanes 0 and 63 hold the
// neighbours), fetched ahead of their use.
struct ColRaw {
    int4 ta, tb, tt, tw;
};

template <bool TW>
__device__ __forceinline__ ColRaw col_fetch(const SolDev &S, int cb) {
    const int lane = threadIdx.x & 63;
    const int tc = min(max(cb - 1 + lane, 0), S.Q);
    ColRaw c;
    c.ta = gld(S.a4 + tc);
    c.tb = gld(S.b4 + tc);
    if (TW) {
        c.tt = gld(S.t4 + tc);
        c.tw = gld(S.w4 + tc);
    } else {
        c.tt = make_int4(0, 0, 0, 0);
        c.tw = make_int4(0, 0, 0, 0);
    }
    return c;
}

// Lane values of the chunk at cb from its raw attributes.  routeLast: route
// of the last owned column (-1 if none), wave-uniform.
__device__ __forceinline__ void col_setup(const SolDev &S, int cb, const ColRaw &c, uint32_t op_mask, LaneCol &L,
                                          int &routeLast) {
    const int lane = threadIdx.x & 63;
    const int Q = S.Q, n = S.n;
    const int t = cb - 1 + lane;
    L.ta = c.ta;
    L.tb = c.tb;
    L.tt = c.tt;
    L.tw = c.tw;
    L.node = nodeof(L.ta.x);
    const int fl = flagsof(L.ta.x);
    const bool cust = fl & kFlagCustomer;
    const bool own = lane >= 1 && lane <= kColsPerWave && t < Q;
    L.refT = cust ? L.node - 1 : n + L.ta.y;
    L.tyOwn = own ? L.ta.y - 1 : -(1 << 30);
    L.tInval = cust ? 0 : (int)0x80000000;
    L.tRemCap = (fl & kFlagRemCap) ? 0 : (int)0x80000000;
    L.tRemTw = (fl & kFlagRemTw) ? 0 : (int)0x80000000;
    L.negTz = -L.ta.z;
    L.negTw = -L.tb.w;
    L.zx = L.tb.z - L.tb.x;
    L.zy = L.tb.z - L.tb.y;
    const int offRel = (op_mask & 1) ? 0 : (1 << 30);
    const int offSwap = (op_mask & 2) ? 0 : (1 << 30);
    const int off2s = (op_mask & 4) ? 0 : (1 << 30);
    L.cRel = L.negTz + offRel;
    L.cRel2 = L.ta.w + offRel;
    L.cSwap = L.negTw + offSwap;
    L.c2s = L.negTz + off2s;
    const int lastLane = min(kColsPerWave, Q - cb);
    const int rl = __shfl(L.ta.y, max(lastLane, 0));
    routeLast = __builtin_amdgcn_readfirstlane(lastLane >= 1 ? rl : -1);
}

// ---- LDS block of distance rows of an inter-route item.  While the rows of
// a sub-block starting at row sb are evaluated, slot x (sb - 1 <= x <= the
// sub-block's last row + 1) sits at row position x - sb + 1; slots outside
// [0, Q] are read clamped.

// Distance rows of slots [x0, x0 + cnt) copied straight from HBM into the
// block (global_load_lds, four dwords per lane for 16-bit rows, else one),
// slot `base` at position 0,
// from the 16-bit copy of D when W16.  The issuing wavefront must wait
// (vmcnt) before a barrier publishes them.  `wave` is the wavefront index
// (uniform).
template <bool W16>
__device__ __forceinline__ void drow_issue(const SolDev &S, void *rows, int base, int x0, int cnt, int wave) {
    const int lane = threadIdx.x & 63;
    const int words = W16 ? S.stride16 / 2 : S.np1;  // dwords per row
    for (int r = wave; r < cnt; r += kInterWaves) {
        const int x = x0 + r;
        const int node = nodeof(sld(S.a4 + min(max(x, 0), S.Q)).x);
        const int *src = W16 ? (const int *)(S.D16 + (size_t)node * S.stride16) : S.D + (size_t)node * S.np1;
        int *dst = (int *)rows + (x - base) * words;
        if (W16) {  // rows are 16-byte aligned multiples of 16 bytes: four dwords per lane
            for (int c = 0; c < words; c += 256) {
                if (c + 4 * lane < words)
                    __builtin_amdgcn_global_load_lds((global_void_ptr)(src + c + 4 * lane), (lds_void_ptr)(dst + c), 16,
                                                     0, 0);
            }
        } else {
            for (int c = 0; c < words; c += 64) {
                if (c + lane < words)
                    __builtin_amdgcn_global_load_lds((global_void_ptr)(src + c + lane), (lds_void_ptr)(dst + c), 4, 0,
                                                     0);
            }
        }
    }
}

template <bool W16> struct DistElem { typedef int type; };
template <> struct DistElem<true> { typedef uint16_t type; };

constexpr int kSign = (int)0x80000000;
constexpr int kPenalty = 1 << 30;     // added to the delta of an inadmissible move
constexpr int kAdmissible = 1 << 29;  // every admissible delta is below this

// delta, plus kPenalty when viol < 0
__device__ __forceinline__ int penalise(int d, int viol) {
    return d + (int)(((uint32_t)viol >> 31) << 30);
}

// Row-side (scalar) values of one row slot s.
struct RowVals {
    int rs, refS;
    int sInval, sRemCap, sRemTw;   // 0 or negative, as the lane's
    int capA, capB, capC, capD, capE;
    int rw_ra, rz;                 // removal delta of s, edge(s)
    int rbw;                       // incident edges of s
};

__device__ __forceinline__ RowVals row_vals(const int4 &ra, const int4 &rb, int cap, int n) {
    RowVals R;
    const int fl = flagsof(ra.x);
    const bool cust = fl & kFlagCustomer;
    R.rs = ra.y;
    R.refS = cust ? nodeof(ra.x) - 1 : n + ra.y;
    R.sInval = cust ? 0 : kSign;
    R.sRemCap = (fl & kFlagRemCap) ? 0 : kSign;
    R.sRemTw = (fl & kFlagRemTw) ? 0 : kSign;
    R.capA = cap - rb.x;          // relocate s->t: load(t) <= capA; swap: load(t) - dem(t) <= capA
    R.capB = cap - rb.z;          // relocate t->s: dem(t) <= capB
    R.capC = cap - rb.z + rb.x;   // swap: dem(t) <= capC
    R.capD = cap - rb.y;          // 2-opt*: load(t) - prefix(t) <= capD
    R.capE = cap - rb.z + rb.y;   // 2-opt*: prefix(t) <= capE
    R.rw_ra = ra.w;
    R.rz = ra.z;
    R.rbw = rb.w;
    return R;
}

// The four inter-route moves of row slot s against the lane's column slot t:
// RELOCATE s -> after t, RELOCATE t -> after s, SWAP s <-> t, 2OPT*(s, t).
// g = D[s][t], gp = D[pred(s)][t], gn = D[succ(s)][t], gR = D[s][succ(t)],
// gL = D[s][pred(t)].  rt / rw: the row's time values and window (TW only).
template <bool TW, bool DUMP>
__device__ __forceinline__ void pair_moves(const LaneCol &L, const RowVals &R, const int4 &rt, const int4 &rw,
                                           int gp, int g, int gn, int gR, int gL, uint32_t uQ, bool opRel,
                                           bool opSwap, bool op2s, int32_t *__restrict__ dump_delta,
                                           uint8_t *__restrict__ dump_feas, int &bd, uint32_t &bid) {
    const int4 ta = L.ta, tb = L.tb, tt = L.tt, tw = L.tw;
    const int pairViol = L.tyOwn - R.rs;  // >= 0 iff the lane owns t and route(t) > route(s)

    // RELOCATE s -> right after t
    const int d1 = g + gR + L.negTz + R.rw_ra;
    const int cap1 = R.capA - tb.z;
    int tw1 = 0;
    if (TW) {
        const int arr = tt.x + g;
        const int st = max(arr, rw.x);
        tw1 = (rw.y - arr) | ((tt.y - rw.z) - (st + gR)) | R.sRemTw;
    }
    const int v1 = pairViol | R.sInval;
    const int e1 = penalise(d1, v1 | cap1 | R.sRemCap | tw1);

    // RELOCATE t -> right after s
    const int d2 = g + gn + ta.w - R.rz;
    const int cap2 = R.capB - tb.x;
    int tw2 = 0;
    if (TW) {
        const int arr = rt.x + g;
        const int st = max(arr, tw.x);
        tw2 = (tw.y - arr) | (rt.y - (st + tw.z + gn)) | L.tRemTw;
    }
    const int v2 = pairViol | L.tInval;
    const int e2 = penalise(d2, v2 | cap2 | L.tRemCap | tw2);

    // SWAP s <-> t
    const int d3 = gp + gn + gL + gR + L.negTw - R.rbw;
    const int cap3 = (R.capC - tb.x) | (R.capA - L.zx);
    int tw3 = 0;
    if (TW) {
        const int arrS = rt.z + gp;  // t placed where s was
        const int stS = max(arrS, tw.x);
        const int arrT = tt.z + gL;  // s placed where t was
        const int stT = max(arrT, rw.x);
        tw3 = (tw.y - arrS) | (rt.y - (stS + tw.z + gn)) | (rw.y - arrT) | (tt.y - (stT + rw.z + gR));
    }
    const int v3 = pairViol | R.sInval | L.tInval;
    const int e3 = penalise(d3, v3 | cap3 | tw3);

    // 2OPT*(s, t): heads keep their slots, tails are exchanged
    const int d4 = gR + gn + L.negTz - R.rz;
    const int cap4 = (R.capD - L.zy) | (R.capE - tb.y);
    int tw4 = 0;
    if (TW) tw4 = ((tt.y - gR) - rt.x) | ((rt.y - gn) - tt.x);
    const int e4 = penalise(d4, pairViol | cap4 | tw4);

    const uint32_t lo = min((uint32_t)R.refS, (uint32_t)L.refT), hi = max((uint32_t)R.refS, (uint32_t)L.refT);
    if (DUMP) {
        // exact feasibility bits of every valid move
        if (opRel && v1 >= 0) {
            const uint32_t id = (uQ + R.refS) * uQ + L.refT;
            dump_delta[id] = d1;
            dump_feas[id] = (uint8_t)(((cap1 | R.sRemCap) >= 0) | ((tw1 >= 0) << 1));
        }
        if (opRel && v2 >= 0) {
            const uint32_t id = (uQ + L.refT) * uQ + R.refS;
            dump_delta[id] = d2;
            dump_feas[id] = (uint8_t)(((cap2 | L.tRemCap) >= 0) | ((tw2 >= 0) << 1));
        }
        if (opSwap && v3 >= 0) {
            const uint32_t id = (5u * uQ + lo) * uQ + hi;
            dump_delta[id] = d3;
            dump_feas[id] = (uint8_t)((cap3 >= 0) | ((tw3 >= 0) << 1));
        }
        if (op2s && pairViol >= 0) {
            const uint32_t id = (8u * uQ + lo) * uQ + hi;
            dump_delta[id] = d4;
            dump_feas[id] = (uint8_t)((cap4 >= 0) | ((tw4 >= 0) << 1));
        }
    }
    const int m1 = opRel ? e1 : kNoDelta;
    const int m2 = opRel ? e2 : kNoDelta;
    const int m3 = opSwap ? e3 : kNoDelta;
    const int m4 = op2s ? e4 : kNoDelta;
    const int m = min(min(m1, m2), min(m3, m4));
    if (m <= bd) {  // rare: only an admissible move can reach bd (< kAdmissible)
        consider(m1, (uQ + R.refS) * uQ + L.refT, bd, bid);
        consider(m2, (uQ + L.refT) * uQ + R.refS, bd, bid);
        consider(m3, (5u * uQ + lo) * uQ + hi, bd, bid);
        consider(m4, (8u * uQ + lo) * uQ + hi, bd, bid);
    }
}

// Delta of the best admissible move committed so far for S (kAdmissibleBound
// if none): every workgroup working on S may skip moves that cannot beat it.
__device__ __forceinline__ int committed_delta(const SolDev &S) {
    const unsigned long long k = __hip_atomic_load(S.best_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return k == ~0ull ? kAdmissibleBound : (int)((uint32_t)(k >> 32) ^ 0x80000000u);
}

// The (column chunk, row) pairs of the sub-block of nr rows starting at slot
// sb, chunk-major, with chunks of kColsPerWave columns from slot sb + 1:
// [lo, hi) is the equal share of wavefront `wave`.
__device__ __forceinline__ void wave_share(int Q, int sb, int nr, int wave, int &lo, int &hi) {
    const int k = (Q - sb - 1 + kColsPerWave - 1) / kColsPerWave;
    const long long T = (long long)k * nr;
    lo = (int)(T * wave / kInterWaves);
    hi = (int)(T * (wave + 1) / kInterWaves);
}

// Whole-workgroup evaluation of one inter-route item: the row slots
// [s0, s1) against every column slot after the row.  The distance rows
// (16-bit when W16) are staged in LDS in sub-blocks of h = S.tile_rows rows
// plus a halo row on each side (one sub-block per item by default); row
// attributes are wave-uniform and come through the scalar cache, one row
// ahead of their use.  The (column chunk, row) pairs of a
// sub-block are split into kInterWaves equal contiguous runs, chunk-major, so
// every wavefront gets the same work whatever the shape of the triangle; the
// column attributes of a wavefront's next run are fetched while the current
// one is evaluated.
//
// Each pair first gets the deltas of its four moves only; the feasibility
// conditions and move ids are evaluated only where some delta is <= the
// run's threshold: the best any wavefront of the workgroup has published in
// LDS (thr_sh, read at the start of a run; each wavefront publishes its own
// best at the end of a run) or the solution has committed, bounded by the
// initial bound.  Every threshold is the delta of an admissible move of this
// neighbourhood (or the bound), so no move that could be the minimum (or tie
// with it) is ever skipped.
// With dump arrays every move is evaluated.  smem4 is the dynamic LDS area;
// red holds kInterWaves keys.
template <bool TW, bool DUMP, bool W16, bool CNT = false>
__device__ __forceinline__ void inter_item(const SolDev &S, const InterItem &item, uint32_t op_mask,
                           int32_t *__restrict__ dump_delta, uint8_t *__restrict__ dump_feas,
                           int4 *smem4, unsigned long long *red, int *thr_sh) {
    typedef typename DistElem<W16>::type DT;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const bool opRel = op_mask & 1, opSwap = op_mask & 2, op2s = op_mask & 4;
    const int Q = S.Q, np1 = S.np1, n = S.n, cap = S.cap, h = S.tile_rows;
    const uint32_t uQ = (uint32_t)Q;
    const int s0 = item.s0, s1 = item.s1;
    const int nsb = (s1 - s0 + h - 1) / h;
    const int NB = h + 2;
    const int rs = W16 ? S.stride16 : np1;  // row stride in LDS (elements)
    DT *rows = (DT *)smem4;
    const DT *rowsLast = rows + (NB - 1) * rs;  // the last row position

    int bd = initial_bound(op_mask);
    uint32_t bid = 0xFFFFFFFFu;
    uint32_t nfull = 0;  // CNT: this wavefront's pairs evaluated in full (wave-uniform)

    // prologue: the distance rows of sub-block 0 (with its halo rows)
    __syncthreads();  // the previous item is done with LDS
    if (!DUMP && threadIdx.x == 0) *thr_sh = committed_delta(S);
    drow_issue<W16>(S, rows, s0 - 1, s0 - 1, min(h, s1 - s0) + 2, wave);
    __builtin_amdgcn_s_waitcnt(0);

    ColRaw nxt;  // column attributes fetched ahead for the chunk at nxt_cb
    int nxt_cb = -1;
    for (int i = 0; i < nsb; ++i) {
        const int sb = s0 + i * h;
        const int nr = min(h, s1 - sb);  // rows of this sub-block
        __syncthreads();                 // rows of sub-block i resident (i = 0), or i - 1 consumed
        if (i > 0) {
            // The previous sub-block (h rows) ended with rows sb - 1 and sb
            // at positions h and h + 1: they become this one's first halo
            // row and first row, so only rows sb + 1 .. sb + nr come from
            // memory and a strip of sub-blocks reads each row once.
            {
                const int words = (int)((size_t)rs * sizeof(DT) / 4);  // dwords per row
                int *blk = (int *)rows;
                const int *from = blk + h * words;
                if (h >= 2) {  // positions h, h + 1 and 0, 1 do not overlap
                    for (int w = threadIdx.x; w < 2 * words; w += blockDim.x) blk[w] = from[w];
                } else {  // position 1 is source and destination: read a chunk, wait, write it
                    for (int w0 = 0; w0 < 2 * words; w0 += blockDim.x) {
                        const int w = w0 + threadIdx.x;
                        const int v = w < 2 * words ? from[w] : 0;
                        __syncthreads();
                        if (w < 2 * words) blk[w] = v;
                        __syncthreads();
                    }
                }
            }
            __syncthreads();
            drow_issue<W16>(S, rows, sb - 1, sb + 1, nr, wave);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        // columns: every slot after the sub-block's first row (pairs in the
        // same route are skipped per pair)
        if (sb + 1 < Q) {
            int idx, hi;
            wave_share(Q, sb, nr, wave, idx, hi);
            // run = (chunk j, rows [r0, r1)); every run after the first of a
            // share starts the next chunk at row 0
            int j = idx / nr, r0 = idx - j * nr;
            for (; idx < hi; ++j, r0 = 0) {
                const int r1 = min(nr, r0 + (hi - idx));
                idx += r1 - r0;
                const int cb = sb + 1 + j * kColsPerWave;
                const ColRaw cur = nxt_cb == cb ? nxt : col_fetch<TW>(S, cb);
                // fetch the chunk of this wavefront's next run (here or in a
                // later sub-block) while this one is evaluated
                int cb2 = -1;
                if (idx < hi) {
                    cb2 = cb + kColsPerWave;
                } else {
                    for (int i2 = i + 1; i2 < nsb && cb2 < 0; ++i2) {
                        const int sb2 = s0 + i2 * h, nr2 = min(h, s1 - sb2);
                        int lo2, hi2;
                        if (sb2 + 1 >= Q) break;
                        wave_share(Q, sb2, nr2, wave, lo2, hi2);
                        if (lo2 < hi2) cb2 = sb2 + 1 + (lo2 / nr2) * kColsPerWave;
                    }
                }
                if (cb2 >= 0 && cb2 != cb) nxt = col_fetch<TW>(S, cb2);
                else if (cb2 == cb) nxt = cur;
                nxt_cb = cb2;
                LaneCol L;
                int routeLast;
                col_setup(S, cb, cur, op_mask, L, routeLast);
                int x = sb + r0;  // row slot
                // rows whose route precedes the chunk's last route (slots are
                // route-major, so those before that route's first slot), at
                // most up to the end of the run
                const int xlim = routeLast >= 0 ? min(sb + r1, sld1(S.roff + routeLast)) : x;
                // register window over the distance rows: x - 1, x, x + 1
                const DT *pp = rows + (x - sb) * rs;
                int gp = pp[L.node];
                pp += rs;
                int g = pp[L.node];
                pp += rs;
                int gn = pp[L.node];
                uint32_t ro = (uint32_t)x * 16u;  // byte offset of row x's slot attributes
                int4 ra = sld_at(S.a4, ro), rb = sld_at(S.b4, ro);
                const int thrRun = DUMP ? 0 : __hip_atomic_load(thr_sh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                // The passes screen against the run's threshold alone (the delta
                // of an admissible move, or the initial bound): a lane's own
                // better move found during the run tightens it only from the
                // next run, which saves an instruction per pass and lets a few
                // more pairs into the full evaluation.
                const int thrScreen = min(thrRun, initial_bound(op_mask));
                // Each pass first consumes what the previous one fetched, then
                // fetches row x + 1 (attributes) and the gather of row x + 2,
                // then evaluates row x from registers (the rare full
                // evaluation also reads the row's time attributes).  Passes
                // go in fours so that the two sets of row attributes and the
                // four window registers take turns without copies.
                auto pass = [&](const int4 &rA, const int4 &rB, int4 &rAn, int4 &rBn, int wp, int w0, int wn,
                                int &wnn) {
                    pp = min(pp + rs, rowsLast);
                    wnn = pp[L.node];  // row x + 2 (past the halo on the last row: unused)
                    rAn = sld_at(S.a4, ro + 16u);  // x + 1 <= Q
                    rBn = sld_at(S.b4, ro + 16u);
                    const int gR = from_next_lane(w0);  // D[s][succ(t)]
                    const int gL = from_prev_lane(w0);  // D[s][pred(t)]
                    bool full = true;
                    if (!DUMP) {
                        const int thr = thrScreen;
                        const int wz = wn - rA.z;  // shared by RELOCATE t -> s and 2OPT*
                        const int d1 = w0 + gR + (L.cRel + rA.w);
                        const int d2 = w0 + wz + L.cRel2;
                        const int d3 = (wp + wn) + gL + (gR + (L.cSwap - rB.w));
                        const int d4 = gR + wz + L.c2s;
                        const int m = min(min(d1, d2), min(d3, d4));
                        full = m <= thr && L.tyOwn >= rA.y;
                        if (full) {
                            // capacity screen: a move whose capacity condition
                            // fails is inadmissible whatever its delta (most
                            // screened-in moves late in a search are such)
                            const int capA = cap - rB.x, capB = cap - rB.z;
                            const int e1 = (capA - L.tb.z) >= 0 ? d1 : kNoDelta;
                            const int e2 = (capB - L.tb.x) >= 0 ? d2 : kNoDelta;
                            const int e3 = ((capB + rB.x - L.tb.x) | (capA - L.zx)) >= 0 ? d3 : kNoDelta;
                            const int e4 = ((cap - rB.y - L.zy) | (capB + rB.y - L.tb.y)) >= 0 ? d4 : kNoDelta;
                            full = min(min(e1, e2), min(e3, e4)) <= thr;
                        }
                        if (CNT) nfull += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(full));
                    }
                    if (full) {
                        int4 rt = make_int4(0, 0, 0, 0), rw = make_int4(0, 0, 0, 0);
                        if (TW) {
                            rt = sld_at(S.t4, ro);
                            rw = sld_at(S.w4, ro);
                        }
                        const RowVals R = row_vals(rA, rB, cap, n);
                        pair_moves<TW, DUMP>(L, R, rt, rw, wp, w0, wn, gR, gL, uQ, opRel, opSwap, op2s, dump_delta,
                                             dump_feas, bd, bid);
                    }
                    ++x;
                    ro += 16u;
                };
                int4 ra2, rb2;
                int g3 = 0;
                // four passes per iteration: the four window registers take
                // turns, so the window is back in gp, g, gn without copies
                for (int q = (xlim - x) >> 2; q > 0; --q) {  // whole groups of four rows
                    pass(ra, rb, ra2, rb2, gp, g, gn, g3);  // rows x - 1, x, x + 1; fetches x + 2
                    pass(ra2, rb2, ra, rb, g, gn, g3, gp);
                    pass(ra, rb, ra2, rb2, gn, g3, gp, g);
                    pass(ra2, rb2, ra, rb, g3, gp, g, gn);
                }
                if (x < xlim) {  // the last one to three rows
                    pass(ra, rb, ra2, rb2, gp, g, gn, g3);
                    if (x < xlim) {
                        pass(ra2, rb2, ra, rb, g, gn, g3, gp);
                        if (x < xlim) pass(ra, rb, ra2, rb2, gn, g3, gp, g);
                    }
                }
                // publish this wavefront's best to the workgroup (one lane, one
                // LDS atomic, only when some lane improved on the shared value)
                if (!DUMP && __builtin_amdgcn_ballot_w64(bd < thrRun)) {
                    int wmin = bd;
#pragma unroll
                    for (int off = 32; off >= 1; off >>= 1) wmin = min(wmin, __shfl_xor(wmin, off));
                    if (lane == 0) atomicMin(thr_sh, wmin);
                }
            }
        }
    }
    if (CNT && !DUMP && (op_mask & kImprovingOnly) && lane == 0 && nfull)
        atomicAdd((unsigned long long *)(S.acc + kAccFullPairs), (unsigned long long)nfull);
    block_argmin_commit(bd, bid, S.best_key, red);
}

template <bool TW, bool DUMP>
__global__ __launch_bounds__(kInterThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_inter(const SolDev *__restrict__ sols,
                                                              const InterItem *__restrict__ items,
                                                              int nitems, uint32_t op_mask,
                                                              int32_t *__restrict__ dump_delta,
                                                              uint8_t *__restrict__ dump_feas) {
    extern __shared__ int4 smem4[];
    __shared__ unsigned long long red[kInterWaves];
    __shared__ int thr_sh;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const InterItem item = items[it];
        const SolDev &S = sols[item.sol];
        if (skip_solution(S, op_mask)) continue;
        if (S.D16)
            inter_item<TW, DUMP, true>(S, item, op_mask, dump_delta, dump_feas, smem4, red, &thr_sh);
        else
            inter_item<TW, DUMP, false>(S, item, op_mask, dump_delta, dump_feas, smem4, red, &thr_sh);
    }
}

// ------------------------------------------- granular inter-route eval ---
// Edge-based extraction (Section 5.3.1): only the node pairs kept by the
// granular mask, the symmetric closure of each node's theta nearest
// neighbours, get their inter-route moves evaluated.  The mask is an
// adjacency list over nodes 0..n (CSR; node 0 is the depot and stands for
// the start depot of every route).  One thread per adjacency entry (u, v) of
// a customer u: the pair of slots (slot(u), slot(v)) is evaluated by the
// entry whose row route comes first (each pair once, as in the full kernel:
// row route < column route); an entry (u, depot) evaluates u against the
// start depot of every other route.  The depot's own row is never walked:
// its pairs are those of its customers.  Attributes are gathered per thread
// (no LDS staging): E is small next to the Q^2 pairs of the full
// neighbourhood.

// Column attributes of slot t for one thread (the fields pair_moves reads).
__device__ __forceinline__ void lane_col_single(const SolDev &S, int t, LaneCol &L) {
    L.ta = gld(S.a4 + t);
    L.tb = gld(S.b4 + t);
    if (S.has_tw) {
        L.tt = gld(S.t4 + t);
        L.tw = gld(S.w4 + t);
    } else {
        L.tt = make_int4(0, 0, 0, 0);
        L.tw = make_int4(0, 0, 0, 0);
    }
    L.node = nodeof(L.ta.x);
    const int fl = flagsof(L.ta.x);
    const bool cust = fl & kFlagCustomer;
    L.refT = cust ? L.node - 1 : S.n + L.ta.y;
    L.tyOwn = L.ta.y - 1;
    L.tInval = cust ? 0 : (int)0x80000000;
    L.tRemCap = (fl & kFlagRemCap) ? 0 : (int)0x80000000;
    L.tRemTw = (fl & kFlagRemTw) ? 0 : (int)0x80000000;
    L.negTz = -L.ta.z;
    L.negTw = -L.tb.w;
    L.zx = L.tb.z - L.tb.x;
    L.zy = L.tb.z - L.tb.y;
}

// The four inter-route moves of row slot x against column slot t (route(x)
// < route(t)), with every attribute gathered from the slot arrays and D.
// Returns the number of moves of N_theta(S) the pair stands for.
template <bool TW, bool DUMP>
__device__ __forceinline__ int gran_pair(const SolDev &S, int x, int t, uint32_t op_mask,
                                         int32_t *__restrict__ dump_delta, uint8_t *__restrict__ dump_feas,
                                         int &bd, uint32_t &bid) {
    const bool opRel = op_mask & 1, opSwap = op_mask & 2, op2s = op_mask & 4;
    LaneCol L;
    lane_col_single(S, t, L);
    const int4 ra = gld(S.a4 + x), rb = gld(S.b4 + x);
    int4 rt = make_int4(0, 0, 0, 0), rw = make_int4(0, 0, 0, 0);
    if (TW) {
        rt = gld(S.t4 + x);
        rw = gld(S.w4 + x);
    }
    const RowVals R = row_vals(ra, rb, S.cap, S.n);
    const int np1 = S.np1;
    const int nx = nodeof(ra.x), npx = nodeof(gld(S.a4 + max(x - 1, 0)).x), nsx = nodeof(gld(S.a4 + x + 1).x);
    const int nt = L.node, npt = nodeof(gld(S.a4 + t - 1).x), nst = nodeof(gld(S.a4 + t + 1).x);
    const int32_t *D = S.D;
    const int g = gld(D + (size_t)nx * np1 + nt), gp = gld(D + (size_t)npx * np1 + nt),
              gn = gld(D + (size_t)nsx * np1 + nt), gR = gld(D + (size_t)nx * np1 + nst),
              gL = gld(D + (size_t)nx * np1 + npt);
    pair_moves<TW, DUMP>(L, R, rt, rw, gp, g, gn, gR, gL, (uint32_t)S.Q, opRel, opSwap, op2s, dump_delta,
                         dump_feas, bd, bid);
    const bool cx = R.sInval == 0, ct = L.tInval == 0;
    return (opRel ? (int)cx + (int)ct : 0) + (opSwap && cx && ct ? 1 : 0) + (op2s ? 1 : 0);
}

// Work items: e < gcc, a customer-customer adjacency entry (gsrc[e],
// gadj[e]); gcc <= e < gcc + gdep * R, customer gsrc[gcc + (e - gcc) / R]
// (one the depot is paired with) against the start depot of route
// (e - gcc) % R, so that no thread walks every route.  The inter-route moves
// of N_theta(S) evaluated are added to S.acc[kAccGranInter].
// One block of work items, item e for this thread (every thread of the
// block calls it; red holds blockDim / 64 keys).
template <bool TW, bool DUMP>
__device__ __forceinline__ void gran_block(const SolDev &S, const int32_t *__restrict__ gsrc,
                                           const int32_t *__restrict__ gadj, int gcc, int gdep, int e,
                                           uint32_t op_mask, int32_t *__restrict__ dump_delta,
                                           uint8_t *__restrict__ dump_feas, unsigned long long *red,
                                           long long *cnt_sh) {
    if (threadIdx.x == 0) *cnt_sh = 0;
    __syncthreads();
    int bd = DUMP ? kAdmissibleBound : initial_bound(op_mask);
    uint32_t bid = 0xFFFFFFFFu;
    long long cnt = 0;
    if (e < gcc) {
        const int x = gld(S.ref2slot + gsrc[e] - 1), t = gld(S.ref2slot + gadj[e] - 1);
        if (gld(S.a4 + t).y > gld(S.a4 + x).y)
            cnt += gran_pair<TW, DUMP>(S, x, t, op_mask, dump_delta, dump_feas, bd, bid);
    } else if (e - gcc < gdep * S.R) {
        const int k = (e - gcc) / S.R, r = (e - gcc) - k * S.R;
        const int x = gld(S.ref2slot + gsrc[gcc + k] - 1);
        const int rx = gld(S.a4 + x).y;
        if (r != rx) {
            const int d = gld(S.roff + r);  // start depot slot of route r
            cnt += r > rx ? gran_pair<TW, DUMP>(S, x, d, op_mask, dump_delta, dump_feas, bd, bid)
                          : gran_pair<TW, DUMP>(S, d, x, op_mask, dump_delta, dump_feas, bd, bid);
        }
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd((unsigned long long *)cnt_sh, (unsigned long long)cnt);
    block_argmin_commit(bd, bid, S.best_key, red);  // its barriers also order cnt_sh
    if (threadIdx.x == 0 && *cnt_sh) atomicAdd((unsigned long long *)(S.acc + kAccGranInter), (unsigned long long)*cnt_sh);
}

template <bool TW, bool DUMP>
__global__ __launch_bounds__(256) void k_eval_gran(const SolDev *__restrict__ sols, const int32_t *__restrict__ gsrc,
                                                   const int32_t *__restrict__ gadj, int gcc, int gdep,
                                                   uint32_t op_mask, int32_t *__restrict__ dump_delta,
                                                   uint8_t *__restrict__ dump_feas) {
    __shared__ unsigned long long red[256 / 64];
    __shared__ long long cnt_sh;
    const SolDev &S = sols[0];
    if (skip_solution(S, op_mask)) return;  // uniform for the grid
    gran_block<TW, DUMP>(S, gsrc, gadj, gcc, gdep, blockIdx.x * blockDim.x + threadIdx.x, op_mask, dump_delta,
                         dump_feas, red, &cnt_sh);
}

// ------------------------------------------- penalised-mode evaluation ---
// Feasible and infeasible search (Alg. A2): every move of N(S) is admissible
// and scores dD + w_L dL_V + w_T dT_V over the touched routes (Section 5.3.3
// attribute deltas, eq. scoring_tensor).  New routes are concatenations of
// the stored prefix / suffix summaries with the moved nodes (Section 4.3.3);
// loads come from the prefix loads.  One thread per pair of slots (inter-
// route) or per first position of an intra-route walk: the attributes are
// gathered, nothing is staged (this mode serves the search, not the
// headline rate).  The dumps hold the score and the hard capacity / window
// bits of the touched routes (load excess and time warp both zero).

// Suffix summary strictly after slot x (the end depot when x is last).
__device__ __forceinline__ Tw tw_after(const SolDev &S, int x, const Tw &dep) {
    return nodeof(gld(S.a4 + x + 1).x) == 0 ? dep : tw_of(gld(S.pb4 + x + 1));
}

__device__ __forceinline__ Tw tw_node_at(const SolDev &S, int x) {
    const int4 w = gld(S.w4 + x);
    return tw_node(w.x, w.y, w.z);
}

// Record one move of the general path.  Penalised mode: the score is
// dD + w_L dL_V + w_T dT_V and every move is admissible.  Otherwise (pickups
// with hard feasibility): the distance delta, admissible when the touched
// routes have no load excess and no time warp.  The dumps hold the score
// (penalised) or the delta, and the hard capacity / window bits.
__device__ __forceinline__ void gen_record(const SolDev &S, int dD, int dlv, int dtv, bool capok, bool twok, uint32_t id,
                                           bool dump, int32_t *dd, uint8_t *df, int &bd, uint32_t &bid) {
    const int feas = (capok ? 1 : 0) | (twok ? 2 : 0);
    const int score = S.pen ? dD + S.wL * dlv + S.wT * dtv : dD;
    if (dump) {
        dd[id] = score;
        df[id] = (uint8_t)feas;
    }
    consider(S.pen || feas == 3 ? score : score + kPenalty, id, bd, bid);
}

// Load summary strictly after slot x (the end depot: empty, when x is last).
__device__ __forceinline__ Ld ld_after(const SolDev &S, int x) {
    return nodeof(gld(S.a4 + x + 1).x) == 0 ? Ld{0, 0, 0} : ld_of(gld(S.ql4 + x + 1));
}

// Distances of a 16 x 16 pair tile, staged in LDS: Dc[i][j] between the
// row-side slot x0 - 1 + i and the column-side slot t0 - 1 + j (i, j < 20),
// Rr[i][k - 1] between row-side slots x0 - 1 + i and x0 - 1 + i + k
// (k = 1..4), Cc likewise on the column side.  Every distance a pair's
// moves need is one of these (segments reach three slots past x or t).
constexpr int kTileSpan = 20;
struct PairTileD {
    int Dc[kTileSpan][kTileSpan];
    int Rr[kTileSpan][4];
    int Cc[kTileSpan][4];
};

// The inter-route moves of slots x, t (route(x) < route(t)); T holds the
// tile's distances, xi = x - x0 + 1 and tj = t - t0 + 1 locate the pair.
template <bool TW, bool PD, bool DUMP>
__device__ __forceinline__ void pen_pair(const SolDev &S, int x, int t, const PairTileD &T, int xi, int tj,
                                         uint32_t op_mask, int32_t *dd, uint8_t *df, int &bd, uint32_t &bid,
                                         int &cntExt) {
    const int n = S.n, cap = S.cap;
    const uint32_t uQ = (uint32_t)S.Q;
    const int4 ax = gld(S.a4 + x), at = gld(S.a4 + t), bx = gld(S.b4 + x), bt = gld(S.b4 + t);
    const bool cx = flagsof(ax.x) & kFlagCustomer, ct = flagsof(at.x) & kFlagCustomer;
    const int nx = nodeof(ax.x), nt = nodeof(at.x);
    // X(a, b): distance between slots x + a and t + b; RX(a, k): between
    // x + a and x + a + k; CT likewise on t's side
    auto X = [&](int a, int b) { return T.Dc[xi + a][tj + b]; };
    auto RX = [&](int a, int k) { return T.Rr[xi + a][k - 1]; };
    auto CT = [&](int b, int k) { return T.Cc[tj + b][k - 1]; };
    const int refX = cx ? nx - 1 : n + ax.y, refT = ct ? nt - 1 : n + at.y;
    const int Lx = bx.z, Lt = bt.z, dx = bx.x, dtt = bt.x;
    const int lvOld = route_excess(S, ax.y) + route_excess(S, at.y);
    int tvOld = 0;
    Tw dep{}, Fx{}, Ft{}, Fpx{}, Fpt{}, Bax{}, Bat{}, Nx{}, Nt{};
    if (TW) {
        dep = tw_depot(S);
        Fx = tw_of(gld(S.pf4 + x));
        Ft = tw_of(gld(S.pf4 + t));
        Fpx = tw_of(gld(S.pf4 + max(x - 1, 0)));
        Fpt = tw_of(gld(S.pf4 + t - 1));
        Bax = tw_after(S, x, dep);
        Bat = tw_after(S, t, dep);
        Nx = tw_node_at(S, x);
        Nt = tw_node_at(S, t);
        tvOld = route_warp(S, ax.y) + route_warp(S, at.y);
    }
    Ld Px{}, Pt{}, Ppx{}, Ppt{}, Sax{}, Sat{}, Mx{}, Mt{};
    if (PD) {
        Px = ld_of(gld(S.pl4 + x));
        Pt = ld_of(gld(S.pl4 + t));
        Ppx = ld_of(gld(S.pl4 + max(x - 1, 0)));
        Ppt = ld_of(gld(S.pl4 + t - 1));
        Sax = ld_after(S, x);
        Sat = ld_after(S, t);
        Mx = ld_node_at(S, x);
        Mt = ld_node_at(S, t);
    }
    const int exx = RX(0, 1), ett = CT(0, 1);  // edges leaving x and t
    // peak loads of the two new routes are passed in (lx, lt)
    auto rec = [&](int dD, int lx, int lt, int tvx, int tvt, uint32_t id) {
        const int lv = max(lx - cap, 0) + max(lt - cap, 0);
        gen_record(S, dD, lv - lvOld, tvx + tvt - tvOld, lv == 0, tvx + tvt == 0, id, DUMP, dd, df, bd, bid);
    };
    if ((op_mask & 1) && cx) {  // RELOCATE x -> right after t
        const int dD = X(0, 0) + X(0, 1) - ett + RX(-1, 2) - RX(-1, 1) - exx;
        const int tvx = TW ? tw_cat(Fpx, RX(-1, 2), Bax).v : 0;
        const int tvt = TW ? tw_cat(tw_cat(Ft, X(0, 0), Nx), X(0, 1), Bat).v : 0;
        const int lx = PD ? ld_cat(Ppx, Sax).lm : Lx - dx;
        const int lt = PD ? ld_cat(ld_cat(Pt, Mx), Sat).lm : Lt + dx;
        rec(dD, lx, lt, tvx, tvt, (uQ + (uint32_t)refX) * uQ + (uint32_t)refT);
    }
    if ((op_mask & 1) && ct) {  // RELOCATE t -> right after x
        const int dD = X(0, 0) + X(1, 0) - exx + CT(-1, 2) - CT(-1, 1) - ett;
        const int tvx = TW ? tw_cat(tw_cat(Fx, X(0, 0), Nt), X(1, 0), Bax).v : 0;
        const int tvt = TW ? tw_cat(Fpt, CT(-1, 2), Bat).v : 0;
        const int lx = PD ? ld_cat(ld_cat(Px, Mt), Sax).lm : Lx + dtt;
        const int lt = PD ? ld_cat(Ppt, Sat).lm : Lt - dtt;
        rec(dD, lx, lt, tvx, tvt, (uQ + (uint32_t)refT) * uQ + (uint32_t)refX);
    }
    const uint32_t lo = min((uint32_t)refX, (uint32_t)refT), hi = max((uint32_t)refX, (uint32_t)refT);
    if ((op_mask & 2) && cx && ct) {  // SWAP x <-> t
        const int dD = X(-1, 0) + X(1, 0) + X(0, -1) + X(0, 1) - RX(-1, 1) - exx - CT(-1, 1) - ett;
        const int tvx = TW ? tw_cat(tw_cat(Fpx, X(-1, 0), Nt), X(1, 0), Bax).v : 0;
        const int tvt = TW ? tw_cat(tw_cat(Fpt, X(0, -1), Nx), X(0, 1), Bat).v : 0;
        const int lx = PD ? ld_cat(ld_cat(Ppx, Mt), Sax).lm : Lx - dx + dtt;
        const int lt = PD ? ld_cat(ld_cat(Ppt, Mx), Sat).lm : Lt - dtt + dx;
        rec(dD, lx, lt, tvx, tvt, (5u * uQ + lo) * uQ + hi);
    }
    if (op_mask & 4) {  // 2OPT*: heads keep their routes, tails exchanged
        const int dD = X(0, 1) + X(1, 0) - exx - ett;
        const int tvx = TW ? tw_cat(Fx, X(0, 1), Bat).v : 0;
        const int tvt = TW ? tw_cat(Ft, X(1, 0), Bax).v : 0;
        const int lx = PD ? ld_cat(Px, Sat).lm : bx.y + (Lt - bt.y);
        const int lt = PD ? ld_cat(Pt, Sax).lm : bt.y + (Lx - bx.y);
        rec(dD, lx, lt, tvx, tvt, (8u * uQ + lo) * uQ + hi);
    }
    if (!(op_mask & 0xE0u)) return;
    // ---- operator variants: segments of up to three customers starting at
    // x and at t (kept and reversed summaries, the slot after each segment)
    struct Seg3 {
        int k;         // customers available from the slot on, within its route (<= 3)
        int dem[3];    // deliveries of the first k customers
        Tw f[3], r[3];
        Ld lf[3], lr[3];
        Tw sa[3];
        Ld la[3];
    };
    auto seg3 = [&](int y, Seg3 &g) {
        const int last = gld(S.roff + gld(S.a4 + y).y + 1) - 1;
        g.k = min(3, last - y + 1);
        int dsum = 0;
        for (int q = 0; q < 3; ++q) {
            const bool in = q < g.k;
            dsum += in ? gld(S.b4 + y + q).x : 0;
            g.dem[q] = dsum;
            if (!in) continue;
            if (TW) {
                const Tw nq = tw_node_at(S, y + q);
                g.f[q] = q == 0 ? nq : tw_cat(g.f[q - 1], gld(S.a4 + y + q - 1).z, nq);
                g.r[q] = q == 0 ? nq : tw_cat(nq, gld(S.a4 + y + q - 1).z, g.r[q - 1]);
                g.sa[q] = tw_after(S, y + q, dep);
            }
            if (PD) {
                const Ld lq = ld_node_at(S, y + q);
                g.lf[q] = q == 0 ? lq : ld_cat(g.lf[q - 1], lq);
                g.lr[q] = q == 0 ? lq : ld_cat(lq, g.lr[q - 1]);
                g.la[q] = ld_after(S, y + q);
            }
        }
    };
    Seg3 gx, gt;
    if (cx) seg3(x, gx);
    if (ct) seg3(t, gt);
    // SEGMENT RELOCATE (op 5 kept, op 6 reversed), k = 2, 3: the segment
    // starting at slot y of route `from` (prefix summaries before it Fp /
    // Pp, route load Lf) moves right after slot z of route `to` (prefix Fy /
    // Py, suffix after it Bay / Say, route load Lto); (y, z) = (x, t) when
    // fromIsX, else (t, x).
    auto segrel = [&](const Seg3 &g, const Tw &Fp, const Ld &Pp, int Lf, const Tw &Fy, const Ld &Py, const Tw &Bay,
                      const Ld &Say, int Lto, bool fromIsX, uint32_t refA, uint32_t refB) {
        auto rf = [&](int a, int k) { return fromIsX ? RX(a, k) : CT(a, k); };  // within `from`
        auto rt = [&](int b, int k) { return fromIsX ? CT(b, k) : RX(b, k); };  // within `to`
        auto cr = [&](int a, int b) { return fromIsX ? X(a, b) : X(b, a); };    // y + a and z + b
        for (int k = 2; k <= g.k; ++k) {
            const int cut = rf(-1, k + 1) - rf(-1, 1) - rf(k - 1, 1);
            for (int op = 5; op <= 6; ++op) {
                if (!(op_mask & (op == 5 ? 32u : 64u))) continue;
                const int first = op == 5 ? 0 : k - 1, lastp = op == 5 ? k - 1 : 0;  // offsets from y
                const int dD = cut + cr(first, 0) + cr(lastp, 1) - rt(0, 1);
                int tvFrom = 0, tvTo = 0;
                if (TW) {
                    tvFrom = tw_cat(Fp, rf(-1, k + 1), g.sa[k - 1]).v;
                    tvTo = tw_cat(tw_cat(Fy, cr(first, 0), op == 5 ? g.f[k - 1] : g.r[k - 1]), cr(lastp, 1), Bay).v;
                }
                const int lFrom = PD ? ld_cat(Pp, g.la[k - 1]).lm : Lf - g.dem[k - 1];
                const int lTo = PD ? ld_cat(ld_cat(Py, op == 5 ? g.lf[k - 1] : g.lr[k - 1]), Say).lm : Lto + g.dem[k - 1];
                const uint32_t id = (((uint32_t)op * 4u + (uint32_t)k) * uQ + refA) * uQ + refB;
                if (fromIsX)
                    rec(dD, lFrom, lTo, tvFrom, tvTo, id);
                else
                    rec(dD, lTo, lFrom, tvTo, tvFrom, id);
                ++cntExt;
            }
        }
    };
    if (cx) segrel(gx, Fpx, Ppx, Lx, Ft, Pt, Bat, Sat, Lt, true, (uint32_t)refX, (uint32_t)refT);
    if (ct) segrel(gt, Fpt, Ppt, Lt, Fx, Px, Bax, Sax, Lx, false, (uint32_t)refT, (uint32_t)refX);
    // CROSS-EXCHANGE (ops 7..9): x's first ka customers and t's first kb
    if ((op_mask & 128u) && cx && ct) {
        for (int ka = 1; ka <= gx.k; ++ka)
            for (int kb = 1; kb <= gt.k; ++kb) {
                if (ka == 1 && kb == 1) continue;
                // segment x .. x + ka - 1 and t .. t + kb - 1 exchanged
                const int dD = X(-1, 0) + X(ka, kb - 1) + X(0, -1) + X(ka - 1, kb) - RX(-1, 1) - RX(ka - 1, 1) -
                               CT(-1, 1) - CT(kb - 1, 1);
                int tvx = 0, tvt = 0;
                if (TW) {
                    tvx = tw_cat(tw_cat(Fpx, X(-1, 0), gt.f[kb - 1]), X(ka, kb - 1), gx.sa[ka - 1]).v;
                    tvt = tw_cat(tw_cat(Fpt, X(0, -1), gx.f[ka - 1]), X(ka - 1, kb), gt.sa[kb - 1]).v;
                }
                const int lx = PD ? ld_cat(ld_cat(Ppx, gt.lf[kb - 1]), gx.la[ka - 1]).lm
                                  : Lx - gx.dem[ka - 1] + gt.dem[kb - 1];
                const int lt = PD ? ld_cat(ld_cat(Ppt, gx.lf[ka - 1]), gt.la[kb - 1]).lm
                                  : Lt - gt.dem[kb - 1] + gx.dem[ka - 1];
                const bool xFirst = refX < refT;
                const uint32_t op = 6u + (uint32_t)(xFirst ? ka : kb), k = (uint32_t)(xFirst ? kb : ka);
                rec(dD, lx, lt, tvx, tvt, ((op * 4u + k) * uQ + lo) * uQ + hi);
                ++cntExt;
            }
    }
}

// Inter-route pairs: 16 x 16 tiles of (row slot, column slot) on and above
// the diagonal, blockIdx.x enumerating the tiles row by row.
template <bool TW, bool PD, bool DUMP>
__global__ __launch_bounds__(256) void k_eval_pen_pairs(const SolDev *__restrict__ sols, int tiles, uint32_t op_mask,
                                                        int32_t *__restrict__ dd, uint8_t *__restrict__ df) {
    __shared__ unsigned long long red[4];
    const SolDev &S = sols[0];
    if (skip_solution(S, op_mask)) return;
    int bi = 0, rem = blockIdx.x;  // tile row bi holds tiles - bi tiles
    while (rem >= tiles - bi) {
        rem -= tiles - bi;
        ++bi;
    }
    const int bj = bi + rem;
    const int x0 = bi * 16, t0 = bj * 16;
    const int x = x0 + (threadIdx.x >> 4), t = t0 + (threadIdx.x & 15);
    // the tile's distances: nodes of slots x0 - 1 .. x0 + 22 and t0 - 1 ..
    // t0 + 22 (clamped to [0, Q]), then one gather per distance
    __shared__ PairTileD T;
    __shared__ int nodeX[kTileSpan + 4], nodeT[kTileSpan + 4];
    {
        const int Q = S.Q, np1 = S.np1;
        const int32_t *D = S.D;
        const int i = threadIdx.x;
        if (i < kTileSpan + 4) nodeX[i] = nodeof(gld(S.a4 + min(max(x0 - 1 + i, 0), Q)).x);
        else if (i >= 32 && i < 32 + kTileSpan + 4)
            nodeT[i - 32] = nodeof(gld(S.a4 + min(max(t0 - 1 + i - 32, 0), Q)).x);
        __syncthreads();
        for (int e = threadIdx.x; e < kTileSpan * kTileSpan; e += blockDim.x) {
            const int a = e / kTileSpan, b = e - a * kTileSpan;
            T.Dc[a][b] = gld(D + (size_t)nodeX[a] * np1 + nodeT[b]);
        }
        for (int e = threadIdx.x; e < 2 * kTileSpan * 4; e += blockDim.x) {
            const int side = e / (kTileSpan * 4), a = (e / 4) % kTileSpan, k = e % 4 + 1;
            const int *nd = side ? nodeT : nodeX;
            const int v = gld(D + (size_t)nd[a] * np1 + nd[a + k]);
            if (side) T.Cc[a][k - 1] = v;
            else T.Rr[a][k - 1] = v;
        }
        __syncthreads();
    }
    int bd = DUMP ? kAdmissibleBound : initial_bound(op_mask);
    uint32_t bid = 0xFFFFFFFFu;
    int ext = 0;  // operator-variant moves of this thread's pair
    if (x < S.Q && t < S.Q && gld(S.a4 + x).y < gld(S.a4 + t).y) {
        pen_pair<TW, PD, DUMP>(S, x, t, T, x - x0 + 1, t - t0 + 1, op_mask, dd, df, bd, bid, ext);
        // every move of this pair of slots touches exactly their two routes
        if ((op_mask & kMulti) && bd < 0 && bid != 0xFFFFFFFFu)
            atomicMin(S.pairkey + (size_t)gld(S.a4 + x).y * S.R + gld(S.a4 + t).y, pack_key(bd, bid));
    }
    if (op_mask & 0xE0u) {  // one atomic per workgroup
        __shared__ int ext_sh;
        if (threadIdx.x == 0) ext_sh = 0;
        __syncthreads();
        for (int off = 32; off >= 1; off >>= 1) ext += __shfl_xor(ext, off);
        if ((threadIdx.x & 63) == 0 && ext) atomicAdd(&ext_sh, ext);
        __syncthreads();
        if (threadIdx.x == 0 && ext_sh) atomicAdd((unsigned long long *)(S.acc + kAccExtMoves), (unsigned long long)ext_sh);
    }
    block_argmin_commit(bd, bid, S.best_key, red);
}

// Intra-route moves whose first position is the customer at slot s: the
// 2-opt / same-route swap walk and the or-opt walks, the middle summaries
// (time warp and, with pickups, load) growing one node per step.  Seven
// threads per slot, one walk each (walk 0: 2-opt / swap; 1..3: or-opt of
// k = walk nodes moved forward; 4..6: k = walk - 3 moved backward), so that a
// launch has seven times the threads and each its own short chain.
template <bool TW, bool PD, bool DUMP>
__global__ __launch_bounds__(256) void k_eval_pen_intra(const SolDev *__restrict__ sols, uint32_t op_mask,
                                                        int32_t *__restrict__ dd, uint8_t *__restrict__ df) {
    __shared__ unsigned long long red[4];
    const SolDev &S = sols[0];
    if (skip_solution(S, op_mask)) return;
    int bd = DUMP ? kAdmissibleBound : initial_bound(op_mask);
    uint32_t bid = 0xFFFFFFFFu;
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int walk = gid / S.Q, s = gid - walk * S.Q;
    if (walk < 7 && (flagsof(gld(S.a4 + s).x) & kFlagCustomer)) {
        const int r = gld(S.a4 + s).y, off = gld(S.roff + r), L = gld(S.roff + r + 1) - off - 1, i = s - off;
        const int n = S.n, np1 = S.np1, cap = S.cap;
        const uint32_t uQ = (uint32_t)S.Q;
        const int32_t *D = S.D;
        const bool opSwap = op_mask & 2, op2o = op_mask & 8, opOr = op_mask & 16;
        auto node = [&](int p) { return (p == 0 || p > L) ? 0 : nodeof(gld(S.a4 + off + p).x); };
        auto d = [&](int a, int b) { return gld(D + (size_t)a * np1 + b); };
        auto ref = [&](int p) { return p == 0 ? (uint32_t)(n + r) : (uint32_t)(node(p) - 1); };
        auto edge = [&](int p) { return gld(S.a4 + off + p).z; };  // position p to p + 1
        const Tw dep = TW ? tw_depot(S) : Tw{};
        auto Npos = [&](int p) { return TW ? tw_node_at(S, off + p) : Tw{}; };
        auto Fpos = [&](int p) { return TW ? tw_of(gld(S.pf4 + off + p)) : Tw{}; };
        auto Bafter = [&](int p) { return TW ? (p >= L ? dep : tw_of(gld(S.pb4 + off + p + 1))) : Tw{}; };
        auto LNpos = [&](int p) { return PD ? ld_node_at(S, off + p) : Ld{}; };
        auto LFpos = [&](int p) { return PD ? ld_of(gld(S.pl4 + off + p)) : Ld{}; };
        auto LBafter = [&](int p) { return PD ? (p >= L ? Ld{0, 0, 0} : ld_of(gld(S.ql4 + off + p + 1))) : Ld{}; };
        const int lvR = route_excess(S, r);
        const int tvR = TW ? gld(S.pb4 + off).w : 0;
        // new route: time warp tvNew, largest load peakNew (without pickups
        // an intra-route move keeps the load)
        auto rec = [&](int dD, int tvNew, int lvNew, uint32_t id) {
            gen_record(S, dD, lvNew - lvR, tvNew - tvR, lvNew == 0, tvNew == 0, id, DUMP, dd, df, bd, bid);
        };
        auto excess = [&](const Ld &x) { return PD ? max(x.lm - cap, 0) : lvR; };
        const int cI = node(i), cP = node(i - 1);
        const int eP = edge(i - 1), eI = edge(i);
        const Tw Fi1 = Fpos(i - 1);
        const Ld LFi1 = LFpos(i - 1);
        // ---- 2OPT(i, j) and SWAP(i, j), j > i
        if ((op2o || opSwap) && walk == 0) {
            Tw rev = Npos(i), mid{};
            Ld lrev = LNpos(i), lmid{};
            for (int j = i + 1; j <= L; ++j) {
                const int cJ = node(j), cJ1 = node(j + 1), ej = edge(j), ejm = edge(j - 1);
                if (TW) rev = tw_cat(Npos(j), ejm, rev);
                if (PD) lrev = ld_cat(LNpos(j), lrev);
                const int d1 = d(cP, cJ), d2 = d(cI, cJ1);
                const uint32_t lo = min(ref(i), ref(j)), hi = max(ref(i), ref(j));
                const Tw Ba = Bafter(j);
                const Ld LBa = LBafter(j);
                if (op2o) {
                    const int tv = TW ? tw_cat(tw_cat(Fi1, d1, rev), d2, Ba).v : 0;
                    const int lv = excess(ld_cat(ld_cat(LFi1, lrev), LBa));
                    rec(d1 + d2 - eP - ej, tv, lv, (12u * uQ + lo) * uQ + hi);
                }
                if (opSwap) {
                    int dS, tv = 0, lv;
                    if (j == i + 1) {
                        dS = d1 + d2 - eP - ej;
                        if (TW) tv = tw_cat(tw_cat(tw_cat(Fi1, d1, Npos(j)), ejm, Npos(i)), d2, Ba).v;
                        lv = excess(ld_cat(ld_cat(ld_cat(LFi1, LNpos(j)), LNpos(i)), LBa));
                    } else {
                        const int dA = d(cJ, node(i + 1)), dB = d(node(j - 1), cI);
                        dS = d1 + dA + dB + d2 - eP - eI - ejm - ej;
                        if (TW)
                            tv = tw_cat(tw_cat(tw_cat(tw_cat(Fi1, d1, Npos(j)), dA, mid), dB, Npos(i)), d2, Ba).v;
                        lv = excess(ld_cat(ld_cat(ld_cat(ld_cat(LFi1, LNpos(j)), lmid), LNpos(i)), LBa));
                    }
                    rec(dS, tv, lv, (5u * uQ + lo) * uQ + hi);
                }
                if (TW) mid = (j == i + 1) ? Npos(j) : tw_cat(mid, ejm, Npos(j));  // c_{i+1} .. c_j
                if (PD) lmid = (j == i + 1) ? LNpos(j) : ld_cat(lmid, LNpos(j));
            }
        }
        // ---- OR-OPT: segment c_i .. c_{i+k-1} moved right after c_j
        if (opOr && walk >= 1) {
            const int k = walk <= 3 ? walk : walk - 3;
            const bool fwd = walk <= 3;
            if (i + k - 1 <= L) {
                const int g = i + k - 1, w = i + k, cG = node(g), cW = node(w);
                const int base = d(cP, cW) - eP - edge(g);
                Tw sig{};
                Ld lsig{};
                if (TW) {
                    sig = Npos(i);
                    for (int q = 1; q < k; ++q) sig = tw_cat(sig, edge(i + q - 1), Npos(i + q));
                }
                if (PD) {
                    lsig = LNpos(i);
                    for (int q = 1; q < k; ++q) lsig = ld_cat(lsig, LNpos(i + q));
                }
                Tw mid{};
                Ld lmid{};
                for (int j = w; fwd && j <= L; ++j) {  // forward: middle c_{i+k} .. c_j
                    const int cJ = node(j), cJ1 = node(j + 1);
                    if (TW) mid = (j == w) ? Npos(j) : tw_cat(mid, edge(j - 1), Npos(j));
                    if (PD) lmid = (j == w) ? LNpos(j) : ld_cat(lmid, LNpos(j));
                    const int dVF = d(cJ, cI), dGV = d(cG, cJ1);
                    const int tv = TW ? tw_cat(tw_cat(tw_cat(Fi1, d(cP, cW), mid), dVF, sig), dGV, Bafter(j)).v : 0;
                    const int lv = excess(ld_cat(ld_cat(ld_cat(LFi1, lmid), lsig), LBafter(j)));
                    rec(base + dVF + dGV - edge(j), tv, lv, ((16u + k) * uQ + ref(i)) * uQ + ref(j));
                }
                for (int j = i - 2; !fwd && j >= 0; --j) {  // backward: middle c_{j+1} .. c_{i-1}
                    const int cJ = node(j), cJ1 = node(j + 1);
                    if (TW) mid = (j == i - 2) ? Npos(i - 1) : tw_cat(Npos(j + 1), edge(j + 1), mid);
                    if (PD) lmid = (j == i - 2) ? LNpos(i - 1) : ld_cat(LNpos(j + 1), lmid);
                    const int dVF = d(cJ, cI), dGV = d(cG, cJ1);
                    const int tv =
                        TW ? tw_cat(tw_cat(tw_cat(Fpos(j), dVF, sig), dGV, mid), d(cP, cW), Bafter(g)).v : 0;
                    const int lv = excess(ld_cat(ld_cat(ld_cat(LFpos(j), lsig), lmid), LBafter(g)));
                    rec(base + dVF + dGV - edge(j), tv, lv, ((16u + k) * uQ + ref(i)) * uQ + ref(j));
                }
            }
        }
        if ((op_mask & kMulti) && bd < 0 && bid != 0xFFFFFFFFu)  // moves inside route r
            atomicMin(S.pairkey + (size_t)r * S.R + r, pack_key(bd, bid));
    }
    block_argmin_commit(bd, bid, S.best_key, red);
}

// theta nearest neighbours of every node (distance, then node id; the node
// itself excluded), one workgroup per node: the theta-th smallest key
// (d << 14 | j) is found by bisection over the key range with block-wide
// counts, then the theta keys at or below it are collected and ranked.
// out: (n+1) x theta node ids, nearest first.  Requires theta <= n and
// theta <= kKnnMax.
constexpr int kKnnMax = 512;

__global__ __launch_bounds__(256) void k_knn(const int32_t *__restrict__ D, int np1, int theta,
                                             int32_t *__restrict__ out) {
    __shared__ unsigned long long keys[kKnnMax];
    __shared__ int cnt_w[4];
    __shared__ int nsel;
    const int i = blockIdx.x, tid = threadIdx.x;
    const int32_t *row = D + (size_t)i * np1;
    auto key = [&](int j) { return ((unsigned long long)(uint32_t)gld(row + j) << 14) | (unsigned)j; };
    unsigned long long lo = 0, hi = (1ull << 38) - 1;  // the answer is in [lo, hi]
    while (lo < hi) {
        const unsigned long long mid = lo + (hi - lo) / 2;
        int c = 0;
        for (int j = tid; j < np1; j += 256) c += (j != i && key(j) <= mid) ? 1 : 0;
        for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
        if ((tid & 63) == 0) cnt_w[tid >> 6] = c;
        __syncthreads();
        const int total = cnt_w[0] + cnt_w[1] + cnt_w[2] + cnt_w[3];
        __syncthreads();
        if (total >= theta)
            hi = mid;
        else
            lo = mid + 1;
    }
    if (tid == 0) nsel = 0;
    __syncthreads();
    for (int j = tid; j < np1; j += 256)
        if (j != i && key(j) <= lo) keys[atomicAdd(&nsel, 1)] = key(j);
    __syncthreads();
    for (int a = tid; a < theta; a += 256) {
        int rank = 0;
        for (int b = 0; b < theta; ++b) rank += keys[b] < keys[a] ? 1 : 0;
        out[(size_t)i * theta + rank] = (int32_t)(keys[a] & 0x3FFF);
    }
}

// ------------------------------------------------------ intra-route eval ---
// One wavefront per route (the route-based extraction of Section 5.3.1,
// eq. 2_opt, eq. ext_intra_relocate, eq. ext_intra_swap).  Lane i takes the
// first position i; the second position j walks the route while the
// summaries of the middle segments grow by one node per step, so every move
// costs O(1).  Positions p = 0..L+1 index the route (0 and L+1 are the
// depot).  A route that fits the wavefront's LDS region is staged there
// first (per-position data and the (L+2)^2 distance sub-block), so the walks
// never wait on global memory; a longer route reads the same values from
// the slot arrays and D directly.

constexpr int kIntraRegionBytes = 8192;  // LDS per wavefront in the intra phase

// Staged view: seven per-position arrays and the distance sub-block.
struct RouteLds {
    const int *pn, *pe, *pdep, *pz, *pe_, *pl, *ps, *dm;
    int stride;
    __device__ int node(int p) const { return pn[p]; }
    __device__ int edge(int p) const { return pe[p]; }
    __device__ int dep(int p) const { return pdep[p]; }
    __device__ int z(int p) const { return pz[p]; }
    __device__ int e(int p) const { return pe_[p]; }
    __device__ int l(int p) const { return pl[p]; }
    __device__ int s(int p) const { return ps[p]; }
    __device__ int dd(int p, int q) const { return dm[p * stride + q]; }
};

// Direct view over the slot arrays of route r.
struct RouteGlobal {
    const SolDev *S;
    int off, L, l0;
    __device__ int node(int p) const { return p <= L ? nodeof(gld(S->a4 + off + p).x) : 0; }
    __device__ int edge(int p) const { return gld(S->a4 + off + p).z; }
    __device__ int dep(int p) const { return gld(S->t4 + off + p).x; }
    __device__ int z(int p) const { return p <= L ? gld(S->t4 + off + p).w : l0; }
    __device__ int e(int p) const { return gld(S->w4 + off + p).x; }
    __device__ int l(int p) const { return gld(S->w4 + off + p).y; }
    __device__ int s(int p) const { return gld(S->w4 + off + p).z; }
    __device__ int dd(int p, int q) const { return gld(S->D + (size_t)node(p) * S->np1 + node(q)); }
};

// Moves of route r (L customers, view V) whose first position is i, for
// i = i0, i0 + di, ... <= L.  Without SPLIT: all of them; with it only walk per
// first position: 0 the 2-opt / same-route swap walk, 1..3 the forward and
// 4..6 the backward or-opt walk of segment length 1..3 (the seven walks
// cover each move exactly once).
template <bool TW, bool DUMP, bool SPLIT, class RV>
__device__ __forceinline__ void intra_moves(const SolDev &S, const RV &V, int r, int L, int i0, int di,
                                            bool capOK, uint32_t op_mask, int walk_arg,
                                            int32_t *__restrict__ dump_delta, uint8_t *__restrict__ dump_feas, int &bd,
                                            uint32_t &bid) {
    const int walk = SPLIT ? walk_arg : -1;  // a compile-time -1 without the split
    const bool opSwap = op_mask & 2, op2o = op_mask & 8, opOr = op_mask & 16;
    const int n = S.n;
    const uint32_t uQ = (uint32_t)S.Q;
    auto ref = [&](int p) { return p == 0 ? (uint32_t)(n + r) : (uint32_t)(V.node(p) - 1); };
    auto segAt = [&](int p) { return seg_node(V.e(p), V.l(p), V.s(p)); };
#pragma unroll 1
    for (int i = i0; i <= L; i += di) {
        const int eP = V.edge(i - 1);  // c(c_{i-1}, c_i)
        const int eI = V.edge(i);      // c(c_i, c_{i+1})
        const int depP = TW ? V.dep(i - 1) : 0;
        const uint32_t refI = ref(i);
        // Every step computes the deltas (and carries the segment summaries
        // along); feasibility, ids and the running minimum are evaluated
        // only where a delta can still reach the lane's best.
        // ---- 2OPT(i, j) and SWAP(i, j), j > i
        if ((op2o || opSwap) && walk <= 0) {
            Seg rev = TW ? segAt(i) : Seg{0, 0, 0, true};
            Seg mid = Seg{0, 0, 0, true};
#pragma unroll 1
            for (int j = i + 1; j <= L; ++j) {
                const int ej = V.edge(j), ejm = V.edge(j - 1);
                if (TW) rev = seg_cat(segAt(j), ejm, rev);
                const int d1 = V.dd(i - 1, j), d2 = V.dd(i, j + 1);
                const int dlt2 = d1 + d2 - eP - ej;
                int dS = dlt2, dA = 0, dB = 0;
                if (j > i + 1) {
                    dA = V.dd(j, i + 1);
                    dB = V.dd(j - 1, i);
                    dS = d1 + dA + dB + d2 - eP - eI - ejm - ej;
                }
                if (DUMP || (capOK && min(op2o ? dlt2 : kNoDelta, opSwap ? dS : kNoDelta) <= bd)) {
                    bool tw2 = true;
                    if (TW) tw2 = seg_pass(rev, depP + d1) + d2 <= V.z(j + 1);
                    bool twS = tw2;
                    if (TW && j > i + 1) {
                        const int arr0 = depP + d1;
                        bool ok = arr0 <= V.l(j);
                        const int t0 = max(arr0, V.e(j)) + V.s(j);
                        const int dM = seg_pass(mid, t0 + dA);
                        const int arrI = dM + dB;
                        ok = ok && dM < kInf && arrI <= V.l(i);
                        const int t2 = max(arrI, V.e(i)) + V.s(i);
                        twS = ok && (t2 + d2 <= V.z(j + 1));
                    }
                    const uint32_t refJ = ref(j);
                    const uint32_t lo = min(refI, refJ), hi = max(refI, refJ);
                    if (op2o) {
                        const uint32_t id = (12u * uQ + lo) * uQ + hi;
                        if (DUMP) {
                            dump_delta[id] = dlt2;
                            dump_feas[id] = (uint8_t)(capOK | (tw2 << 1));
                        }
                        if (capOK && tw2) consider(dlt2, id, bd, bid);
                    }
                    if (opSwap) {
                        const uint32_t id = (5u * uQ + lo) * uQ + hi;
                        if (DUMP) {
                            dump_delta[id] = dS;
                            dump_feas[id] = (uint8_t)(capOK | (twS << 1));
                        }
                        if (capOK && twS) consider(dS, id, bd, bid);
                    }
                }
                // middle c_{i+1} .. c_j for the next j
                if (TW) mid = (j == i + 1) ? segAt(j) : seg_cat(mid, ejm, segAt(j));
            }
        }
        if (!opOr || walk == 0) continue;
#pragma unroll 1
        for (int k = 1; k <= 3; ++k) {
            if (walk > 0 && k != (walk <= 3 ? walk : walk - 3)) continue;
            if (i + k - 1 > L) break;
            // segment c_i..c_{i+k-1} (first f = i, last g = i+k-1), followed by w = i+k
            const int g = i + k - 1, w = i + k;
            const int eG = V.edge(g);  // c(g, w)
            const int dPW = V.dd(i - 1, w);
            const int base = dPW - eP - eG;
            Seg sig = Seg{0, 0, 0, true};
            if (TW) {
                sig = segAt(i);
#pragma unroll 1
                for (int q = 1; q < k; ++q) sig = seg_cat(sig, V.edge(i + q - 1), segAt(i + q));
            }
            // ---- forward: right after c_j, j >= i+k (middle c_{i+k} .. c_j)
            Seg mid = Seg{0, 0, 0, true};
#pragma unroll 1
            for (int j = w; j <= (walk <= 3 ? L : w - 1); ++j) {
                if (TW) mid = (j == w) ? segAt(j) : seg_cat(mid, V.edge(j - 1), segAt(j));
                const int dVF = V.dd(j, i), dGV = V.dd(g, j + 1);
                const int dlt = base + dVF + dGV - V.edge(j);
                if (DUMP || (capOK && dlt <= bd)) {
                    bool tw = true;
                    if (TW) {
                        const int dm = seg_pass(mid, depP + dPW);
                        const int ds = dm >= kInf ? kInf : seg_pass(sig, dm + dVF);
                        tw = ds < kInf && ds + dGV <= V.z(j + 1);
                    }
                    const uint32_t id = ((16u + k) * uQ + refI) * uQ + ref(j);
                    if (DUMP) {
                        dump_delta[id] = dlt;
                        dump_feas[id] = (uint8_t)(capOK | (tw << 1));
                    }
                    if (capOK && tw) consider(dlt, id, bd, bid);
                }
            }
            // ---- backward: right after c_j, j <= i-2 (middle c_{j+1} .. c_{i-1})
            const int zW = TW ? V.z(w) : 0;
            mid = Seg{0, 0, 0, true};
#pragma unroll 1
            for (int j = i - 2; j >= (walk < 0 || walk >= 4 ? 0 : i - 1); --j) {
                if (TW) mid = (j == i - 2) ? segAt(i - 1) : seg_cat(segAt(j + 1), V.edge(j + 1), mid);
                const int dVF = V.dd(j, i), dGV = V.dd(g, j + 1);
                const int dlt = base + dVF + dGV - V.edge(j);
                if (DUMP || (capOK && dlt <= bd)) {
                    bool tw = true;
                    if (TW) {
                        const int ds = seg_pass(sig, V.dep(j) + dVF);
                        const int dmm = ds >= kInf ? kInf : seg_pass(mid, ds + dGV);
                        tw = dmm < kInf && dmm + dPW <= zW;
                    }
                    const uint32_t id = ((16u + k) * uQ + refI) * uQ + ref(j);
                    if (DUMP) {
                        dump_delta[id] = dlt;
                        dump_feas[id] = (uint8_t)(capOK | (tw << 1));
                    }
                    if (capOK && tw) consider(dlt, id, bd, bid);
                }
            }
        }
    }
}

// Stage route r (P = L + 2 positions) at `base` in LDS: seven per-position
// arrays followed by the P x P distance sub-block.  Returns the view.
template <bool TW>
__device__ __forceinline__ RouteLds stage_route(const SolDev &S, int off, int L, int l0, int *base) {
    const int lane = threadIdx.x & 63;
    const int P = L + 2;
    int *pn = base, *pe = pn + P, *pdep = pe + P, *pz = pdep + P, *pe_ = pz + P, *pl = pe_ + P, *ps = pl + P,
        *dm = ps + P;
    for (int p = lane; p < P; p += 64) {
        if (p <= L) {
            const int4 a = gld(S.a4 + off + p);
            pn[p] = nodeof(a.x);
            pe[p] = a.z;
            if (TW) {
                const int4 t = gld(S.t4 + off + p);
                const int4 w = gld(S.w4 + off + p);
                pdep[p] = t.x;
                pz[p] = t.w;
                pe_[p] = w.x;
                pl[p] = w.y;
                ps[p] = w.z;
            }
        } else {
            pn[p] = 0;
            pe[p] = 0;
            pz[p] = l0;
        }
    }
    return RouteLds{pn, pe, pdep, pz, pe_, pl, ps, dm, P};
}

constexpr int kIntraMaxGroup = 8;  // routes per intra-route work item
constexpr int kIntraWalks = 7;     // walks per first position (2-opt / swap, 3 forward and 3 backward or-opt)
constexpr int kGatherBatch = 8;    // distance gathers in flight per lane while staging

// The P x P distance sub-blocks of G staged routes (route k = r0 + k: P[k]
// positions, staged at word offset at[k] of the region, nodes first):
// element y of route k's block is D[node(y / P)][node(y % P)].  With cache,
// a route whose cache entry holds the same P and nodes copies its block from
// there (LDS DMA) and any other route gathers it from D and, when
// P <= kRouteBlockMaxP, rewrites its entry; without it every block is
// gathered and no entry is read or written.  Each lane keeps up to
// kGatherBatch loads in flight before it stores them, so a group costs a
// couple of memory round trips.
__device__ __forceinline__ void gather_dist_blocks(const SolDev &S, int *region, const int (&P)[kIntraMaxGroup],
                                                   const int (&at)[kIntraMaxGroup], int G, int r0, uint32_t hit,
                                                   uint32_t fill);

__device__ __forceinline__ void stage_dist_blocks(const SolDev &S, int *region, const int (&P)[kIntraMaxGroup],
                                                  const int (&at)[kIntraMaxGroup], int G, int r0, bool cache) {
    const int lane = threadIdx.x & 63;
    // which routes' cached blocks are current (bit k), and which entries to rewrite
    uint32_t hit = 0, fill = 0;
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        if (cache && k < G && P[k] <= kRouteBlockMaxP) {
            const int *c = S.rblk + (size_t)(r0 + k) * kRouteBlockWords;
            const bool same = lane >= P[k] || gld(c + kRouteBlockNodes + lane) == region[at[k] + lane];
            const bool ok = __builtin_amdgcn_readfirstlane(gld(c)) == P[k] && __builtin_amdgcn_ballot_w64(!same) == 0;
            hit |= (ok ? 1u : 0u) << k;
            fill |= (ok ? 0u : 1u) << k;
        }
    }
    // current cached blocks: straight from the cache into LDS (LDS DMA, no
    // register round trip)
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        if ((hit >> k) & 1) {
            const int *src = S.rblk + (size_t)(r0 + k) * kRouteBlockWords + kRouteBlockData;
            int *dst = region + at[k] + 7 * P[k];
            const int PP = P[k] * P[k];
            for (int c = 0; c < PP; c += 64)
                if (c + lane < PP)
                    __builtin_amdgcn_global_load_lds((global_void_ptr)(src + c + lane), (lds_void_ptr)(dst + c), 4, 0, 0);
        }
    }
    gather_dist_blocks(S, region, P, at, G, r0, hit, fill);
}

// The P x P blocks of the routes of the group not in `hit`, gathered from D
// into the region (and, for the routes in `fill`, into their cache
// entries); then, once every load issued before has landed, the nodes and
// P of the rewritten entries.
__device__ __forceinline__ void gather_dist_blocks(const SolDev &S, int *region, const int (&P)[kIntraMaxGroup],
                                                   const int (&at)[kIntraMaxGroup], int G, int r0, uint32_t hit,
                                                   uint32_t fill) {
    const int lane = threadIdx.x & 63;
    int cum[kIntraMaxGroup + 1];
    cum[0] = 0;
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) cum[k + 1] = cum[k] + (k < G ? P[k] * P[k] : 0);
    const int E = cum[kIntraMaxGroup];
    if (hit != (1u << G) - 1u) {
        for (int x0 = 0; x0 < E; x0 += 64 * kGatherBatch) {
            int val[kGatherBatch], dst[kGatherBatch], cst[kGatherBatch];
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) {
                const int x = x0 + u * 64 + lane;
                dst[u] = -1;
                cst[u] = -1;
                val[u] = 0;
                if (x < E) {
                    int k = 0, c = 0, pk = P[0], ak = at[0];
#pragma unroll
                    for (int kk = 1; kk < kIntraMaxGroup; ++kk) {
                        if (kk < G && x >= cum[kk]) {
                            k = kk;
                            c = cum[kk];
                            pk = P[kk];
                            ak = at[kk];
                        }
                    }
                    if (!((hit >> k) & 1)) {
                        const int y = x - c;
                        const int pp = y / pk, qq = y - pp * pk;
                        const int *pn = region + ak;
                        val[u] = gld(S.D + (size_t)pn[pp] * S.np1 + pn[qq]);
                        if ((fill >> k) & 1) cst[u] = (r0 + k) * kRouteBlockWords + kRouteBlockData + y;
                        dst[u] = ak + 7 * pk + y;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kGatherBatch; ++u) {
                if (dst[u] >= 0) region[dst[u]] = val[u];
                if (cst[u] >= 0) S.rblk[cst[u]] = val[u];
            }
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the gathers and the caller's LDS DMA have landed (the caller then syncs the wavefront)
    // entries rewritten above: their nodes, then P
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        if ((fill >> k) & 1) {
            int *c = S.rblk + (size_t)(r0 + k) * kRouteBlockWords;
            if (lane < P[k]) c[kRouteBlockNodes + lane] = region[at[k] + lane];
            if (lane == 0) c[0] = P[k];
        }
    }
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront evaluates every intra-route move of routes [r0, r1) of one
// solution (with SPLIT, only the moves of walk `walk`, so that seven
// wavefronts share a group) and commits the best to the solution's key.
// When all their positions fit (sum of L <= 64 first positions, staged data
// within the wavefront's LDS region), lane l takes one (route, first
// position) pair of the whole group; otherwise routes are taken one at a
// time.  Only a wavefront that evaluates every walk of its routes (no SPLIT,
// or walk 0) reads or rewrites the route distance-block cache, so no two
// wavefronts of a launch ever touch the same entry.
template <bool TW, bool DUMP, bool SPLIT = false>
__device__ __forceinline__ void intra_group(const SolDev &S, const IntraItem &item, uint32_t op_mask, int walk,
                                            int32_t *__restrict__ dump_delta, uint8_t *__restrict__ dump_feas,
                                            int *region) {
    const int lane = threadIdx.x & 63;
    int bd = initial_bound(op_mask);
    uint32_t bid = 0xFFFFFFFFu;
    const int l0 = S.has_tw ? S.node4[0].z : kTwOff;
    const int G = min(item.r1 - item.r0, kIntraMaxGroup);
    int offs[kIntraMaxGroup + 1];
    offs[0] = gld(S.roff + item.r0);
    int sumL = 0, words = 0;
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        if (k < G) {
            offs[k + 1] = gld(S.roff + item.r0 + k + 1);
            const int L = offs[k + 1] - offs[k] - 1, P = L + 2;
            sumL += L;
            words += 7 * P + P * P;
        }
    }
    if (sumL <= 64 && words <= kIntraRegionBytes / 4) {
        // stage every route of the group, then one lane per (route, first position)
        int *base = region;
#pragma unroll
        for (int k = 0; k < kIntraMaxGroup; ++k) {
            if (k < G) {
                const int L = offs[k + 1] - offs[k] - 1;
                stage_route<TW>(S, offs[k], L, l0, base);
                base += 7 * (L + 2) + (L + 2) * (L + 2);
            }
        }
        wave_lds_sync();
        {
            int Pk[kIntraMaxGroup], at[kIntraMaxGroup], w = 0;
#pragma unroll
            for (int k = 0; k < kIntraMaxGroup; ++k) {
                Pk[k] = k < G ? offs[k + 1] - offs[k] + 1 : 0;
                at[k] = w;
                w += 7 * Pk[k] + Pk[k] * Pk[k];
            }
            stage_dist_blocks(S, region, Pk, at, G, item.r0, !SPLIT || walk == 0);
        }
        wave_lds_sync();
        // lane -> (route k, first position i) and that route's staged view
        int myk = -1, myi = 0, myL = 0, myOff = 0, myBase = 0, cum = 0, words2 = 0;
#pragma unroll
        for (int k = 0; k < kIntraMaxGroup; ++k) {
            if (k < G) {
                const int L = offs[k + 1] - offs[k] - 1, P = L + 2;
                if (myk < 0 && lane < cum + L) {
                    myk = k;
                    myi = lane - cum + 1;
                    myL = L;
                    myOff = offs[k];
                    myBase = words2;
                }
                cum += L;
                words2 += 7 * P + P * P;
            }
        }
        if (myk >= 0) {
            const int P = myL + 2;
            int *b = region + myBase;
            const RouteLds V{b, b + P, b + 2 * P, b + 3 * P, b + 4 * P, b + 5 * P, b + 6 * P, b + 7 * P, P};
            const bool capOK = gld(S.b4 + myOff).z <= S.cap;
            intra_moves<TW, DUMP, SPLIT>(S, V, item.r0 + myk, myL, myi, 1 << 30, capOK, op_mask, walk, dump_delta, dump_feas,
                                  bd, bid);
        }
        wave_lds_sync();
    } else {
        for (int k = 0; k < G; ++k) {
            const int r = item.r0 + k;
            const int off = gld(S.roff + r);
            const int L = gld(S.roff + r + 1) - off - 1;
            const bool capOK = gld(S.b4 + off).z <= S.cap;
            const int P = L + 2;
            if (7 * P + P * P <= kIntraRegionBytes / 4) {
                const RouteLds V = stage_route<TW>(S, off, L, l0, region);
                wave_lds_sync();
                {
                    int Pk[kIntraMaxGroup], at[kIntraMaxGroup];
#pragma unroll
                    for (int k = 0; k < kIntraMaxGroup; ++k) {
                        Pk[k] = k == 0 ? P : 0;
                        at[k] = 0;
                    }
                    stage_dist_blocks(S, region, Pk, at, 1, r, !SPLIT || walk == 0);
                }
                wave_lds_sync();
                intra_moves<TW, DUMP, SPLIT>(S, V, r, L, lane + 1, 64, capOK, op_mask, walk, dump_delta, dump_feas, bd, bid);
                wave_lds_sync();
            } else {
                const RouteGlobal V{&S, off, L, l0};
                intra_moves<TW, DUMP, SPLIT>(S, V, r, L, lane + 1, 64, capOK, op_mask, walk, dump_delta, dump_feas, bd, bid);
            }
        }
    }
    wave_argmin(bd, bid);
    if (lane == 0 && bd < kAdmissibleBound && bid != 0xFFFFFFFFu) atomicMin(S.best_key, pack_key(bd, bid));
}

// The intra-route moves of one (i, j) cell of route r (L customers, staged
// view V, 1 <= i <= L, 0 <= j <= L): 2OPT(i, j) and SWAP(i, j) when i < j,
// and the or-opt moves of the segments of length k = 1..3 that start at c_i
// to right after c_j (j >= i + k forward, j <= i - 2 backward).  The cells of
// the grid hold every intra-route move exactly once, with the deltas,
// feasibility and ids of intra_moves; the deltas come first (every position
// clamped into the route, invalid moves masked), and the time-window
// summaries of a move are built only when its delta can still reach bd, in
// the order intra_moves builds them.
template <bool TW>
__device__ __forceinline__ void intra_cell(const SolDev &S, const RouteLds &V, int r, int L, int i, int j,
                                           bool opSwap, bool op2o, bool opOr, int &bd, uint32_t &bid) {
    const int jm = max(j - 1, 0);
    const int eP = V.edge(i - 1), eI = V.edge(i), eJ = V.edge(j), eJm = V.edge(jm);
    const int d1 = V.dd(i - 1, j), d2 = V.dd(i, j + 1);  // j + 1 <= L + 1
    const int dA = V.dd(j, i + 1), dB = V.dd(jm, i);
    const int dVF = V.dd(j, i);
    const bool up = j > i;
    const int dlt2 = d1 + d2 - eP - eJ;
    const int dS = j > i + 1 ? d1 + dA + dB + d2 - eP - eI - eJm - eJ : dlt2;
    int m = kNoDelta;
    if (up && op2o) m = min(m, dlt2);
    if (up && opSwap) m = min(m, dS);
    int dOr[3];
    bool vOr[3];
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        const int g = min(i + k - 1, L);  // last node of the segment (clamped when it does not fit)
        dOr[k - 1] = V.dd(i - 1, g + 1) - eP - V.edge(g) + dVF + V.dd(g, j + 1) - eJ;
        vOr[k - 1] = opOr && i + k - 1 <= L && (j >= i + k || j <= i - 2);
        if (vOr[k - 1]) m = min(m, dOr[k - 1]);
    }
    if (m > bd) return;  // rare late in a search: no move of the cell can reach the lane's best

    const uint32_t uQ = (uint32_t)S.Q;
    const uint32_t refI = (uint32_t)(V.node(i) - 1);
    const uint32_t refJ = j == 0 ? (uint32_t)(S.n + r) : (uint32_t)(V.node(j) - 1);
    const int depP = TW ? V.dep(i - 1) : 0;
    auto segAt = [&](int p) { return seg_node(V.e(p), V.l(p), V.s(p)); };
    if (up && min(op2o ? dlt2 : kNoDelta, opSwap ? dS : kNoDelta) <= bd) {
        bool tw2 = true, twS = true;
        if (TW) {
            // c_i .. c_j reversed
            Seg rev = segAt(i);
            for (int q = i + 1; q <= j; ++q) rev = seg_cat(segAt(q), V.edge(q - 1), rev);
            tw2 = seg_pass(rev, depP + d1) + d2 <= V.z(j + 1);
            twS = tw2;
            if (j > i + 1) {
                const int arr0 = depP + d1;
                bool ok = arr0 <= V.l(j);
                const int t0 = max(arr0, V.e(j)) + V.s(j);
                // middle c_{i+1} .. c_{j-1}
                Seg mid = segAt(i + 1);
                for (int q = i + 2; q <= j - 1; ++q) mid = seg_cat(mid, V.edge(q - 1), segAt(q));
                const int dM = seg_pass(mid, t0 + dA);
                const int arrI = dM + dB;
                ok = ok && dM < kInf && arrI <= V.l(i);
                const int t2 = max(arrI, V.e(i)) + V.s(i);
                twS = ok && (t2 + d2 <= V.z(j + 1));
            }
        }
        const uint32_t lo = min(refI, refJ), hi = max(refI, refJ);
        if (op2o && tw2) consider(dlt2, (12u * uQ + lo) * uQ + hi, bd, bid);
        if (opSwap && twS) consider(dS, (5u * uQ + lo) * uQ + hi, bd, bid);
    }
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        if (!vOr[k - 1] || dOr[k - 1] > bd) continue;
        bool tw = true;
        if (TW) {
            const int g = i + k - 1, w = i + k;
            Seg sig = segAt(i);
            for (int q = 1; q < k; ++q) sig = seg_cat(sig, V.edge(i + q - 1), segAt(i + q));
            const int dPW = V.dd(i - 1, w), dGV = V.dd(g, j + 1);
            if (j >= w) {  // forward: middle c_w .. c_j
                Seg mid = segAt(w);
                for (int q = w + 1; q <= j; ++q) mid = seg_cat(mid, V.edge(q - 1), segAt(q));
                const int dm = seg_pass(mid, depP + dPW);
                const int ds = dm >= kInf ? kInf : seg_pass(sig, dm + dVF);
                tw = ds < kInf && ds + dGV <= V.z(j + 1);
            } else {  // backward: middle c_{j+1} .. c_{i-1}
                Seg mid = segAt(i - 1);
                for (int q = i - 2; q >= j + 1; --q) mid = seg_cat(segAt(q), V.edge(q), mid);
                const int ds = seg_pass(sig, V.dep(j) + dVF);
                const int dmm = ds >= kInf ? kInf : seg_pass(mid, ds + dGV);
                tw = dmm < kInf && dmm + dPW <= V.z(w);
            }
        }
        if (tw) consider(dOr[k - 1], ((16u + k) * uQ + refI) * uQ + refJ, bd, bid);
    }
}

// A route staged in a region has fewer than 64 positions, so a row of its
// cell grid (L + 1 cells) fits the wavefront.
static_assert(7 * 64 + 64 * 64 > kIntraRegionBytes / 4, "staged route within one wavefront row");

// The moves of intra_moves (no dump, every walk) whose first position is i,
// in two walks of the second position instead of seven: forward (j = i + 1
// .. L) the 2-opt and same-route swap moves together with the forward or-opt
// moves of the three segment lengths, backward (j = i - 2 .. 0) the backward
// or-opt moves, whose middle c_{j+1} .. c_{i-1} is the same for the three
// lengths.  The walks share their reads of position j; the segment summaries
// they carry are the ones intra_moves carries (the swap's middle
// c_{i+1} .. c_{j-1} is the length-1 or-opt middle of the step before), and
// concatenation is associative, so every feasibility test is the same.
template <bool TW>
__device__ __forceinline__ void intra_moves_joint(const SolDev &S, const RouteLds &V, int r, int L, int i,
                                                  bool capOK, uint32_t op_mask, int &bd, uint32_t &bid) {
    if (!capOK) return;  // over capacity: no admissible move
    const bool opSwap = op_mask & 2, op2o = op_mask & 8, opOr = op_mask & 16;
    const uint32_t uQ = (uint32_t)S.Q;
    auto ref = [&](int p) { return p == 0 ? (uint32_t)(S.n + r) : (uint32_t)(V.node(p) - 1); };
    auto segAt = [&](int p) { return seg_node(V.e(p), V.l(p), V.s(p)); };
    const int eP = V.edge(i - 1), eI = V.edge(i);
    const int depP = TW ? V.dep(i - 1) : 0;
    const uint32_t refI = ref(i);
    // or-opt segments c_i .. c_g (g = i + k - 1), then w = i + k
    bool okK[3];
    int baseK[3], dPW[3], zW[3];
    Seg sig[3];
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        const int g = min(i + k - 1, L);
        okK[k - 1] = opOr && i + k - 1 <= L;
        dPW[k - 1] = V.dd(i - 1, g + 1);
        baseK[k - 1] = dPW[k - 1] - eP - V.edge(g);
        zW[k - 1] = TW ? V.z(g + 1) : 0;
        if (TW) sig[k - 1] = k == 1 ? segAt(i) : seg_cat(sig[k - 2], V.edge(g - 1), segAt(g));
    }
    // ---- forward: j = i + 1 .. L.  The step is written once; the first
    // three steps (where the or-opt middles start) are peeled with their
    // offset PH = j - i known at compile time, so that the main loop updates
    // every summary unconditionally.
    Seg rev = TW ? segAt(i) : Seg{0, 0, 0, true};  // c_i .. c_j reversed
    Seg m1 = Seg{0, 0, 0, true}, m2 = m1, m3 = m1;  // c_{i+k} .. c_j (k = 1, 2, 3)
    auto fwd = [&](int j, auto phc) {
        constexpr int PH = decltype(phc)::value;  // j - i, or 4 for any j >= i + 4
        const int ej = V.edge(j), ejm = V.edge(j - 1);
        Seg sj = Seg{0, 0, 0, true};
        if (TW) {
            sj = segAt(j);
            rev = seg_cat(sj, ejm, rev);
        }
        const uint32_t refJ = ref(j);
        if (op2o || opSwap) {
            const int d1 = V.dd(i - 1, j), d2 = V.dd(i, j + 1);
            const int dlt2 = d1 + d2 - eP - ej;
            int dS = dlt2, dA = 0, dB = 0;
            if (PH > 1) {
                dA = V.dd(j, i + 1);
                dB = V.dd(j - 1, i);
                dS = d1 + dA + dB + d2 - eP - eI - ejm - ej;
            }
            if (min(op2o ? dlt2 : kNoDelta, opSwap ? dS : kNoDelta) <= bd) {
                bool tw2 = true;
                if (TW) tw2 = seg_pass(rev, depP + d1) + d2 <= V.z(j + 1);
                bool twS = tw2;
                if (TW && PH > 1) {
                    const int arr0 = depP + d1;
                    bool ok = arr0 <= V.l(j);
                    const int t0 = max(arr0, V.e(j)) + V.s(j);
                    const int dM = seg_pass(m1, t0 + dA);  // m1 is c_{i+1} .. c_{j-1} here
                    const int arrI = dM + dB;
                    ok = ok && dM < kInf && arrI <= V.l(i);
                    const int t2 = max(arrI, V.e(i)) + V.s(i);
                    twS = ok && (t2 + d2 <= V.z(j + 1));
                }
                const uint32_t lo = min(refI, refJ), hi = max(refI, refJ);
                if (op2o && tw2) consider(dlt2, (12u * uQ + lo) * uQ + hi, bd, bid);
                if (opSwap && twS) consider(dS, (5u * uQ + lo) * uQ + hi, bd, bid);
            }
        }
        if (TW) {
            m1 = PH == 1 ? sj : seg_cat(m1, ejm, sj);
            if (PH >= 2) m2 = PH == 2 ? sj : seg_cat(m2, ejm, sj);
            if (PH >= 3) m3 = PH == 3 ? sj : seg_cat(m3, ejm, sj);
        }
        if (opOr) {
            const int dVF = V.dd(j, i);
#pragma unroll
            for (int k = 1; k <= 3; ++k) {
                if (!okK[k - 1] || PH < k) continue;
                const int dGV = V.dd(i + k - 1, j + 1);
                const int dlt = baseK[k - 1] + dVF + dGV - ej;
                if (dlt > bd) continue;
                bool tw = true;
                if (TW) {
                    const Seg &mid = k == 1 ? m1 : (k == 2 ? m2 : m3);
                    const int dm = seg_pass(mid, depP + dPW[k - 1]);
                    const int ds = dm >= kInf ? kInf : seg_pass(sig[k - 1], dm + dVF);
                    tw = ds < kInf && ds + dGV <= V.z(j + 1);
                }
                if (tw) consider(dlt, ((16u + k) * uQ + refI) * uQ + refJ, bd, bid);
            }
        }
    };
    if (i + 1 <= L) fwd(i + 1, std::integral_constant<int, 1>{});
    if (i + 2 <= L) fwd(i + 2, std::integral_constant<int, 2>{});
    if (i + 3 <= L) fwd(i + 3, std::integral_constant<int, 3>{});
#pragma unroll 1
    for (int j = i + 4; j <= L; ++j) fwd(j, std::integral_constant<int, 4>{});
    if (!opOr) return;
    // ---- backward: j = i - 2 .. 0, middle c_{j+1} .. c_{i-1} (the first
    // step, where the middle is c_{i-1} alone, peeled as above)
    Seg mid = Seg{0, 0, 0, true};
    auto bwd = [&](int j, auto firstc) {
        if (TW) mid = decltype(firstc)::value ? segAt(i - 1) : seg_cat(segAt(j + 1), V.edge(j + 1), mid);
        const int dVF = V.dd(j, i), ej = V.edge(j);
        const int depJ = TW ? V.dep(j) : 0;
        const uint32_t refJ = ref(j);
#pragma unroll
        for (int k = 1; k <= 3; ++k) {
            if (!okK[k - 1]) continue;
            const int dGV = V.dd(i + k - 1, j + 1);
            const int dlt = baseK[k - 1] + dVF + dGV - ej;
            if (dlt > bd) continue;
            bool tw = true;
            if (TW) {
                const int ds = seg_pass(sig[k - 1], depJ + dVF);
                const int dmm = ds >= kInf ? kInf : seg_pass(mid, ds + dGV);
                tw = dmm < kInf && dmm + dPW[k - 1] <= zW[k - 1];
            }
            if (tw) consider(dlt, ((16u + k) * uQ + refI) * uQ + refJ, bd, bid);
        }
    };
    if (i - 2 >= 0) bwd(i - 2, std::true_type{});
#pragma unroll 1
    for (int j = i - 3; j >= 0; --j) bwd(j, std::false_type{});
}

// bits [lo, hi) of a 64-bit word (lo and hi clamped to [0, 64])
__device__ __forceinline__ unsigned long long bit_range(int lo, int hi) {
    lo = max(lo, 0);
    hi = min(hi, 64);
    if (lo >= hi) return 0ull;
    const unsigned long long top = hi >= 64 ? ~0ull : ((1ull << hi) - 1ull);
    return top & ~((1ull << lo) - 1ull);
}

// intra_group for the batched local-search launch (no dump, every walk of
// every route of the group in one wavefront).  A group that fits the region
// is staged with every load issued at once: the routes' per-position
// attributes and loads, their cache entries' P and nodes, and the cached
// distance blocks themselves (LDS DMA, before it is known whether they are
// current; a route whose entry turns out stale is then gathered from D over
// it).  With current entries the staging thus costs one memory round trip
// after the route offsets instead of several per route.  The moves of a
// VRPTW route are then taken by one lane per first position (the joint
// walks of intra_moves_joint), those of a CVRP route one (i, j) cell per
// lane (intra_cell), the cells laid over the wavefront as rows of L + 1
// lanes.  Any other group goes to intra_group.
template <bool TW>
__device__ __forceinline__ void intra_group_flat(const SolDev &S, const IntraItem &item, uint32_t op_mask,
                                                 int *region) {
    const int lane = threadIdx.x & 63;
    const int G = min(item.r1 - item.r0, kIntraMaxGroup);
    int offs[kIntraMaxGroup + 1];
#pragma unroll
    for (int k = 0; k <= kIntraMaxGroup; ++k) offs[k] = sld1(S.roff + min(item.r0 + k, item.r1));
    int P[kIntraMaxGroup], at[kIntraMaxGroup], cumP[kIntraMaxGroup + 1];
    int sumL = 0, words = 0;
    cumP[0] = 0;
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        P[k] = k < G ? offs[k + 1] - offs[k] + 1 : 0;
        at[k] = words;
        if (k < G) {
            sumL += P[k] - 2;
            words += 7 * P[k] + P[k] * P[k];
        }
        cumP[k + 1] = cumP[k] + P[k];
    }
    if (!(sumL <= 64 && words <= kIntraRegionBytes / 4)) {
        intra_group<TW, false>(S, item, op_mask, -1, nullptr, nullptr, region);
        return;
    }
    const int l0 = TW ? S.node4[0].z : kTwOff;
    const int NP = cumP[kIntraMaxGroup];  // positions of the group, <= 64 + 2 * kIntraMaxGroup
    // flat position f = lane + 64 u -> route k, position p: every load first
    int4 va[2], vt[2], vw[2];
    int cn[2], hd[2], ld[2], fk[2], fp[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int f = lane + 64 * u;
        int k = 0, pk = P[0], ok = offs[0], ck = 0;
#pragma unroll
        for (int kk = 1; kk < kIntraMaxGroup; ++kk) {
            if (kk < G && f >= cumP[kk]) {
                k = kk;
                pk = P[kk];
                ok = offs[kk];
                ck = cumP[kk];
            }
        }
        const int p = f - ck;
        fk[u] = f < NP ? k : -1;
        fp[u] = p;
        va[u] = vt[u] = vw[u] = make_int4(0, 0, 0, 0);
        cn[u] = hd[u] = -2;
        ld[u] = 0;
        if (f < NP) {
            const int *c = S.rblk + (size_t)(item.r0 + k) * kRouteBlockWords;
            if (p <= pk - 2) {
                va[u] = gld(S.a4 + ok + p);
                if (TW) {
                    vt[u] = gld(S.t4 + ok + p);
                    vw[u] = gld(S.w4 + ok + p);
                }
            }
            if (pk <= kRouteBlockMaxP) cn[u] = gld(c + kRouteBlockNodes + p);
            if (p == 0) {
                hd[u] = gld(c);
                ld[u] = gld(S.b4 + ok).z;
            }
        }
    }
    // the cached blocks, copied whether or not they are current
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        if (k < G && P[k] <= kRouteBlockMaxP) {
            const int *src = S.rblk + (size_t)(item.r0 + k) * kRouteBlockWords + kRouteBlockData;
            int *dst = region + at[k] + 7 * P[k];
            const int PP = P[k] * P[k];
            for (int c = 0; c < PP; c += 64)
                if (c + lane < PP)
                    __builtin_amdgcn_global_load_lds((global_void_ptr)(src + c + lane), (lds_void_ptr)(dst + c), 4, 0, 0);
        }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the DMA has landed before any of it is overwritten or read
    // per-position arrays (as stage_route), and per route: cache entry
    // current, route load within capacity (bits at the route's first
    // flat position)
    unsigned long long mism[2], hdok[2], capok[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        bool bad = false, hok = false, cok = false;
        if (fk[u] >= 0) {
            int k = 0;
#pragma unroll
            for (int kk = 1; kk < kIntraMaxGroup; ++kk) k = fk[u] == kk ? kk : k;
            int pk = P[0], ak = at[0];
#pragma unroll
            for (int kk = 1; kk < kIntraMaxGroup; ++kk) {
                if (k == kk) {
                    pk = P[kk];
                    ak = at[kk];
                }
            }
            const int p = fp[u];
            int *b = region + ak;
            int node;
            if (p <= pk - 2) {
                node = nodeof(va[u].x);
                b[p] = node;
                b[pk + p] = va[u].z;
                if (TW) {
                    b[2 * pk + p] = vt[u].x;
                    b[3 * pk + p] = vt[u].w;
                    b[4 * pk + p] = vw[u].x;
                    b[5 * pk + p] = vw[u].y;
                    b[6 * pk + p] = vw[u].z;
                }
            } else {
                node = 0;
                b[p] = 0;
                b[pk + p] = 0;
                b[3 * pk + p] = l0;
            }
            bad = pk <= kRouteBlockMaxP && cn[u] != node;
            hok = p == 0 && hd[u] == pk;
            cok = p == 0 && ld[u] <= S.cap;
        }
        mism[u] = __builtin_amdgcn_ballot_w64(bad);
        hdok[u] = __builtin_amdgcn_ballot_w64(hok);
        capok[u] = __builtin_amdgcn_ballot_w64(cok);
    }
    uint32_t hit = 0, fill = 0, capOK = 0;
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        if (k < G) {
            const int c0 = cumP[k], c1 = cumP[k + 1];
            const bool stale = ((mism[0] & bit_range(c0, c1)) | (mism[1] & bit_range(c0 - 64, c1 - 64))) != 0ull;
            const bool hdr = ((c0 < 64 ? hdok[0] >> c0 : hdok[1] >> (c0 - 64)) & 1ull) != 0ull;
            const bool cap = ((c0 < 64 ? capok[0] >> c0 : capok[1] >> (c0 - 64)) & 1ull) != 0ull;
            if (P[k] <= kRouteBlockMaxP) {
                const bool cur = hdr && !stale;
                hit |= (cur ? 1u : 0u) << k;
                fill |= (cur ? 0u : 1u) << k;
            }
            capOK |= (cap ? 1u : 0u) << k;
        }
    }
    wave_lds_sync();  // the nodes are in place for the gathers
    gather_dist_blocks(S, region, P, at, G, item.r0, hit, fill);
    wave_lds_sync();

    int bd = initial_bound(op_mask);
    uint32_t bid = 0xFFFFFFFFu;
    if (TW) {
        // Time windows: most moves with a negative delta break a window, and
        // the walks carry the segment summaries from one move to the next,
        // so their check is O(1) where a cell's would be O(L): one lane per
        // (route, first position), as intra_group.
        int myk = -1, myi = 0, cum = 0;
#pragma unroll
        for (int k = 0; k < kIntraMaxGroup; ++k) {
            const int L = P[k] - 2;
            if (k < G && myk < 0 && lane < cum + L) {
                myk = k;
                myi = lane - cum + 1;
            }
            cum += k < G ? L : 0;
        }
        if (myk >= 0) {
            int pk = P[0], ak = at[0];
#pragma unroll
            for (int kk = 1; kk < kIntraMaxGroup; ++kk) {
                if (myk == kk) {
                    pk = P[kk];
                    ak = at[kk];
                }
            }
            int *b = region + ak;
            const RouteLds V{b, b + pk, b + 2 * pk, b + 3 * pk, b + 4 * pk, b + 5 * pk, b + 6 * pk, b + 7 * pk, pk};
            intra_moves_joint<TW>(S, V, item.r0 + myk, pk - 2, myi, (capOK >> myk) & 1, op_mask, bd, bid);
        }
        wave_lds_sync();
        wave_argmin(bd, bid);
        if (lane == 0 && bd < kAdmissibleBound && bid != 0xFFFFFFFFu) atomicMin(S.best_key, pack_key(bd, bid));
        return;
    }
    const bool opSwap = op_mask & 2, op2o = op_mask & 8, opOr = op_mask & 16;
    // route k's P and region offset sit in lane k (read back uniformly below,
    // so that the route loop is not unrolled)
    int laneP = 0, laneAt = 0;
#pragma unroll
    for (int k = 0; k < kIntraMaxGroup; ++k) {
        laneP = lane == k ? P[k] : laneP;
        laneAt = lane == k ? at[k] : laneAt;
    }
#pragma unroll 1
    for (int k = 0; k < G; ++k) {
        const int Pk = __builtin_amdgcn_readlane(laneP, k), L = Pk - 2;
        if (L < 1 || !((capOK >> k) & 1)) continue;  // over capacity: no admissible move
        int *b = region + __builtin_amdgcn_readlane(laneAt, k);
        const RouteLds V{b, b + Pk, b + 2 * Pk, b + 3 * Pk, b + 4 * Pk, b + 5 * Pk, b + 6 * Pk, b + 7 * Pk, Pk};
        // cells per row, rows per pass (W <= 62, see above)
        const int W = L + 1, rpi = 64 / W;
        const int di = lane / W, j = lane - di * W;
#pragma unroll 1
        for (int i0 = 1; i0 <= L; i0 += rpi) {
            const int i = i0 + di;
            if (di < rpi && i <= L) intra_cell<TW>(S, V, item.r0 + k, L, i, j, opSwap, op2o, opOr, bd, bid);
        }
    }
    wave_lds_sync();  // the region is free for the next group
    wave_argmin(bd, bid);
    if (lane == 0 && bd < kAdmissibleBound && bid != 0xFFFFFFFFu) atomicMin(S.best_key, pack_key(bd, bid));
}

template <bool TW, bool DUMP>
__global__ __launch_bounds__(kInterThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_intra(
    const SolDev *__restrict__ sols, const IntraItem *__restrict__ items, int nitems, uint32_t op_mask,
    int32_t *__restrict__ dump_delta, uint8_t *__restrict__ dump_feas) {
    extern __shared__ int4 smem4[];
    const int wave = threadIdx.x >> 6;
    int *region = (int *)smem4 + wave * (kIntraRegionBytes / 4);
    if ((int)gridDim.x >= nitems) {  // one workgroup per group: wavefront w < 7 takes walk w
        if ((int)blockIdx.x >= nitems) return;
        const IntraItem item = items[blockIdx.x];
        const SolDev &S = sols[item.sol];
        if (wave < kIntraWalks && !skip_solution(S, op_mask))
            intra_group<TW, DUMP, true>(S, item, op_mask, wave, dump_delta, dump_feas, region);
        return;
    }
    for (int itx = wave * gridDim.x + blockIdx.x; itx < nitems; itx += gridDim.x * kInterWaves) {
        const IntraItem item = items[itx];
        const SolDev &S = sols[item.sol];
        if (skip_solution(S, op_mask)) continue;
        intra_group<TW, DUMP>(S, item, op_mask, -1, dump_delta, dump_feas, region);
    }
}

// Single-solution form with both operator kinds: workgroups below nbintra
// take the intra-route groups (as k_eval_intra; with one workgroup per group
// every walk has a compute unit to itself), the others the inter-route items
// (as k_eval_inter), so both run at once in one launch and the long
// intra-route chains are dispatched first.  The dynamic LDS is the larger of
// the two needs.
template <bool TW, bool DUMP>
__global__ __launch_bounds__(kInterThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_solution(
    const SolDev *__restrict__ sols, const InterItem *__restrict__ items, int nitems,
    const IntraItem *__restrict__ intra, int nintra, int nbintra, uint32_t op_mask, int32_t *__restrict__ dump_delta,
    uint8_t *__restrict__ dump_feas) {
    extern __shared__ int4 smem4[];
    __shared__ unsigned long long red[kInterWaves];
    __shared__ int thr_sh;
    if ((int)blockIdx.x >= nbintra) {
        const int ninter = gridDim.x - nbintra;
        for (int it = blockIdx.x - nbintra; it < nitems; it += ninter) {
            const InterItem item = items[it];
            const SolDev &S = sols[item.sol];
            if (skip_solution(S, op_mask)) continue;
            if (S.D16)
                inter_item<TW, DUMP, true>(S, item, op_mask, dump_delta, dump_feas, smem4, red, &thr_sh);
            else
                inter_item<TW, DUMP, false>(S, item, op_mask, dump_delta, dump_feas, smem4, red, &thr_sh);
        }
    } else {
        const int wave = threadIdx.x >> 6, b = blockIdx.x;
        int *region = (int *)smem4 + wave * (kIntraRegionBytes / 4);
        if (nbintra >= nintra) {  // one workgroup per group: wavefront w < 7 takes walk w
            if (b >= nintra) return;
            const IntraItem item = intra[b];
            const SolDev &S = sols[item.sol];
            if (wave < kIntraWalks && !skip_solution(S, op_mask))
                intra_group<TW, DUMP, true>(S, item, op_mask, wave, dump_delta, dump_feas, region);
        } else {
            for (int itx = wave * nbintra + b; itx < nintra; itx += nbintra * kInterWaves) {
                const IntraItem item = intra[itx];
                const SolDev &S = sols[item.sol];
                if (skip_solution(S, op_mask)) continue;
                intra_group<TW, DUMP>(S, item, op_mask, -1, dump_delta, dump_feas, region);
            }
        }
    }
}

// Granular mode with both operator kinds in one launch (as k_eval_solution):
// workgroups below nintra take the intra-route groups (one per group, seven
// wavefronts with one walk each), the others kInterThreads granular work
// items each.
template <bool TW, bool DUMP>
__global__ __launch_bounds__(kInterThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_gran_fused(
    const SolDev *__restrict__ sols, const int32_t *__restrict__ gsrc, const int32_t *__restrict__ gadj, int gcc,
    int gdep, const IntraItem *__restrict__ intra, int nintra, uint32_t op_mask, int32_t *__restrict__ dump_delta,
    uint8_t *__restrict__ dump_feas) {
    extern __shared__ int4 smem4[];
    __shared__ unsigned long long red[kInterWaves];
    __shared__ long long cnt_sh;
    const SolDev &S = sols[0];
    if (skip_solution(S, op_mask)) return;  // uniform for the grid
    if ((int)blockIdx.x < nintra) {
        const int wave = threadIdx.x >> 6;
        int *region = (int *)smem4 + wave * (kIntraRegionBytes / 4);
        if (wave < kIntraWalks)
            intra_group<TW, DUMP, true>(S, intra[blockIdx.x], op_mask, wave, dump_delta, dump_feas, region);
        return;
    }
    gran_block<TW, DUMP>(S, gsrc, gadj, gcc, gdep, ((int)blockIdx.x - nintra) * blockDim.x + threadIdx.x, op_mask,
                         dump_delta, dump_feas, red, &cnt_sh);
}

// Batched form: persistent launches evaluate every solution of the batch.
// PH bit 1: intra-route groups (one wavefront per group of routes); PH bit 0:
// inter-route items (whole workgroup per item, largest first).  PH = 3 runs
// both phases in one launch, the latency-bound intra-route walks first so
// that they overlap other workgroups' inter-route work and the small
// inter-route items fill the tail; PH = 1 and PH = 2 are the two halves as
// separate launches.
// Solutions of both problem types and both distance widths share a launch;
// each item takes the path of its own solution.  Workgroup b is dispatched
// to XCD x = b mod nx and works on the items of the solutions placed there:
// its wavefronts take the intra-route groups j * 8 + wave, then every
// (G' * 8)-th after it, of the XCD's group list (j = b / nx, G' =
// gridDim.x / nx); then the workgroup pulls the XCD's inter-route items
// items[woff[x] ..  woff[x + 1]) (largest first) from a queue, counter
// qctr[2x] (items taken), so that whichever workgroup is free takes the
// next one.  Each workgroup's next pull is issued while it evaluates its
// current item.  A workgroup that finds the queue empty counts itself in
// qctr[2x + 1]; the last of the XCD's workgroups to do so puts both
// counters back to zero, ready for the next launch.
template <int PH>
__global__ __launch_bounds__(kInterThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_eval_batch(
    const SolDev *__restrict__ sols, const InterItem *__restrict__ items, const int *__restrict__ woff,
    uint32_t *__restrict__ qctr, const IntraItem *__restrict__ intra, const int *__restrict__ ixoff, int nx,
    uint32_t op_mask) {
    extern __shared__ int4 smem4[];
    __shared__ unsigned long long red[kInterWaves];
    __shared__ int thr_sh;
    const int wave = threadIdx.x >> 6;
    const int x = blockIdx.x % nx, j = blockIdx.x / nx, step = gridDim.x / nx;
    if ((PH & 2) && (op_mask & (2 | 8 | 16))) {
        int *region = (int *)smem4 + wave * (kIntraRegionBytes / 4);
        const int end = ixoff[x + 1];
        for (int it = ixoff[x] + j * kInterWaves + wave; it < end; it += step * kInterWaves) {
            const IntraItem item = intra[it];
            const SolDev &S = sols[item.sol];
            if (skip_solution(S, op_mask)) continue;
            if (S.has_tw)
                intra_group_flat<true>(S, item, op_mask, region);
            else
                intra_group_flat<false>(S, item, op_mask, region);
        }
    }
    __syncthreads();  // the intra-route regions and the inter-route rows share LDS
    if ((PH & 1) && (op_mask & 7)) {
        __shared__ int q_sh[2];  // pulled item index, alternate slots by iteration
        const int first = woff[x], cnt = woff[x + 1] - first;
        uint32_t *taken = qctr + 2 * x, *finished = taken + 1;
        if (threadIdx.x == 0) q_sh[0] = (int)atomicAdd(taken, 1u);
        __syncthreads();
        for (int round = 0;; ++round) {
            const int k = q_sh[round & 1];
            if (k >= cnt) break;  // the same for the whole workgroup
            int next = 0;
            if (threadIdx.x == 0) next = (int)atomicAdd(taken, 1u);  // lands while this item is evaluated
            const InterItem item = items[first + k];
            const SolDev &S = sols[item.sol];
            if (skip_solution(S, op_mask)) {
                if (threadIdx.x == 0) q_sh[(round + 1) & 1] = next;
                __syncthreads();
                continue;
            }
            constexpr bool CNT = (PH & 4) != 0;
            if (S.has_tw) {
                if (S.D16)
                    inter_item<true, false, true, CNT>(S, item, op_mask, nullptr, nullptr, smem4, red, &thr_sh);
                else
                    inter_item<true, false, false, CNT>(S, item, op_mask, nullptr, nullptr, smem4, red, &thr_sh);
            } else {
                if (S.D16)
                    inter_item<false, false, true, CNT>(S, item, op_mask, nullptr, nullptr, smem4, red, &thr_sh);
                else
                    inter_item<false, false, false, CNT>(S, item, op_mask, nullptr, nullptr, smem4, red, &thr_sh);
            }
            // slot (round + 1) & 1 was last read in the previous round, before
            // that round's closing barrier
            if (threadIdx.x == 0) q_sh[(round + 1) & 1] = next;
            __syncthreads();
        }
        if (threadIdx.x == 0 && atomicAdd(finished, 1u) == gridDim.x / nx - 1) {
            // every workgroup of the XCD has made its last pull
            atomicExch(taken, 0u);
            atomicExch(finished, 0u);
        }
    }
}

// ------------------------------------------------- finalize / apply / LS ---

enum { kModeRecord = 0, kModeLS = 1, kModeApplyRec = 2 };

struct MoveInfo {
    int op, k, a, b, ra, rb, pa, pb, La, Lb, nLa, nLb, valid, delta;
    uint32_t id;
};

__device__ __forceinline__ int old_node(const SolDev &S, int r, int p) {
    return p == 0 ? 0 : nodeof(S.a4[S.roff[r] + p].x);
}

// Node at new position p of a touched route r (Section 4.1 operators).
__device__ __forceinline__ int new_node(const SolDev &S, const MoveInfo &m, int r, int p) {
    if (p == 0) return 0;
    switch (m.op) {
    case 0:
        if (r == m.ra) return p < m.pa ? old_node(S, r, p) : old_node(S, r, p + 1);
        if (p <= m.pb) return old_node(S, r, p);
        if (p == m.pb + 1) return m.a + 1;
        return old_node(S, r, p - 1);
    case 1:
        if (r == m.ra && p == m.pa) return m.b + 1;
        if (r == m.rb && p == m.pb) return m.a + 1;
        return old_node(S, r, p);
    case 2:
        if (r == m.ra) return p <= m.pa ? old_node(S, r, p) : old_node(S, m.rb, m.pb + p - m.pa);
        return p <= m.pb ? old_node(S, r, p) : old_node(S, m.ra, m.pa + p - m.pb);
    case 3: {
        const int i = min(m.pa, m.pb), j = max(m.pa, m.pb);
        return (p >= i && p <= j) ? old_node(S, r, i + j - p) : old_node(S, r, p);
    }
    case 5:
    case 6: {  // the k-segment at (ra, pa) moves right after position pb of rb, kept or reversed
        const int k = m.k;
        if (r == m.ra) return p < m.pa ? old_node(S, r, p) : old_node(S, r, p + k);
        if (p <= m.pb) return old_node(S, r, p);
        if (p > m.pb + k) return old_node(S, r, p - k);
        const int q = p - m.pb - 1;
        return old_node(S, m.ra, m.pa + (m.op == 5 ? q : k - 1 - q));
    }
    case 7:
    case 8:
    case 9: {  // segments (ra, pa, ka) and (rb, pb, kb) exchange places
        const int ka = m.op - 6, kb = m.k;
        if (r == m.ra) {
            if (p < m.pa) return old_node(S, r, p);
            if (p < m.pa + kb) return old_node(S, m.rb, m.pb + p - m.pa);
            return old_node(S, r, p - kb + ka);
        }
        if (p < m.pb) return old_node(S, r, p);
        if (p < m.pb + ka) return old_node(S, m.ra, m.pa + p - m.pb);
        return old_node(S, r, p - ka + kb);
    }
    default: {
        const int i = m.pa, j = m.pb, k = m.k;
        if (j > i) {  // forward
            if (p < i || p > j) return old_node(S, r, p);
            if (p <= j - k) return old_node(S, r, p + k);
            return old_node(S, r, i + p - (j - k + 1));
        }
        if (p <= j || p >= i + k) return old_node(S, r, p);
        if (p <= j + k) return old_node(S, r, i + p - j - 1);
        return old_node(S, r, p - k);
    }
    }
}

__device__ __forceinline__ void decode_move(const SolDev &S, uint32_t id, MoveInfo &m) {
    const uint32_t Q = (uint32_t)S.Q, qq = Q * Q;
    const uint32_t opk = id / qq, rem = id % qq;
    m.id = id;
    m.op = (int)(opk >> 2);
    m.k = (int)(opk & 3);
    m.a = (int)(rem / Q);
    m.b = (int)(rem % Q);
    m.valid = 0;
    if (m.op > 9) return;
    const int sa = S.ref2slot[m.a], sb = S.ref2slot[m.b];
    m.ra = S.a4[sa].y;
    m.rb = S.a4[sb].y;
    m.pa = sa - S.roff[m.ra];
    m.pb = sb - S.roff[m.rb];
    m.La = S.roff[m.ra + 1] - S.roff[m.ra] - 1;
    m.Lb = S.roff[m.rb + 1] - S.roff[m.rb] - 1;
    const int n = S.n;
    const bool aC = m.a < n, bC = m.b < n;
    bool ok = false;
    m.nLa = m.La;
    m.nLb = m.Lb;
    switch (m.op) {
    case 0:
        ok = m.k == 1 && aC && m.ra != m.rb;
        m.nLa = m.La - 1;
        m.nLb = m.Lb + 1;
        break;
    case 1: ok = m.k == 1 && m.a < m.b && bC; break;
    case 2:
        ok = m.k == 0 && m.a < m.b && m.ra != m.rb;
        m.nLa = m.pa + m.Lb - m.pb;
        m.nLb = m.pb + m.La - m.pa;
        break;
    case 3: ok = m.k == 0 && m.a < m.b && bC && m.ra == m.rb; break;
    case 4:
        ok = m.k >= 1 && m.k <= 3 && aC && m.ra == m.rb && m.pa + m.k - 1 <= m.La &&
             !(m.pb >= m.pa - 1 && m.pb <= m.pa + m.k - 1);
        break;
    case 5:
    case 6:
        ok = m.k >= 2 && m.k <= 3 && aC && m.ra != m.rb && m.pa + m.k - 1 <= m.La;
        m.nLa = m.La - m.k;
        m.nLb = m.Lb + m.k;
        break;
    default: {  // 7..9: cross-exchange of (a, op - 6) and (b, k)
        const int ka = m.op - 6, kb = m.k;
        ok = kb >= 1 && kb <= 3 && m.a < m.b && bC && m.ra != m.rb && m.pa + ka - 1 <= m.La &&
             m.pb + kb - 1 <= m.Lb && !(ka == 1 && kb == 1);
        m.nLa = m.La - ka + kb;
        m.nLb = m.Lb - kb + ka;
        break;
    }
    }
    m.valid = ok;
}

// Apply m (valid).  All threads of the block participate.  Every slot
// attribute is route-local, so only the touched routes are rebuilt; the
// routes strictly between two touched routes of different lengths move as a
// block by the first one's length change (a plain copy of their records).
__device__ __forceinline__ void apply_move_block(const SolDev &S, const MoveInfo &m, ApplyShared &sh) {
    const int R = S.R, T = blockDim.x, tid = threadIdx.x;
    const bool inter = m.ra != m.rb;
    const int dA = m.nLa - m.La, dB = inter ? m.nLb - m.Lb : 0;
    auto shift = [&](int r) { return (r > m.ra ? dA : 0) + (inter && r > m.rb ? dB : 0); };
    // 1. new offsets, and the touched routes' nodes (read from the old layout)
    for (int r = tid; r <= R; r += T) S.roff_alt[r] = S.roff[r] + shift(r);
    const int baseA = S.roff[m.ra] + shift(m.ra);
    for (int p = tid; p <= m.nLa; p += T) S.nr_alt[baseA + p] = make_int2(new_node(S, m, m.ra, p), m.ra);
    int baseB = 0;
    if (inter) {
        baseB = S.roff[m.rb] + shift(m.rb);
        for (int p = tid; p <= m.nLb; p += T) S.nr_alt[baseB + p] = make_int2(new_node(S, m, m.rb, p), m.rb);
    }
    __threadfence_block();
    __syncthreads();
    // 2. routes strictly between the touched ones move by d; rounds of T
    //    slots, each read completely before it is written, taken in the
    //    direction of the move so no round overwrites a later one's source
    if (inter) {
        const int r1 = min(m.ra, m.rb), r2 = max(m.ra, m.rb);
        const int d = r1 == m.ra ? dA : dB;
        const int lo = S.roff[r1 + 1], hi = S.roff[r2];  // old slots of the routes between
        if (d != 0 && hi > lo) {
            const int rounds = (hi - lo + T - 1) / T;
            for (int k = 0; k < rounds; ++k) {
                const int rk = d < 0 ? k : rounds - 1 - k;
                const int src = lo + rk * T + tid;
                const bool on = src < hi;
                int4 a = make_int4(0, 0, 0, 0), b = a, t = a, w = a, pf = a, pb = a, pl = a, ql = a;
                int pd = 0;
                if (on) {
                    a = S.a4[src];
                    b = S.b4[src];
                    t = S.t4[src];
                    w = S.w4[src];
                    pd = S.pdist[src];
                    if (S.pen || S.pd || S.gen) {
                        pf = S.pf4[src];
                        pb = S.pb4[src];
                        pl = S.pl4[src];
                        ql = S.ql4[src];
                    }
                }
                __syncthreads();
                if (on) {
                    const int dst = src + d;
                    S.a4[dst] = a;
                    S.b4[dst] = b;
                    S.t4[dst] = t;
                    S.w4[dst] = w;
                    S.pdist[dst] = pd;
                    if (S.pen || S.pd || S.gen) {
                        S.pf4[dst] = pf;
                        S.pb4[dst] = pb;
                        S.pl4[dst] = pl;
                        S.ql4[dst] = ql;
                    }
                    const int node = nodeof(a.x);
                    S.ref2slot[(flagsof(a.x) & kFlagCustomer) ? node - 1 : S.n + a.y] = dst;
                }
                __threadfence_block();
                __syncthreads();
            }
        }
    }
    for (int r = tid; r <= R; r += T) S.roff[r] = S.roff_alt[r];
    __threadfence_block();
    __syncthreads();
    // 3. rebuild the touched routes in place: one wavefront each when they
    //    fit one (the usual case), else the block scans
    if (m.nLa < 64 && (!inter || m.nLb < 64)) {
        const int wave = threadIdx.x >> 6;
        if (wave == 0) rebuild_route_wave(S, S.nr_alt, m.ra, baseA, m.nLa);
        if (wave == 1 && inter) rebuild_route_wave(S, S.nr_alt, m.rb, baseB, m.nLb);
        __threadfence_block();
        __syncthreads();
        solution_totals(S, S.roff_alt, sh);
    } else {
        rebuild_range(S, S.nr_alt, S.roff_alt, baseA, baseA + m.nLa + 1, false, sh);
        if (inter) rebuild_range(S, S.nr_alt, S.roff_alt, baseB, baseB + m.nLb + 1, false, sh);
    }
    if (S.pen || S.pd || S.gen) {  // summaries of the touched routes, then the totals
        __threadfence_block();
        __syncthreads();
        if (threadIdx.x == 0) gen_route(S, m.ra);
        if (threadIdx.x == 64 && inter) gen_route(S, m.rb);
        __threadfence_block();
        __syncthreads();
        pen_totals(S, sh);
    }
}

// Local-search accounting of one evaluation (thread 0): |N(S)| of the
// enabled operators (granular: the inter-route moves as counted; variants:
// as counted) into acc[kAccMoves], and with kCountFull the slot pairs the
// screens visited.
__device__ __forceinline__ void ls_count_moves(const SolDev &S, uint32_t op_mask) {
    long long m = 0;
    if (op_mask & 0xE0u) m += S.acc[kAccExtMoves];  // operator variants, as counted
    if (op_mask & kGranular) {  // inter-route moves as counted; intra-route ones complete
        m = S.acc[kAccGranInter];
        if (op_mask & 2) m += S.acc[kAccCnt0 + 3];  // same-route swaps: L(L-1)/2 per route, as 2-opt
        if (op_mask & 8) m += S.acc[kAccCnt0 + 3];
        if (op_mask & 16) m += S.acc[kAccCnt0 + 4];
    } else {
        for (int op = 0; op < 5; ++op)
            if (op_mask >> op & 1) m += S.acc[kAccCnt0 + op];
    }
    S.acc[kAccMoves] += m;
    if ((op_mask & kCountFull) && (op_mask & 7))
        S.acc[kAccScreenPairs] += S.acc[kAccCnt0 + 2];  // = slot pairs of different routes
}

// One block per solution.  kModeRecord: publish the best move (status 1 if
// none) and reset the key.  kModeLS: also apply it when its delta is negative
// and the step cap allows, else mark the solution converged.  kModeApplyRec:
// apply the move record the host wrote into S.rec.
__device__ __forceinline__ void finalize_block(const SolDev &S, int mode, uint32_t op_mask) {
    __shared__ ApplyShared sh;
    __shared__ MoveInfo mi;
    __shared__ int act;
    if (threadIdx.x == 0) {
        act = 0;
        if (mode == kModeApplyRec) {
            decode_move(S, (uint32_t)S.rec[6], mi);
            mi.delta = S.rec[4];
            act = mi.valid;
            S.state[kStStatus] = mi.valid ? 0 : -1;
        } else if (!(mode == kModeLS && S.state[kStDone])) {
            const unsigned long long key = *S.best_key;
            *S.best_key = ~0ull;
            if (mode == kModeLS) ls_count_moves(S, op_mask);
            S.acc[kAccGranInter] = 0;
            S.acc[kAccExtMoves] = 0;
            if (key == ~0ull) {
                for (int q = 0; q < 8; ++q) S.rec[q] = 0;
                S.rec[7] = S.state[kStVersion];
                S.state[kStStatus] = 1;
                if (mode == kModeLS) S.state[kStDone] = 1;
            } else {
                const uint32_t id = (uint32_t)(key & 0xFFFFFFFFu);
                const int delta = (int)((uint32_t)(key >> 32) ^ 0x80000000u);
                decode_move(S, id, mi);
                mi.delta = delta;
                S.rec[0] = mi.op;
                S.rec[1] = mi.k;
                S.rec[2] = mi.a;
                S.rec[3] = mi.b;
                S.rec[4] = delta;
                S.rec[5] = 3;
                S.rec[6] = (int)id;
                S.rec[7] = S.state[kStVersion];
                S.state[kStStatus] = 0;
                if (mode == kModeLS) {
                    if (delta < 0 && S.state[kStSteps] < S.state[kStMaxSteps] && mi.valid)
                        act = 1;
                    else
                        S.state[kStDone] = 1;
                }
            }
        }
    }
    __syncthreads();
    if (!act) return;
    const MoveInfo m = mi;
    apply_move_block(S, m, sh);
    if (threadIdx.x == 0) {
        S.state[kStVersion] += 1;
        S.state[kStSteps] += 1;
        if (mode == kModeLS && S.state[kStSteps] >= S.state[kStMaxSteps]) S.state[kStDone] = 1;
    }
}

// `steps` (nullable): a batch's step counter, advanced once per launch.
// Empty slots of a slot batch (Q = 0) are skipped.  host_out (nullable,
// single solution): pinned host memory that receives the move record and
// state[0..3] straight from the kernel (12 ints), so that no copy follows.
__global__ __launch_bounds__(kApplyThreads) void k_finalize(const SolDev *__restrict__ sols, int mode,
                                                            uint32_t op_mask, int *__restrict__ steps,
                                                            int32_t *__restrict__ host_out = nullptr) {
    if (steps && blockIdx.x == 0 && threadIdx.x == 0) *steps += 1;
    if (sols[blockIdx.x].Q == 0) return;
    const SolDev &S = sols[blockIdx.x];
    finalize_block(S, mode, op_mask);
    if (host_out && threadIdx.x == 0) {  // thread 0 wrote the record and state itself
        for (int q = 0; q < 8; ++q) host_out[q] = S.rec[q];
        for (int q = 0; q < 4; ++q) host_out[8 + q] = S.state[q];
        __threadfence_system();
    }
}


// ------------------------------------------------------------ multi-move --
// Several independent moves per step (Section 7, after Dynasearch): the
// candidates are the per-route-pair bests of the last evaluation
// (S.pairkey); taken in (delta, id) order, a candidate is selected when
// neither of its routes is used by an earlier selection.  Moves on disjoint
// routes keep their deltas and feasibility when applied one after another.
// Up to kMultiCands improving candidates are compacted into LDS and sorted
// (bitonic); with more, rounds of locally dominant candidates give the same
// set.  Requires R <= kMultiMaxR.
constexpr int kMultiCands = 4096;
constexpr int kMultiMaxR = 4096;

__device__ __forceinline__ bool key_improving(unsigned long long k) { return k < 0x8000000000000000ull; }

// kModeRecord: selection only, written to S.msel.  kModeLS: also apply the
// selected moves in order, count the step, and mark the solution converged
// when nothing is selected or the step cap is reached.  Clears S.pairkey.
__global__ __launch_bounds__(kApplyThreads) void k_multi_step(const SolDev *__restrict__ sols, int mode,
                                                              uint32_t op_mask) {
    __shared__ ApplyShared sh;
    __shared__ MoveInfo mi;
    __shared__ unsigned long long keys[kMultiCands];
    __shared__ int pidx[kMultiCands];
    __shared__ unsigned char used[kMultiMaxR];
    __shared__ int cnt_sh, nsel_sh, stop_sh;
    const SolDev &S = sols[0];
    const int tid = threadIdx.x, T = blockDim.x, R = S.R;
    const size_t RR = (size_t)R * R;
    if (mode == kModeLS && S.state[kStDone]) return;
    if (tid == 0) {
        cnt_sh = 0;
        nsel_sh = 0;
        if (mode == kModeLS) ls_count_moves(S, op_mask);
        S.acc[kAccGranInter] = 0;
        S.acc[kAccExtMoves] = 0;
        *S.best_key = ~0ull;
    }
    for (int r = tid; r < R; r += T) used[r] = 0;
    __syncthreads();
    // 1. compact the improving candidates
    for (size_t q = tid; q < RR; q += T) {
        const unsigned long long k = S.pairkey[q];
        if (key_improving(k)) {
            const int slot = atomicAdd(&cnt_sh, 1);
            if (slot < kMultiCands) {
                keys[slot] = k;
                pidx[slot] = (int)q;
            }
        }
    }
    __syncthreads();
    const int cnt = cnt_sh;
    int32_t *sel = S.msel + 1;  // (id, delta) per selected move
    if (cnt <= kMultiCands) {
        // 2a. sort (key, pair) ascending: bitonic over the next power of two
        int np2 = 1;
        while (np2 < cnt) np2 <<= 1;
        for (int q = cnt + tid; q < np2; q += T) {
            keys[q] = ~0ull;
            pidx[q] = 0;
        }
        __syncthreads();
        for (int kk = 2; kk <= np2; kk <<= 1)
            for (int j = kk >> 1; j > 0; j >>= 1) {
                for (int q = tid; q < np2; q += T) {
                    const int p = q ^ j;
                    if (p > q) {
                        const bool up = (q & kk) == 0;
                        const unsigned long long a = keys[q], b = keys[p];
                        if ((a > b) == up) {
                            keys[q] = b;
                            keys[p] = a;
                            const int t2 = pidx[q];
                            pidx[q] = pidx[p];
                            pidx[p] = t2;
                        }
                    }
                }
                __syncthreads();
            }
        // greedy scan in order (one thread)
        if (tid == 0) {
            int ns = 0;
            for (int q = 0; q < cnt; ++q) {
                const int r1 = pidx[q] / R, r2 = pidx[q] - r1 * R;
                if (used[r1] || used[r2]) continue;
                used[r1] = used[r2] = 1;
                sel[2 * ns] = (int32_t)(uint32_t)(keys[q] & 0xFFFFFFFFu);
                sel[2 * ns + 1] = (int)((uint32_t)(keys[q] >> 32) ^ 0x80000000u);
                ++ns;
            }
            nsel_sh = ns;
        }
    } else {
        // 2b. rounds of locally dominant candidates: a candidate whose key is
        // the smallest among the candidates at each of its (free) routes is
        // taken by the sequential greedy too (no smaller key can take one of
        // its routes first), and the candidates dominant in one round share
        // no route; repeating on the routes still free gives the greedy set
        // in a few passes.  The set is then sorted into (delta, id) order.
        unsigned long long *bestr = keys;  // per route (R <= kMultiCands)
        for (;;) {
            for (int r = tid; r < R; r += T) bestr[r] = ~0ull;
            if (tid == 0) stop_sh = 1;
            __syncthreads();
            for (size_t q = tid; q < RR; q += T) {
                const unsigned long long k = S.pairkey[q];
                if (!key_improving(k)) continue;
                const int r1 = (int)(q / R), r2 = (int)(q - (size_t)r1 * R);
                if (used[r1] || used[r2]) continue;
                atomicMin(&bestr[r1], k);
                if (r2 != r1) atomicMin(&bestr[r2], k);
            }
            __syncthreads();
            const int before = nsel_sh;
            for (size_t q = tid; q < RR; q += T) {
                const unsigned long long k = S.pairkey[q];
                if (!key_improving(k)) continue;
                const int r1 = (int)(q / R), r2 = (int)(q - (size_t)r1 * R);
                if (used[r1] || used[r2] || bestr[r1] != k || bestr[r2] != k) continue;
                const int slot = atomicAdd(&nsel_sh, 1);  // < R: the taken candidates share no route
                pidx[slot] = (int)q;
                sel[2 * slot] = (int32_t)(uint32_t)(k & 0xFFFFFFFFu);
                sel[2 * slot + 1] = (int)((uint32_t)(k >> 32) ^ 0x80000000u);
                stop_sh = 0;
            }
            __syncthreads();
            for (int q = before + tid; q < nsel_sh; q += T) {
                const int r1 = pidx[q] / R, r2 = pidx[q] - (pidx[q] / R) * R;
                used[r1] = used[r2] = 1;
            }
            __syncthreads();
            if (stop_sh) break;
        }
        // (delta, id) order: sort the selection's keys (bitonic, in LDS)
        const int cntSel = nsel_sh;
        int np2 = 1;
        while (np2 < cntSel) np2 <<= 1;
        for (int q = tid; q < np2; q += T)
            keys[q] = q < cntSel ? pack_key(sel[2 * q + 1], (uint32_t)sel[2 * q]) : ~0ull;
        __syncthreads();
        for (int kk = 2; kk <= np2; kk <<= 1)
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int q = tid; q < np2; q += T) {
                    const int p2 = q ^ jj;
                    if (p2 > q) {
                        const bool up = (q & kk) == 0;
                        const unsigned long long a = keys[q], b = keys[p2];
                        if ((a > b) == up) {
                            keys[q] = b;
                            keys[p2] = a;
                        }
                    }
                }
                __syncthreads();
            }
        for (int q = tid; q < cntSel; q += T) {
            sel[2 * q] = (int32_t)(uint32_t)(keys[q] & 0xFFFFFFFFu);
            sel[2 * q + 1] = (int)((uint32_t)(keys[q] >> 32) ^ 0x80000000u);
        }
    }
    __syncthreads();
    const int ns = nsel_sh;
    if (tid == 0) S.msel[0] = ns;
    // 3. clear the table for the next evaluation
    for (size_t q = tid; q < RR; q += T) S.pairkey[q] = ~0ull;
    __syncthreads();
    if (mode != kModeLS) return;
    // 4. apply the selection.  Routes are disjoint, so the new layout is the
    // old one with each touched route replaced by its new node sequence: its
    // nodes go into nr_alt (with the new route offsets), then one rebuild of
    // every attribute.  The decoded moves reuse the key array; a selection
    // too large for it is applied move by move instead.
    MoveInfo *mv = reinterpret_cast<MoveInfo *>(keys);
    constexpr int kBatchApply = (int)(sizeof(keys) / (sizeof(MoveInfo)));
    if (ns <= kBatchApply) {
        int *mov_of = pidx;  // per route: the selected move touching it, or -1
        for (int r = tid; r < R; r += T) mov_of[r] = -1;
        __syncthreads();
        for (int q = tid; q < ns; q += T) {
            decode_move(S, (uint32_t)sel[2 * q], mv[q]);
            mv[q].delta = sel[2 * q + 1];
        }
        __syncthreads();
        for (int q = tid; q < ns; q += T)
            if (mv[q].valid) {
                mov_of[mv[q].ra] = q;
                mov_of[mv[q].rb] = q;
            }
        __syncthreads();
        auto newL = [&](int r) {
            const int q = mov_of[r];
            if (q < 0) return S.roff[r + 1] - S.roff[r] - 1;
            return r == mv[q].ra ? mv[q].nLa : mv[q].nLb;
        };
        // new offsets: an exclusive scan of newL + 1 over the routes (each
        // thread a contiguous run of routes, then the threads' totals)
        const int per = (R + T - 1) / T, r0 = min(tid * per, R), r1 = min(r0 + per, R);
        int own = 0;
        for (int r = r0; r < r1; ++r) own += newL(r) + 1;
        int incl = own;
        const int lane = tid & 63, wave = tid >> 6;
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        if (lane == 63) sh.red[wave][0] = incl;
        __syncthreads();
        int before = incl - own;
        for (int w = 0; w < wave; ++w) before += (int)sh.red[w][0];
        for (int r = r0; r < r1; ++r) {
            S.roff_alt[r] = before;
            before += newL(r) + 1;
        }
        if (tid == 0) S.roff_alt[R] = S.Q;
        __syncthreads();
        // nodes of the new layout, one wavefront per route
        for (int r = wave; r < R; r += T / 64) {
            const int q = mov_of[r], base = S.roff_alt[r], nl = newL(r);
            for (int p = lane; p <= nl; p += 64)
                S.nr_alt[base + p] = make_int2(q < 0 ? old_node(S, r, p) : new_node(S, mv[q], r, p), r);
        }
        if (tid == 0) S.nr_alt[S.Q] = make_int2(0, R);
        __threadfence_block();
        __syncthreads();
        rebuild(S, S.nr_alt, S.roff_alt, sh);
        if (S.pen || S.pd || S.gen) pen_all(S, sh);
        if (tid == 0)
            for (int q = 0; q < ns; ++q) S.state[kStVersion] += mv[q].valid ? 1 : 0;
    } else {
        for (int q = 0; q < ns; ++q) {
            if (tid == 0) {
                decode_move(S, (uint32_t)sel[2 * q], mi);
                mi.delta = sel[2 * q + 1];
            }
            __syncthreads();
            const MoveInfo m = mi;
            if (m.valid) apply_move_block(S, m, sh);
            __syncthreads();
            if (tid == 0 && m.valid) S.state[kStVersion] += 1;
        }
    }
    if (tid == 0) {
        if (ns > 0) {
            const int q = 0;  // the record holds the first (best) selected move
            S.rec[4] = sel[2 * q + 1];
            S.rec[6] = sel[2 * q];
            S.state[kStSteps] += 1;
            S.acc[kAccMultiApplied] += ns;
            S.state[kStStatus] = 0;
        } else {
            S.state[kStStatus] = 1;
        }
        if (ns == 0 || S.state[kStSteps] >= S.state[kStMaxSteps]) S.state[kStDone] = 1;
    }
}

// ------------------------------------------------------ instance checks ----
// out[0] |= 1 value out of range, 2 asymmetric, 4 nonzero diagonal,
//           8 bad node data; out[1] = max distance; out[2] = max e;
// out[3] = max l; out[4] = max s; out[5] = max demand.
__global__ __launch_bounds__(256) void k_check_dist(const int32_t *__restrict__ D, int np1,
                                                    int32_t *out) {
    __shared__ int ta[32][33], tb[32][33];
    const int I = blockIdx.y * 32, J = blockIdx.x * 32;
    const int x = threadIdx.x & 31, y0 = threadIdx.x >> 5;
    int bad = 0, mx = 0;
    for (int y = y0; y < 32; y += 8) {
        const int i = I + y, j = J + x;
        ta[y][x] = (i < np1 && j < np1) ? D[(size_t)i * np1 + j] : 0;
        const int i2 = J + y, j2 = I + x;
        tb[y][x] = (i2 < np1 && j2 < np1) ? D[(size_t)i2 * np1 + j2] : 0;
    }
    __syncthreads();
    for (int y = y0; y < 32; y += 8) {
        const int i = I + y, j = J + x;
        if (i >= np1 || j >= np1) continue;
        const int d = ta[y][x];
        if (d < 0 || d >= (1 << 24)) bad |= 1;
        if (d != tb[x][y]) bad |= 2;
        if (i == j && d != 0) bad |= 4;
        mx = max(mx, d);
    }
    if (bad) atomicOr(&out[0], bad);
    atomicMax(&out[1], mx);
}

// 16-bit copy of D (every value < 2^16), rows padded to `stride` with zeros.
__global__ __launch_bounds__(256) void k_pack16(const int32_t *__restrict__ D, int np1, int stride,
                                                uint16_t *__restrict__ out) {
    const int u = blockIdx.y;
    for (int v = blockIdx.x * 256 + threadIdx.x; v < stride; v += gridDim.x * 256)
        out[(size_t)u * stride + v] = v < np1 ? (uint16_t)D[(size_t)u * np1 + v] : (uint16_t)0;
}

__global__ __launch_bounds__(256) void k_check_nodes(const int4 *__restrict__ nd, int np1, int has_tw,
                                                     int32_t *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np1) return;
    const int4 q = nd[i];
    const int lim = 1 << 26;
    bool bad = q.x < 0 || q.x >= lim || (i == 0 && q.x != 0);
    if (has_tw) {
        bad = bad || q.y < 0 || q.z < q.y || q.w < 0 || q.z >= lim || q.w >= lim || (i == 0 && q.w != 0);
        atomicMax(&out[2], q.y);
        atomicMax(&out[3], q.z);
        atomicMax(&out[4], q.w);
    }
    if (bad) atomicOr(&out[0], 8);
    atomicMax(&out[5], q.x);
}

// Marks every route's distance-block cache entry empty.
// Pickup amounts: chk[0] |= 1 for a negative amount or a nonzero depot
// entry; chk[1] = the largest amount.
__global__ __launch_bounds__(256) void k_check_pick(const int32_t *__restrict__ pick, int np1, int32_t *chk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np1) return;
    const int v = pick[i];
    if (v < 0 || (i == 0 && v != 0)) atomicOr(chk, 1);
    atomicMax(chk + 1, v);
}

__global__ void k_route_blocks_clear(int32_t *rblk, int R) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) rblk[(size_t)r * kRouteBlockWords] = -1;
}

__global__ void k_fill_u64(unsigned long long *p, size_t count) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = ~0ull;
}

__global__ void k_zero_i32(int32_t *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

// Gather the converged flags of a batch into one array (one copy to the
// host); an empty slot reads as converged.
__global__ void k_poll_done(const SolDev *__restrict__ sols, int nsols, int32_t *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsols) out[i] = sols[i].Q == 0 ? 1 : sols[i].state[kStDone];
}

// Per-solution results of a batch in one array: {steps, version | converged
// << 32, moves evaluated, cost} per solution, for a single copy to the host
// (an empty slot: zeros, converged).
__global__ void k_collect(const SolDev *__restrict__ sols, int nsols, long long *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsols) {
        const SolDev &S = sols[i];
        if (S.Q == 0) {
            out[4 * i] = 0;
            out[4 * i + 1] = 1ll << 32;
            out[4 * i + 2] = 0;
            out[4 * i + 3] = 0;
            return;
        }
        out[4 * i] = S.state[kStSteps];
        out[4 * i + 1] = (long long)(uint32_t)S.state[kStVersion] | ((long long)(S.state[kStDone] != 0) << 32);
        out[4 * i + 2] = S.acc[kAccMoves];
        out[4 * i + 3] = S.acc[kAccCost];
    }
}

// Reset per-solution state for a new run (no memset, so it can sit in a
// captured graph).
__global__ void k_reset_state(const SolDev *__restrict__ sols, int nsols, int max_steps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsols || sols[i].Q == 0) return;
    const SolDev &S = sols[i];
    S.state[kStDone] = 0;
    S.state[kStSteps] = 0;
    S.state[kStStatus] = 0;
    S.state[kStMaxSteps] = max_steps;
    S.acc[kAccMoves] = 0;
    S.acc[kAccFullPairs] = 0;
    S.acc[kAccScreenPairs] = 0;
    S.acc[kAccMultiApplied] = 0;
    *S.best_key = ~0ull;
}

// Measurement aid: reads `chunks` KiB from src into LDS with the 16-byte
// LDS DMA that stages 16-bit distance rows (one KiB per wavefront
// instruction) and discards them, so that a profiler's fetch counter can be
// scaled for exactly that kind of request.  Each wavefront cycles through
// four 1 KiB slots of its own and drains them every fourth instruction.
__global__ __launch_bounds__(256) void k_probe_stream(const int *__restrict__ src, long long chunks) {
    __shared__ int4 buf[4 * 4 * 64];  // 4 wavefronts x 4 slots x 1 KiB
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int k = 0;
    for (long long c = (long long)blockIdx.x * 4 + wave; c < chunks; c += (long long)gridDim.x * 4) {
        int *dst = (int *)(buf + (wave * 4 + (k & 3)) * 64);
        __builtin_amdgcn_global_load_lds((global_void_ptr)(src + c * 256 + 4 * lane), (lds_void_ptr)dst, 16, 0, 0);
        if ((++k & 3) == 0) __builtin_amdgcn_s_waitcnt(0);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// Sum of the screening counters over a batch's solutions (one thread).
__global__ void k_screen_sum(const SolDev *__restrict__ sols, int nsols, long long *out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    long long f = 0, p = 0;
    for (int i = 0; i < nsols; ++i)
        if (sols[i].Q) {
            f += sols[i].acc[kAccFullPairs];
            p += sols[i].acc[kAccScreenPairs];
        }
    out[0] = f;
    out[1] = p;
}

}  // namespace tga
