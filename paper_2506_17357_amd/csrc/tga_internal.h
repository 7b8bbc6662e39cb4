// Internal layout shared by the host runtime (api.hip) and the kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tga {

// Time sentinels (hard windows).  Every finite time on the path stays below
// 2^28 (checked when an instance is loaded), so a sentinel plus or minus a few
// finite terms, and differences of two such sums, stay inside int32.
constexpr int32_t kInf = 1 << 29;    // "cannot be reached in time"
constexpr int32_t kNeg = -(1 << 29); // "no feasible arrival time"
constexpr int32_t kNoDelta = 0x7FFFFFFF;

// Slot flags (bits 16.. of a4.x; bits 0..15 hold the node, n < 2^14).
constexpr int32_t kFlagCustomer = 1;
constexpr int32_t kFlagRemCap = 2;  // route load - own demand <= capacity
constexpr int32_t kFlagRemTw = 4;   // route stays window-feasible without this node

// One solution as the kernels see it.  Slots are route-major: route r owns
// slots roff[r] .. roff[r+1]-1, its start depot first; slot Q is a sentinel
// holding node 0 (the end depot of the last route).
struct SolDev {
    // instance (borrowed)
    const int32_t *D;     // (n+1)^2 row-major
    const uint16_t *D16;  // the same values as uint16, rows of stride16 (null when some d >= 2^16)
    int32_t stride16;
    int32_t pad16;
    const int4 *node4;    // {demand, e, l, s}
    int32_t n, np1, cap, has_tw;
    int32_t R, Q;
    int32_t tile_rows;    // rows per inter-route work item for this solution
    int32_t pad0;
    // per slot, Q+1 entries
    int4 *a4;    // {node | flags << 16, route, edge to successor, removal delta}
    int4 *b4;    // {demand, prefix load (incl.), route load, sum of the two incident edges}
    int4 *t4;    // {departure time, latest arrival at successor, departure of predecessor, latest arrival here}
    int4 *w4;    // {e, l, s, 0}
    int32_t *pdist;   // distance from the start depot along the route
    // per ref (Q)
    int32_t *ref2slot;
    // per route
    int32_t *roff;    // R+1
    int32_t *rdist;   // R
    // apply / build staging
    int2 *nr_alt;     // Q+1 {node, route} of the next layout
    int32_t *roff_alt;// R+1
    // per route: the route's distance sub-block as last staged (see kRouteBlock*)
    int32_t *rblk;
    // penalised mode (feasible and infeasible search): per slot the
    // time-warp summary {T_D, T_E, T_L, T_V} of the route prefix ending at
    // the slot (start depot included) and of the suffix starting there (end
    // depot included); weights of load excess and time warp
    int4 *pf4;
    int4 *pb4;
    int32_t pen, wL, wT, pd;  // pd: pickups (VRPSPDTW), evaluated by the same path
    int32_t gen, pad2;        // gen: evaluated by the general path (operator variants)
    // pickups: per node amount (borrowed), per slot the load summary
    // {L_I, L_O, L_M, 0} of the prefix ending at the slot and of the suffix
    // starting there (Section 4.3.2)
    const int32_t *pick;
    int4 *pl4;
    int4 *ql4;
    // multi-move (caller workspace, null when off): per pair of route slots
    // r1 <= r2 the best improving key of the last evaluation (R x R, entry
    // r1 * R + r2), and the selection {count, (id, delta) per move}
    unsigned long long *pairkey;
    int32_t *msel;
    // per-solution state
    unsigned long long *best_key;  // running minimum of (delta, id) keys
    int32_t *rec;     // 8 ints: the tga_move_t of the last finalize
    int32_t *state;   // kState* below
    long long *acc;   // kAcc* below
};

// state[] entries
enum {
    kStDone = 0,       // local optimum (or step cap) reached in LS mode
    kStSteps = 1,      // accepted moves so far
    kStStatus = 2,     // 0 ok, 1 no admissible move, -1 invalid move
    kStVersion = 3,    // applied moves (host-visible version)
    kStMaxSteps = 4,   // step cap for LS mode
    kStCount
};
// acc[] entries
enum {
    kAccCost = 0,       // total distance of the current solution
    kAccMoves = 1,      // sum of |N(S_t)| over evaluations run in LS mode
    kAccCnt0 = 2,       // |N(S)| per operator, 5 entries
    kAccGranInter = 7,  // inter-route moves of the granular neighbourhood counted by the last evaluation
    kAccLoadExcess = 8, // penalised mode: total load above capacity
    kAccTimeWarp = 9,   // penalised mode: total time warp
    kAccExtMoves = 10,  // operator-variant moves counted by the last evaluation
    kAccFullPairs = 11, // local search: slot pairs of different routes evaluated in full (past the screens)
    kAccScreenPairs = 12, // local search: slot pairs of different routes visited by those evaluations
    kAccMultiApplied = 13, // multi-move local search: moves applied
    kAccCount = 14
};

// Inter-route work item: rows [s0, s1) against column slots [c0, c0 + the
// item's column span); only pairs whose column lies in a later route count.
// Row stride (elements) of the 16-bit copy of D: a multiple of 8 keeps every
// row 16-byte aligned.
constexpr int stride16_of(int np1) { return (np1 + 7) & ~7; }

constexpr int kMaxXcds = 8;  // accelerator dies (each with its own L2) the batched items are spread over
constexpr int kMaxBatchGrid = 4096;  // workgroups of one batched evaluation launch

// Route distance-block cache, one entry of kRouteBlockWords ints per route:
// {P, unused, node of positions 0..P-1 (kRouteBlockMaxP slots), the P x P
// block D[node(p)][node(q)] row-major}.  An entry is used only when P and
// every node equal the route's current ones, so it never needs to be
// invalidated; P = -1 marks an empty entry.  Routes with more than
// kRouteBlockMaxP positions are not cached.
constexpr int kRouteBlockMaxP = 40;
constexpr int kRouteBlockNodes = 2;
constexpr int kRouteBlockData = kRouteBlockNodes + kRouteBlockMaxP;
constexpr int kRouteBlockWords = 1664;  // >= kRouteBlockData + kRouteBlockMaxP^2, a multiple of 64
static_assert(kRouteBlockData + kRouteBlockMaxP * kRouteBlockMaxP <= kRouteBlockWords, "route block entry");

struct InterItem {  // row slots [s0, s1) of solution `sol`
    int32_t sol, s0, s1, pad;
};

// Intra-route work item: routes [r0, r1) of one solution, one wavefront.
struct IntraItem {
    int32_t sol, r0, r1, pad;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace tga
