/*
 * tga.h — C ABI of the MI355X (gfx950) full-neighbourhood move evaluator for
 * VRP local search.
 *
 * The library evaluates, for one solution (or a batch of solutions) held on
 * the GPU, every move of the canonical neighbourhood N(S) built from the
 * paper's operators (Section 4.1, Fig. 2: relocate, swap, 2-opt*, 2-opt, and
 * or-opt as the intra-route segment relocation), gives each move its exact
 * integer distance delta and a capacity / time-window feasibility mask,
 * reduces to the best admissible move (Section 5.3.4, eq. scoring_tensor,
 * eq. mask, eq. min_obj: infeasible moves score +infinity, argmin with the
 * lowest move id winning ties), applies it and rebuilds the route attributes
 * (Section 5.3.5) on the device.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All integers are int32 unless stated.  Every value on the path is an
 *   integer; no floating point is used.
 * - Return value: TGA_OK (0) on success, TGA_ENOMOVE (1) when no move is
 *   admissible (not an error), a negative TGA_E* code on failure.  On failure
 *   tga_last_error() returns a message (thread-local, valid until the next
 *   call on the same thread).  Arguments are validated before any device
 *   work; the exceptions are stated per call (instance values checked on the
 *   device by tga_load_instance, move ids by tga_apply_move).
 * - Device memory is owned by the caller (typically PyTorch tensors).  The
 *   library borrows the buffers for the lifetime of the handle that received
 *   them and never frees them.  Host arrays are read during the call only.
 * - `stream` is a hipStream_t passed as void* (NULL = default stream).  A
 *   handle must be used from one stream at a time.
 * - Instance data: node 0 is the depot, customers are 1..n.  Travel time is
 *   the distance (one matrix).  The matrix must be symmetric with a zero
 *   diagonal (2-opt reversal relies on symmetry, as Section 4.1 requires).
 * - Refs: customer c is ref c-1; the start depot of route slot r is ref n+r;
 *   Q = n + R.  Move id = ((op*4 + k)*Q + a)*Q + b with (a, b) refs:
 *     op 0 RELOCATE k=1: customer a moves right after ref b (other route)
 *     op 1 SWAP     k=1: customers a < b exchange places (any routes)
 *     op 2 2OPT*    k=0: refs a < b in different routes exchange their tails
 *     op 3 2OPT     k=0: customers a < b of one route: reverse a..b
 *     op 4 OR-OPT   k=1..3: the k-segment starting at customer a moves,
 *                   orientation kept, right after ref b of the same route
 *   Q <= 14654 keeps every id below 2^32.
 * - Objective: total distance (eq. objective with mu1 = 0, mu2 = 1).
 *   feas bit0: every touched route respects the capacity; bit1: every touched
 *   route respects the windows (depart the depot at e_0, wait when early,
 *   infeasible when arriving after l_i, back by l_0; Section 2).  A move is
 *   admissible when feas == 3.
 */
#ifndef TGA_H
#define TGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TGA_OK = 0,
    TGA_ENOMOVE = 1,   /* no admissible move; not an error */
    TGA_EINVAL = -1,   /* bad argument (null pointer, bad partition, bad move) */
    TGA_ERANGE = -2,   /* a size or value outside the supported range */
    TGA_ENOMEM = -3,   /* workspace too small */
    TGA_EDEVICE = -4,  /* a HIP runtime call failed */
    TGA_ESTALE = -5    /* move record not produced for this solution version */
};

enum {
    TGA_OP_RELOCATE = 1u << 0,
    TGA_OP_SWAP = 1u << 1,
    TGA_OP_2OPTSTAR = 1u << 2,
    TGA_OP_2OPT = 1u << 3,
    TGA_OP_OROPT = 1u << 4,
    TGA_OP_ALL = 0x1Fu,
    /* operator variants (general path only, tga_solution_set_general):
     *   op 5 SEGMENT RELOCATE  k=2,3: the k-segment starting at customer a
     *        moves, orientation kept, right after ref b of another route
     *   op 6 REVERSED RELOCATE k=2,3: the same, the segment reversed
     *   op 7..9 CROSS-EXCHANGE: the (op-6)-segment starting at customer a and
     *        the k-segment (k=1..3) starting at customer b (a < b, different
     *        routes) exchange places, each in its orientation (op 7, k=1 is
     *        SWAP and is left out) */
    TGA_OP_SEGREL = 1u << 5,
    TGA_OP_SEGREL_REV = 1u << 6,
    TGA_OP_CROSS = 1u << 7,
    TGA_OP_VARIANTS = 0xE0u,
    /* modifier: inter-route operators restricted to the granular pairs of the
     * instance (tga_instance_set_granular); single-solution calls only */
    TGA_OP_GRANULAR = 1u << 16,
    /* modifier (batched local search: tga_batch_ls_run, tga_batch_step_part,
     * tga_batch_tick): run the instantiation of the evaluation launch that
     * also counts the slot pairs evaluated in full (tga_batch_screen_stats);
     * the same results, a few per cent slower */
    TGA_OP_COUNT_FULL = 1u << 17,
    /* modifier (general path, after tga_solution_set_multi): several
     * independent moves per local-search step (tga_ls_run), and the
     * per-route-pair table that tga_solution_select_moves reads after
     * tga_eval_neighborhood */
    TGA_OP_MULTI = 1u << 18
};

#define TGA_MAX_Q 14654
/* with the operator variants ids reach 40*Q*Q */
#define TGA_MAX_Q_VARIANTS 10362

typedef struct tga_instance *tga_instance_t;
typedef struct tga_solution *tga_solution_t;
typedef struct tga_batch *tga_batch_t;

/* Best-move record (32 bytes).  op/k/a/b decode `id`; feas is 3 for a
 * returned best move; version is the solution version it was computed on. */
typedef struct {
    int32_t op, k, a, b, delta;
    uint32_t feas, id, version;
} tga_move_t;

/* Device workspace sizes (bytes) for an instance of n customers and for a
 * solution with R route slots.  Returns 0 when n or R is out of range.  A
 * solution workspace holds the slot attributes, the work lists of the
 * single-solution form and, per route, the route's distance sub-block as
 * last staged by the intra-route evaluation (6.5 KB per route; an entry is
 * used only while the route's node sequence is unchanged). */
size_t tga_instance_workspace_bytes(int32_t n);
size_t tga_solution_workspace_bytes(int32_t n, int32_t R);

/* Section 5.1 (the solution tensor lives on the GPU) and Section 2 (instance
 * data).  Registers an instance.
 *   dist   device, (n+1)*(n+1) int32, row-major, symmetric, zero diagonal,
 *          0 <= d < 2^24.
 *   node4  device, (n+1) x {demand, e, l, s} int32; node 0 is the depot with
 *          demand 0 and s = 0; 0 <= e <= l; s >= 0.
 *   capacity  vehicle capacity (>= 0).   has_tw  0 = CVRP, 1 = VRPTW.
 *   ws     device workspace of tga_instance_workspace_bytes(n) bytes,
 *          256-byte aligned (it also holds a 16-bit copy of D, rows 16-byte
 *          aligned, when every distance is below 2^16).
 * Values are checked on the device before the handle is returned
 * (TGA_EINVAL for asymmetry / negative values, TGA_ERANGE when sums along a
 * route could leave the exact int32 range).  Synchronises `stream`. */
int tga_load_instance(int32_t n, const int32_t *dist, const int32_t *node4, int32_t capacity,
                      int32_t has_tw, void *ws, size_t ws_bytes, void *stream,
                      tga_instance_t *out);

/* Section 5.3.1 (edge-based extraction) with the granularity threshold
 * theta of the paper's experiments: the neighbourhood reduction of the
 * edge-implemented form.  Node j is a neighbour of node i when it is among
 * the theta nodes closest to i (distance, then node id; i excluded; node 0
 * is the depot and stands for the start depot of every route); the mask
 * keeps the pairs {i, j} where either is a neighbour of the other.  With
 * TGA_OP_GRANULAR in op_mask, tga_eval_neighborhood and tga_ls_run evaluate
 * the inter-route moves (RELOCATE, SWAP across routes, 2OPT*) only for refs
 * whose nodes form a kept pair; intra-route moves stay complete.  Move ids
 * are unchanged.  The neighbour lists are computed on the device
 * (1 <= theta <= min(n, 512)); the pair lists live in `ws`
 * (tga_granular_workspace_bytes(n, theta) bytes, 256-byte aligned, caller
 * owned, borrowed for the instance's lifetime).  Synchronises `stream`. */
size_t tga_granular_workspace_bytes(int32_t n, int32_t theta);
int tga_instance_set_granular(tga_instance_t inst, int32_t theta, void *ws, size_t ws_bytes, void *stream);

/* Simultaneous pickup and delivery (VRPSPDTW; Section 2 and the load
 * attributes of Section 4.3.2): pickup amounts per node, device, (n+1)
 * int32, 0 at the depot, borrowed for the instance's lifetime.  The vehicle
 * leaves the depot with all of its route's deliveries (node4 demands) and
 * at each customer unloads the delivery and loads the pickup; feas bit0
 * then requires the largest load on every touched route to be within the
 * capacity, intra-route moves included.  Solutions set up after this call
 * use it; they are evaluated one at a time (no batch, no TGA_OP_GRANULAR)
 * by the kernels that concatenate per-slot load and time-warp summaries,
 * in hard or (tga_solution_set_penalty) penalised mode.  TGA_EINVAL for a
 * negative amount or a nonzero depot entry.  Synchronises `stream`. */
int tga_instance_set_pickups(tga_instance_t inst, const int32_t *pickup, void *stream);

/* Adjacency entries of the customer rows of the granular pairs (each kept
 * pair of customers counted twice, a customer-depot pair once); 0 before
 * tga_instance_set_granular. */
int32_t tga_instance_granular_pairs(tga_instance_t inst);

/* Bytes per distance the inter-route kernels stream for this instance: 2
 * when every distance is below 2^16 (tga_load_instance then keeps a 16-bit
 * copy of D in the instance workspace), else 4.  0 for a null handle. */
int32_t tga_instance_dist_bytes(tga_instance_t inst);

/* Section 5.1 and Alg. A2 (initialise the solution tensor from S), Section
 * 5.2 and the positional tensors of Section 5.3.1 (route id and position of
 * every node).  Uploads a solution and builds its attribute arrays.
 *   offsets    host, R+1, offsets[0] = 0, nondecreasing, offsets[R] = n.
 *   customers  host, n; route r holds customers[offsets[r] .. offsets[r+1]);
 *              must be a permutation of 1..n.  Empty routes are allowed.
 *   ws         device workspace of tga_solution_workspace_bytes(n, R).
 * Requires n + R <= TGA_MAX_Q.  Synchronises `stream`. */
int tga_set_solution(tga_instance_t inst, int32_t R, const int32_t *offsets,
                     const int32_t *customers, void *ws, size_t ws_bytes, void *stream,
                     tga_solution_t *out);

/* Replace the routes of an existing solution (same instance, same R) and
 * rebuild its attributes in place: the workspace, and every batch or captured
 * graph that refers to the solution, stay valid.  Resets the version to 0
 * and empties the per-route distance-block cache.  Same argument rules as
 * tga_set_solution.  Synchronises `stream`. */
int tga_solution_reload(tga_solution_t sol, const int32_t *offsets, const int32_t *customers,
                        void *stream);

/* Sections 5.3.1-5.3.4: evaluate every move of N(S) whose operator bit is in
 * op_mask and return the best admissible one in *best (host).  Returns
 * TGA_ENOMOVE when none is admissible (then *best is zeroed).
 * Optional per-move dump (testing): dump_delta (int32) and dump_feas (uint8)
 * are device arrays of 20*Q*Q entries indexed by move id; the library writes
 * only entries that are moves, the caller pre-fills the rest.  Both NULL, or
 * both set.  Synchronises `stream` (the returned record is the best-move
 * latency). */
int tga_eval_neighborhood(tga_solution_t sol, uint32_t op_mask, tga_move_t *best,
                          int32_t *dump_delta, uint8_t *dump_feas, void *stream);

/* For callers that cannot allocate device memory (code being captured into
 * a HIP graph, tight serving loops, harnesses that forbid hipMalloc): the
 * result of tga_set_solution followed by tga_eval_neighborhood(op_mask, no
 * dump) on the routes given, without a caller workspace.  The solution's
 * attribute arrays and work lists go into a library-owned static device
 * buffer of TGA_STATIC_SCRATCH_BYTES per GPU (held from the library's load
 * until the process ends); the call allocates no device or pinned memory.
 *   inst      a loaded instance (its buffers as for tga_load_instance).
 *   R, offsets, customers   as for tga_set_solution (host arrays).
 *   best      host; the best admissible move, version 0.
 * Returns TGA_ENOMOVE as tga_eval_neighborhood does, and TGA_ERANGE when
 * the solution needs more than TGA_STATIC_SCRATCH_BYTES (the workspace size
 * tga_solution_workspace_bytes reports; 8 MiB holds n = 10^4 customers with
 * up to 990 routes).  Every call on one GPU uses that
 * GPU's one buffer and overwrites what the previous call left there: calls
 * that overlap on one GPU (other host threads, or other streams before the
 * previous call returned) race.  Synchronises `stream`. */
#define TGA_STATIC_SCRATCH_BYTES (8u << 20)
int tga_eval_routes_static(tga_instance_t inst, int32_t R, const int32_t *offsets,
                           const int32_t *customers, uint32_t op_mask, tga_move_t *best, void *stream);

/* Section 5.3.5 and Alg. A2: apply a move to the solution on the device and
 * rebuild every attribute.  The move need not be improving or admissible.
 * Returns TGA_ESTALE if move->version is not the solution's current version
 * (checked on the host) and TGA_EINVAL if move->id is not a move of N(S):
 * ids of 40*Q*Q or more (beyond the ten operators' id range) are refused on
 * the host; whether a smaller id names
 * a move of the current routes is decided on the device by the launch that
 * would apply it, which then leaves the solution unchanged.  On success the
 * version increases by one and *new_cost (nullable) receives the total
 * distance.  Synchronises `stream`. */
int tga_apply_move(tga_solution_t sol, const tga_move_t *move, int64_t *new_cost, void *stream);

/* Alg. A2 run on the device: repeat {evaluate, apply the best move if its
 * delta < 0} until a local optimum or max_steps accepted moves.  The host
 * does not inspect any step.  *steps_done (nullable) = accepted moves,
 * *moves_evaluated (nullable) = sum of |N(S_t)| over the evaluations run,
 * *cost (nullable) = final distance.  Synchronises `stream`. */
int tga_ls_run(tga_solution_t sol, uint32_t op_mask, int32_t max_steps, int32_t *steps_done,
               int64_t *moves_evaluated, int64_t *cost, void *stream);

/* Clear the converged flag and the step / move counters of a solution and
 * set its step cap, so that it can join a running batch (tga_batch_step_part)
 * and stop on its own after max_steps accepted moves.  Asynchronous. */
int tga_solution_begin(tga_solution_t sol, int32_t max_steps, void *stream);

/* Read the current solution back: offsets (host, R+1), customers (host, n),
 * *cost (nullable) = total distance.  Synchronises `stream`. */
int tga_get_solution(tga_solution_t sol, int32_t *offsets, int32_t *customers, int64_t *cost,
                     void *stream);

/* Feasible and infeasible search (Alg. A2) with the scoring function of
 * eq. scoring_tensor read as a weighted sum of the attribute deltas of
 * Section 5.3.3: with w_load >= 0 the solution switches to penalised mode,
 * where every move of N(S) is admissible and scores
 *     dD + w_load * dL_V + w_tw * dT_V
 * over the touched routes; L_V = a route's load above the capacity, T_V =
 * its time warp (Section 4.3.3: arriving after l_i costs the lateness and
 * service starts at l_i; leaving the depot at e_0, waiting when early).  The
 * best move is the lexicographic minimum of (score, id); tga_ls_run applies
 * it while the score is negative; tga_move_t.delta is the score and the
 * dumps hold scores (dump_feas still has the hard capacity / window bits).
 * w_load < 0 returns to hard feasibility.  w_tw must be 0 without windows.
 * TGA_ERANGE when the weights could take a score outside +-2^29.  Penalised
 * solutions are evaluated one at a time (no batch, no TGA_OP_GRANULAR); with
 * pickups L_V is the largest load's excess.
 * Synchronises `stream`. */
int tga_solution_set_penalty(tga_solution_t sol, int32_t w_load, int32_t w_tw, void *stream);

/* General path on (on = 1) or off (0): evaluations concatenate per-slot
 * time-warp and load summaries per pair of slots and per intra-route walk
 * (the kernels penalised mode and pickups use), which the operator variants
 * (TGA_OP_SEGREL, TGA_OP_SEGREL_REV, TGA_OP_CROSS; n + R <=
 * TGA_MAX_Q_VARIANTS, dumps of 40*Q*Q entries) require.  Results of the
 * five base operators are identical on either path.  Synchronises
 * `stream`. */
int tga_solution_set_general(tga_solution_t sol, int32_t on, void *stream);

/* Multi-move local search (Section 7: apply several independent moves per
 * iteration instead of one, after Dynasearch).  Candidates: for every pair of
 * route slots r1 <= r2 (r1 = r2: moves inside one route) the best admissible
 * improving move touching exactly those routes.  Selection: candidates in
 * (delta, id) order, each taken when none of its routes is taken yet
 * (greedy, route-disjoint).  Moves on disjoint routes are independent: each
 * keeps its delta and feasibility, so applying the selection in order
 * improves the objective by the sum of the selected deltas.
 *
 * tga_multi_workspace_bytes: device bytes of the table and the selection for
 * R routes.  tga_solution_set_multi: hand a caller-owned device workspace of
 * that size (256-byte aligned; NULL turns multi-move off) to the solution;
 * puts it on the general path (tga_solution_set_general); needs R <= 4096.
 * Then tga_ls_run with TGA_OP_MULTI runs steps of {evaluate, select, apply
 * the selection}: steps_done counts steps, tga_solution_multi_stats reports
 * {steps, moves applied}.  tga_eval_neighborhood with TGA_OP_MULTI fills the
 * table; tga_solution_select_moves then returns the selection (count moves,
 * the first min(count, cap) written to `moves` in selection order) without
 * applying it, and empties the table.  Synchronise `stream`. */
size_t tga_multi_workspace_bytes(int32_t R);
int tga_solution_set_multi(tga_solution_t sol, void *ws, size_t ws_bytes, void *stream);
int tga_solution_select_moves(tga_solution_t sol, tga_move_t *moves, int32_t cap, int32_t *count,
                              void *stream);
int tga_solution_multi_stats(tga_solution_t sol, int64_t out[2], void *stream);

/* General path: total load excess and total time warp of the current
 * solution (nullable outputs).  Synchronises `stream`. */
int tga_solution_violations(tga_solution_t sol, int64_t *load_excess, int64_t *time_warp, void *stream);

/* Counters of a solution (all nullable): accepted moves since the last
 * begin / ls_run, converged flag, moves evaluated since then, current total
 * distance.  Synchronises `stream`. */
int tga_solution_stats(tga_solution_t sol, int32_t *steps_done, int32_t *converged,
                       int64_t *moves_evaluated, int64_t *cost, void *stream);

/* Screening counters of the batched local-search evaluations run with
 * TGA_OP_COUNT_FULL since the last reset (tga_batch_begin, tga_batch_reset,
 * tga_batch_ls_run), for this solution: pairs[0] = slot pairs of different
 * routes whose inter-route moves (RELOCATE, SWAP, 2OPT*) were evaluated in
 * full, feasibility and move ids, because some delta could still reach the
 * evaluation's best (the argmin of Section 5.3.4 needs the mask only there);
 * pairs[1] = slot pairs of different routes the same evaluations visited.
 * Synchronises `stream`. */
int tga_solution_screen_stats(tga_solution_t sol, int64_t pairs[2], void *stream);

/* Measurement aid (profiler calibration, not part of the method): reads
 * `bytes` (a multiple of 1024) of device memory at `src` (16-byte aligned)
 * once, through the same 16-byte LDS DMA that stages the 16-bit distance
 * rows, and discards them, so that a hardware fetch counter can be scaled
 * for that kind of request.  TGA_EINVAL for a misaligned source or size.
 * Synchronises `stream`. */
int tga_probe_stream_read(const void *src, size_t bytes, void *stream);

/* Schedules per problem kind and size, as an autotuner measured them (a
 * table the caller loads, e.g. from a JSON file the tuner wrote): an entry
 * applies to solutions of its kind (has_tw 0 = CVRP, 1 = with time windows
 * or pickups) with n <= n_max, the entry with the smallest such n_max
 * winning.  plain_rows: rows per inter-route item of the single-solution
 * form (capped by what one workgroup's LDS holds); item_rows: rows per
 * inter-route item of the batched form (up to one LDS sub-block: thin items;
 * more: rounded up to whole sub-blocks); 0 keeps the built-in rule.  Results
 * never depend on the schedule. */
typedef struct {
    int32_t has_tw, n_max, plain_rows, item_rows;
} tga_tune_entry_t;

/* Replace the process-wide table (count = 0 clears it).  It applies to
 * solutions set up afterwards (tga_set_solution) and to tga_solution_set_rows
 * with 0 arguments.  TGA_EINVAL for malformed entries.  Thread-safe. */
int tga_set_tuning(const tga_tune_entry_t *entries, int32_t count);

/* Set the schedule of one solution explicitly (an autotuner trying
 * candidates): plain_rows / item_rows as in tga_tune_entry_t, 0 = the table's
 * value or the built-in rule.  Not for a batch member.  Synchronises
 * `stream`. */
int tga_solution_set_rows(tga_solution_t sol, int32_t plain_rows, int32_t item_rows, void *stream);

/* The schedule a solution uses (plain_rows after the LDS cap; item_rows 0 =
 * the built-in rule). */
int tga_solution_get_rows(tga_solution_t sol, int32_t *plain_rows, int32_t *item_rows);

/* |N(S)| per operator for the current solution (5 entries, host). */
int tga_move_counts(tga_solution_t sol, int64_t counts[5], void *stream);

/* Current version counter of a solution (number of applied moves). */
uint32_t tga_solution_version(tga_solution_t sol);

int tga_free_solution(tga_solution_t sol);
int tga_free_instance(tga_instance_t inst);
const char *tga_last_error(void);

/* Compute units of the current device and the LDS bytes one evaluation
 * workgroup may use (which bounds n: a workgroup stages at least three
 * distance rows of 4(n+1) bytes). */
int tga_device_limits(int32_t *compute_units, int32_t *max_lds_bytes);

/* ---------------------------------------------------------------- batch --
 * Many independent solutions (instances of different sizes, CVRP and VRPTW
 * mixed) evaluated in one persistent launch per step; the step loop is
 * captured once into a HIP graph and replayed.  A solution may belong to at
 * most one batch and must not be used through the single-solution calls
 * while the batch exists. */

/* Device workspace bytes for a batch of `count` solutions (enough for every
 * schedule a batch can be given). */
size_t tga_batch_workspace_bytes(const tga_solution_t *sols, int32_t count);

/* Schedule of a batch; none of it changes a result.
 *   lds_kb         LDS budget of an inter-route workgroup, KiB (8..160): it
 *                  sets how many distance-matrix rows one strip stages (at
 *                  most 64), per solution.
 *   split          0: inter- and intra-route phases in one launch (the
 *                  intra-route groups fill the tail); 1: two launches.
 *   rows_per_item, sub_rows  as for tga_batch_create.
 *   us_per_eval    written by tga_batch_autotune: measured microseconds per
 *                  evaluation step of the chosen schedule; ignored on input. */
typedef struct {
    int32_t lds_kb, split, rows_per_item, sub_rows;
    float us_per_eval;
} tga_batch_config_t;

/* rows_per_item: slot rows per inter-route work item (0 = one LDS sub-block);
 * sub_rows: rows staged in LDS at a time (0 = as many as the LDS budget of a
 * workgroup holds for the solution's n; larger values are clamped to it).
 * Both only change the schedule, never a result.  The batch starts with
 * lds_kb = 64 (or TGA_LDS_KB) and split = 0. */
int tga_batch_create(const tga_solution_t *sols, int32_t count, int32_t rows_per_item,
                     int32_t sub_rows, void *ws, size_t ws_bytes, void *stream,
                     tga_batch_t *out);

/* Run `steps` local-search steps on every solution of the batch (solutions
 * already at a local optimum skip their work).  use_graph != 0 captures the
 * step loop into a HIP graph on first use and replays it.  Per solution
 * (host arrays of `count`, nullable): accepted moves, moves evaluated, cost. */
int tga_batch_ls_run(tga_batch_t b, uint32_t op_mask, int32_t steps, int32_t use_graph,
                     int32_t *steps_done, int64_t *moves_evaluated, int64_t *cost,
                     void *stream);

/* The screening counters of tga_solution_screen_stats summed over the
 * batch's solutions.  Synchronises `stream`. */
int tga_batch_screen_stats(tga_batch_t batch, int64_t pairs[2], void *stream);

/* The same loop driven by the caller, one step at a time, so that events or
 * other work can sit between the two launches of a step.
 * tga_batch_begin: clear converged flags and counters, set the step cap.
 * tga_batch_step_part: part 0 launches the evaluation of every solution (one
 *   persistent launch), part 1 the finalize launch (best move, apply when its
 *   delta is negative and the cap allows, rebuild).  Asynchronous.
 * tga_batch_collect: synchronise and read the per-solution results, as
 *   tga_batch_ls_run does. */
int tga_batch_begin(tga_batch_t b, int32_t max_steps, void *stream);
int tga_batch_step_part(tga_batch_t b, uint32_t op_mask, int32_t part, void *stream);
int tga_batch_collect(tga_batch_t b, int32_t *steps_done, int64_t *moves_evaluated, int64_t *cost,
                      void *stream);

/* Converged flags of every solution of the batch (host array of `count`),
 * gathered on the device and copied in one transfer.  Synchronises. */
int tga_batch_poll(tga_batch_t b, int32_t *done, void *stream);

/* One evaluation of every solution in the batch (no apply), converged ones
 * included; best moves to a host array of `count` records; per-solution
 * status to status (nullable).  Converged flags and step counters are left
 * as they are. */
int tga_batch_eval(tga_batch_t b, uint32_t op_mask, tga_move_t *best, int32_t *status,
                   void *stream);

/* Clear the per-solution "converged" flags and step counters. */
int tga_batch_reset(tga_batch_t b, void *stream);

/* The batch's current schedule. */
int tga_batch_get_config(tga_batch_t b, tga_batch_config_t *out);

/* Re-plan the batch for `cfg` (TGA_ERANGE if it does not fit the device;
 * the batch keeps its schedule then).  Drops a captured step loop.
 * Synchronises `stream`. */
int tga_batch_set_config(tga_batch_t b, const tga_batch_config_t *cfg, void *stream);

/* The project's autotuner for the batched form: times `launches` evaluation
 * steps (each followed by a finalize that only records the best move, so no
 * solution changes) of the batch's current state under each candidate
 * schedule (lds_kb in {40, 52, 64, 78, 79, the whole LDS} x split in {0, 1}, keeping
 * rows_per_item and sub_rows), keeps the fastest and writes it to `best`
 * (nullable).  Drops a captured step loop.  Synchronises `stream`. */
int tga_batch_autotune(tga_batch_t b, uint32_t op_mask, int32_t launches, tga_batch_config_t *best,
                       void *stream);

/* ------------------------------------------------------- slot batches --
 * Served form (continuous batching): a batch with a fixed number of slots
 * whose members change while it runs.  Each member steps on its own until a
 * local optimum or the step cap set by tga_solution_begin; a converged
 * member costs nothing and can be replaced.  Membership changes and ticks
 * are asynchronous: nothing here waits for the device, except that the host
 * never runs more than two ticks (and two plan uploads) ahead of it.  The
 * launch shapes, and so a captured tick, stay valid across membership
 * changes.  Every batch call above also accepts a slot batch (empty slots
 * are skipped: converged, no move, zero counters). */

/* Device workspace bytes for `slots` slots whose members together hold at
 * most max_sum_q refs (sum of n + R) and max_sum_r routes.  0 if out of
 * range (1 <= slots <= 1024). */
size_t tga_batch_slots_workspace_bytes(int32_t slots, int32_t max_sum_q, int32_t max_sum_r);

/* An empty slot batch; allocates two pinned staging buffers and two pinned
 * result buffers (host).  Same ownership rules as tga_batch_create. */
int tga_batch_create_slots(int32_t slots, int32_t max_sum_q, int32_t max_sum_r, void *ws,
                           size_t ws_bytes, void *stream, tga_batch_t *out);

/* Replace the membership: sols holds one entry per slot (NULL = empty).  A
 * solution keeps its slot for as long as it is a member; a new member needs
 * tga_solution_begin (on the same stream, before its first tick) and must
 * not belong to another batch.  The new plan is uploaded on `stream` and
 * takes effect for the ticks enqueued after this call; ticks already
 * enqueued still use the old members, so a removed solution's memory may be
 * reused only once those have finished (e.g. after an event recorded on
 * `stream` after this call).  TGA_ERANGE when the members exceed the sizes
 * the batch was created for. */
int tga_batch_set_members(tga_batch_t b, const tga_solution_t *sols, void *stream);

/* Enqueue one tick: `steps` (1..64) local-search steps of every member (the
 * step loop captured once per (steps, op_mask) and replayed), then the
 * per-slot results are copied into a pinned buffer.  *tick (nullable) = the
 * tick's number (0, 1, ...).  Blocks only while two earlier ticks are still
 * running. */
int tga_batch_tick(tga_batch_t b, uint32_t op_mask, int32_t steps, int32_t *tick, void *stream);

/* Per-slot results of the newest finished tick, without waiting: *tick = its
 * number, or -1 when none has finished (the arrays are then untouched).
 * Host arrays of `slots` entries (nullable): converged flag, accepted moves,
 * moves evaluated, cost.  A slot's entry describes the member it had when
 * that tick was enqueued. */
int tga_batch_tick_status(tga_batch_t b, int32_t *tick, int32_t *converged, int32_t *steps_done,
                          int64_t *moves_evaluated, int64_t *cost);

int tga_batch_free(tga_batch_t b);

#ifdef __cplusplus
}
#endif

#endif /* TGA_H */
