/*
 * ddm.h -- C ABI of libddm, an MI355X (gfx950) implementation of Interval
 * Tree Matching for Data Distribution Management.
 *
 * Method: Marzolla, D'Angelo, Mandrioli, "A Parallel Data Distribution
 * Management Algorithm", DS-RT 2013.  Given subscription extents S and
 * update extents U (d-dimensional boxes), the library returns the exact set
 * of intersecting (update, subscription) pairs (Sec. III, problem
 * statement), computed the way the paper's ITM does it: one interval tree per
 * dimension built over S (Sec. IV), every update queried against it in
 * parallel (Algorithm 4 / Algorithm 5, "Parallelizing ITM"), and the
 * per-dimension overlaps combined into d-rectangle overlaps (Sec. III-A).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Coordinates are float32, dimension-major (structure of arrays):
 *    lo[k * count + i], hi[k * count + i] for dimension k < d, element i.
 *  - Segments are CLOSED: [lo, hi] and [lo', hi'] meet iff lo <= hi' and
 *    lo' <= hi (the text's [low, high] segments; Algorithm 1 prints the strict
 *    form).  Two boxes meet iff they meet in every dimension.  -0.0 == +0.0.
 *  - Ids are the 0-based array index (the paper counts from 1).
 *  - A result pair is the 64-bit key (update_id << 32) | subscription_id.
 *    Results are returned sorted ascending, i.e. (update, subscription)
 *    lexicographic: the nonzeros of the paper's n x m intersection matrix M,
 *    column by column.
 *  - "device pointer" means memory allocated on the GPU the stream belongs to
 *    (for instance a torch tensor's data_ptr()).  "host pointer" means
 *    ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it in stream order; an entry point returns before
 *    the enqueued work finishes unless stated otherwise.
 *  - Invalid input (NaN or +-inf anywhere, or lo > hi) makes the call that
 *    detects it return DDM_E_INVALID_INPUT.  Points (lo == hi) are valid.
 *  - No C++ exception crosses this boundary.  On error, a thread-local detail
 *    message is available from ddm_last_error_detail().
 *  - Ownership: the caller owns all inputs and outputs; the library owns the
 *    trees and predictors it creates and frees them in the matching *_free.
 */
#ifndef DDM_H_
#define DDM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDM_MAX_D 4

typedef enum {
  DDM_OK = 0,
  DDM_E_INVALID_ARG = -1,   /* bad pointer, size, dimension or option      */
  DDM_E_INVALID_INPUT = -2, /* NaN/inf coordinate or lo > hi                */
  DDM_E_CAPACITY = -3,      /* result does not fit the caller's buffer      */
  DDM_E_NOMEM = -4,         /* device or pinned host allocation failed      */
  DDM_E_DEVICE = -5         /* HIP runtime error                            */
} ddm_status;

typedef struct ddm_tree ddm_tree;

/* ddm_build -- interval trees over the subscription set (Sec. IV,
 * Interval-Tree-Create in Algorithm 5; Sec. III-A for one tree per dimension).
 *
 *  sub_lo, sub_hi  device pointers, d*n float32 each, dimension-major.
 *  n               number of subscriptions; 0 is valid (every match is empty).
 *  d               dimensions, 1..DDM_MAX_D.
 *  stream          HIP stream the build is enqueued on.
 *  out_tree        host pointer; receives an opaque handle.
 *
 * The trees are flat, implicit and balanced: subscriptions sorted by lower
 * bound (a device radix sort; equal lower bounds keep id order) form the
 * in-order sequence of a complete binary tree, and each position stores the
 * maximum upper bound of its subtree (the paper's maxupper; minlower is the
 * leftmost lower bound of the subtree and needs no storage).  The tree owns
 * its device memory.  The inputs may be freed or overwritten once the stream
 * has passed this call.  Validation of the coordinates runs on the device;
 * its outcome is reported by the first ddm_match on the tree (or by
 * ddm_tree_check), not by ddm_build.
 */
ddm_status ddm_build(const float* sub_lo, const float* sub_hi, uint32_t n, uint32_t d,
                     void* stream, ddm_tree** out_tree);

/* ddm_match -- all (update, subscription) pairs that intersect
 * (Algorithm 5: one Interval-Query, Algorithm 4, per update, run in
 * parallel; Sec. III-A: overlap in every dimension).
 *
 *  t              tree from ddm_build (read only; may be matched concurrently
 *                 on several streams).
 *  upd_lo/upd_hi  device pointers, d*m float32 each, dimension-major, d = the
 *                 tree's d.
 *  m              number of updates; 0 is valid.
 *  out_pairs      device pointer to `capacity` uint64 slots; may be NULL when
 *                 capacity is 0.
 *  out_count      host pointer; ALWAYS receives the exact pair count K when
 *                 the call returns DDM_OK or DDM_E_CAPACITY.
 *
 * Synchronizes the stream once (to read K).  If K > capacity the call returns
 * DDM_E_CAPACITY and writes no pair; call again with capacity >= K.  On
 * DDM_OK the first K slots receive the sorted keys when the stream reaches
 * the end of the enqueued work.
 */
ddm_status ddm_match(const ddm_tree* t, const float* upd_lo, const float* upd_hi, uint32_t m,
                     uint64_t* out_pairs, uint64_t capacity, uint64_t* out_count,
                     void* stream);

/* Traversal kernels selectable through ddm_match_ex (results never differ):
 *  DDM_TRAVERSE_LANE  one GPU lane per update, stackless form of Algorithm 4
 *                     on the implicit tree.
 *  DDM_TRAVERSE_TILE  one wavefront per 64 updates sorted by lower bound:
 *                     Algorithm 4 runs once on the tile's enclosing interval,
 *                     candidates are compacted into LDS with wavefront
 *                     ballots and tested against all 64 updates.
 *  DDM_TRAVERSE_AUTO  library default (currently TILE).                     */
#define DDM_TRAVERSE_AUTO 0u
#define DDM_TRAVERSE_LANE 1u
#define DDM_TRAVERSE_TILE 2u

typedef struct {
  uint32_t traversal;   /* DDM_TRAVERSE_*                                     */
  uint32_t block;       /* threads per workgroup of the traversal kernels:
                           64, 128, 256, 512 or 1024; 0 = default (256)       */
  uint32_t reserved[6]; /* must be zero                                       */
} ddm_match_opts;

/* ddm_match with explicit kernel options (opts may be NULL = defaults). */
ddm_status ddm_match_ex(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                        uint32_t m, uint64_t* out_pairs, uint64_t capacity,
                        uint64_t* out_count, void* stream, const ddm_match_opts* opts);

/* Two-step form of ddm_match_ex for callers that size the output from K.
 *
 * ddm_match_begin runs everything up to the pair count (validation, probe
 * dimension, counts per update, offsets), synchronizes the stream once, and
 * returns K through out_count (host pointer) plus a pending handle (host
 * pointer receives it; NULL when m == 0 or n == 0, and ddm_match_finish
 * accepts NULL).  A non-NULL handle must be passed to ddm_match_finish or
 * ddm_match_abort exactly once.  It keeps the device state of the count; the
 * update coordinates must stay valid until ddm_match_finish.  For d > 1 the
 * count also keeps the hits it finds, 12 bytes each, in scratch with room
 * for 4 hits per update plus six 64-hit chunks per possible work tile
 * (m/64 + min(m, 32768) tiles): if all of them fit, ddm_match_finish places
 * them instead of running the traversal again.  ddm_match_ex sizes this
 * scratch for its capacity instead, and keeps no hits when the capacity
 * exceeds 8 hits per update or 2^28 hits.  Results never depend on it.
 *
 * ddm_match_finish writes the K sorted pairs into out_pairs (device, capacity
 * slots) on the stream given to ddm_match_begin, and releases the handle in
 * every case (also on error).  Returns DDM_E_CAPACITY, writing nothing, if
 * capacity < K.  ddm_match_abort releases a handle without writing.       */
typedef struct ddm_pending ddm_pending;
ddm_status ddm_match_begin(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                           uint32_t m, uint64_t* out_count, void* stream,
                           const ddm_match_opts* opts, ddm_pending** out_pending);
ddm_status ddm_match_finish(ddm_pending* pending, uint64_t* out_pairs, uint64_t capacity);
void ddm_match_abort(ddm_pending* pending);

/* ------------------------------------------------------------------------
 * Learned output sizing (an addition to the paper's method).
 *
 * A small MLP (DDM_FEATURES = 18 inputs -> 64 -> 64 -> 1, ReLU, FP32)
 * predicts y = log1p(number of subscriptions an update meets).  The single-
 * pass matcher gives update j ceil(expm1(yhat_j + delta)) output slots, runs
 * ONE traversal that writes hits into the slots while counting every hit
 * exactly, and sends the updates whose hits exceeded their slots through the
 * plain fill afterwards.  The pairs are exactly those of ddm_match, byte for
 * byte, whatever the network predicts; only the work changes.
 *
 * Parameter layout (DDM_PREDICTOR_PARAMS = 5441 floats, row-major W[out][in]):
 *   W1[64][18], b1[64], W2[64][64], b2[64], w3[64], b3.
 *
 * Features of update j (dimension k < 3, zero for k >= d), with mn_k, W_k
 * the smallest lower bound and the width (largest upper - smallest lower) of
 * the subscriptions in dimension k, and c_k an estimate of how many
 * subscriptions meet j in dimension k from 64-bin prefix histograms of the
 * subscription lower and upper bounds (linear inside a bin):
 *   x[5k+0] = (hi - lo) / W_k          x[5k+1] = ((lo + hi)/2 - mn_k) / W_k
 *   x[5k+2] = c_k / n                  x[5k+3] = log1p(c_k) / 16
 *   x[5k+4] = mean subscription length in k / W_k
 *   x[15] = log2(n) / 20   x[16] = d / 3   x[17] = log1p(e) / 16,
 * where e estimates how many subscriptions have their lower corner in the
 * box prod_k [lo_k - l_k, hi_k] (l_k = mean subscription length in k), from
 * a grid over the subscriptions' bounding box (256, 64x64 or 16x16x16 cells
 * for d = 1, 2, 3) that counts lower corners per cell, corners taken as
 * spread evenly inside a cell.
 * ---------------------------------------------------------------------- */
#define DDM_FEATURES 18
#define DDM_PREDICTOR_PARAMS 5441

typedef struct ddm_predictor ddm_predictor;

/* New predictor on the current device; weights and biases of each layer
 * drawn uniformly in +-1/sqrt(fan_in) from a counter-based generator seeded
 * by `seed`; Adam state zero; delta = 0.  Synchronizes the device.          */
ddm_status ddm_predictor_create(uint64_t seed, ddm_predictor** out);
void ddm_predictor_free(ddm_predictor* p);

/* Copy parameters to / from host memory (count must be 0 or
 * DDM_PREDICTOR_PARAMS; 0 only reads/writes delta).  delta (host pointer for
 * get, value for set) is the margin added to the prediction before sizing. */
ddm_status ddm_predictor_get_params(const ddm_predictor* p, float* host, uint32_t count,
                                    float* delta);
ddm_status ddm_predictor_set_params(ddm_predictor* p, const float* host, uint32_t count,
                                    float delta);

/* The predictor's parameters and delta (not its Adam state) to / from a
 * file (host path): four little-endian 32-bit words -- "DDMP", format
 * version 1, DDM_PREDICTOR_PARAMS, delta's float bits -- then the
 * parameters as little-endian floats.  ddm_predictor_load creates a new
 * predictor on the current device (Adam state zero; free it with
 * ddm_predictor_free).  DDM_E_INVALID_ARG for a NULL argument or a file
 * that cannot be opened, read or written; DDM_E_INVALID_INPUT for a file
 * of another format, version or size, or with non-finite values.           */
ddm_status ddm_predictor_save(const ddm_predictor* p, const char* path);
ddm_status ddm_predictor_load(const char* path, ddm_predictor** out);

/* ddm_tree_prepare_learned -- enqueue on `stream` the tree's statistics
 * that the features read (the 64-bin prefix histograms of the subscription
 * bounds and the lower-corner grid above).  Optional: the first learned
 * match or ddm_features on a tree computes them otherwise, on its own
 * stream, and a plain match never needs them, so a build does not pay for
 * them.  Call it right after ddm_build (same stream) to move that cost out
 * of the first learned match; later users on other streams wait for it.
 * Idempotent; an update of the tree (ddm_tree_update) discards them.
 * DDM_E_INVALID_ARG: t NULL, d > 3, or n = 0 (no features are defined).     */
ddm_status ddm_tree_prepare_learned(const ddm_tree* t, void* stream);

/* Features of m updates against tree t (d <= 3, n > 0): X is a device
 * pointer to m*DDM_FEATURES floats, row j = update j.                        */
ddm_status ddm_features(const ddm_tree* t, const float* upd_lo, const float* upd_hi, uint32_t m,
                        float* X, void* stream);

/* yhat[s] (device, N floats) = network output for row s of X (device).      */
ddm_status ddm_predictor_forward(const ddm_predictor* p, const float* X, uint32_t N, float* yhat,
                                 void* stream);

/* Gradient of the mean squared error (1/N) sum_s (yhat_s - Y_s)^2 with
 * respect to the parameters: grad (device, DDM_PREDICTOR_PARAMS floats),
 * loss (device, one float, may be NULL).  Partial sums are reduced in a fixed
 * order, so the result is deterministic.                                    */
ddm_status ddm_predictor_grad(const ddm_predictor* p, const float* X, const float* Y, uint32_t N,
                              float* grad, float* loss, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * device gradient `grad` and learning rate lr.                              */
ddm_status ddm_predictor_adam(ddm_predictor* p, const float* grad, float lr, void* stream);

/* `epochs` passes of minibatch Adam over (X, Y) (device, N rows), batches of
 * `batch` consecutive rows.  epoch_loss (host, epochs floats, may be NULL)
 * receives the mean batch loss of each epoch; it synchronizes the stream.   */
ddm_status ddm_predictor_train(ddm_predictor* p, const float* X, const float* Y, uint32_t N,
                               uint32_t batch, uint32_t epochs, float lr, void* stream,
                               float* epoch_loss);

/* Single-pass form of ddm_match_begin (d <= 3; for d = 1 the counts are exact
 * without any traversal, so it is the plain path).  slot_budget > 0 fixes
 * the slot arena (updates whose slots fall beyond it are treated as
 * overflowed); 0 sizes the arena to the predicted total, at the cost of one
 * more stream synchronization.  Finish with ddm_match_finish.               */
ddm_status ddm_match_learned_begin(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                                   uint32_t m, const ddm_predictor* pred, uint64_t slot_budget,
                                   uint64_t* out_count, void* stream, const ddm_match_opts* opts,
                                   ddm_pending** out_pending);

/* Sizing outcome of a pending single-pass match (host pointers, may be
 * NULL): slots reserved by the predictions, the arena size, and the number
 * of updates that overflowed their slots (0 for a plain pending match).     */
ddm_status ddm_pending_info(const ddm_pending* pending, uint64_t* slots, uint64_t* budget,
                            uint32_t* overflowed);

/* ddm_count -- exact number of subscriptions each update meets (the length
 * of column j of M), without producing the pairs.
 *  counts     device pointer to m uint32 (caller owned).
 *  out_total  host pointer, receives K = sum of counts (may be NULL).
 * Synchronizes the stream once.                                             */
ddm_status ddm_count(const ddm_tree* t, const float* upd_lo, const float* upd_hi, uint32_t m,
                     uint32_t* counts, uint64_t* out_total, void* stream,
                     const ddm_match_opts* opts);

/* ddm_match_scratch_bytes -- device scratch, in bytes, that a match of m
 * updates against a d-dimensional tree set takes, for a given form:
 *  form       DDM_SCRATCH_PLAIN    count -> scan -> fill (what a match
 *                                  carved from fixed memory takes; a result
 *                                  with more than 2^20 subscriptions and a
 *                                  segment over 2048 pairs also takes 4
 *                                  bytes per pair for its segment sort),
 *             DDM_SCRATCH_STASH    plus the count traversal's stash of hits
 *                                  (d > 1; hint = the caller's capacity, 0 =
 *                                  the default of 4 hits per update),
 *             DDM_SCRATCH_LEARNED  the single pass (d > 1) without its slot
 *                                  arena (4 bytes per predicted slot).
 *  bytes      host pointer, receives the size (0 for m = 0).
 * Computed on the host by the same layout code the match runs, with no GPU
 * and no memory behind it; it also checks that every piece the match takes
 * lies inside what it reserves (DDM_E_DEVICE if not: a defect of the
 * library).  DDM_E_INVALID_ARG for d outside [1, DDM_MAX_D], an unknown
 * form, m >= 2^31 or a NULL `bytes`.                                        */
#define DDM_SCRATCH_PLAIN 0u
#define DDM_SCRATCH_STASH 1u
#define DDM_SCRATCH_LEARNED 2u
ddm_status ddm_match_scratch_bytes(uint32_t m, uint32_t d, uint32_t form, uint64_t hint,
                                   uint64_t* bytes);

/* ddm_match_noalloc -- ddm_match for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, result and errors as ddm_match; it
 * runs the plain count -> scan -> fill path (no stash of hits) and takes all
 * its scratch from one static device array of DDM_NOALLOC_SCRATCH_MB MiB,
 * which each device that runs it keeps until the process ends.  It calls no
 * allocator of any kind (the count is read back into pageable host memory).
 *  Limit: the match takes about 45 bytes per update plus 4.4 MiB
 *  (ddm_match_scratch_bytes with DDM_SCRATCH_PLAIN gives the exact figure),
 *  i.e. up to about 1.38e6 updates; beyond that, and for a result that needs
 *  the segment sort's id copy (more than 2^20 subscriptions and a segment
 *  over 2048 pairs: 4 bytes per pair) beyond what is left, it returns
 *  DDM_E_INVALID_ARG with a detail message, before writing anything.
 *  Concurrency: every call on one device shares that device's array, so
 *  calls that overlap on one device (different streams or threads) race;
 *  the caller serializes them.  Each call sets all the state it reads, so
 *  nothing carries over from the previous call.                            */
#define DDM_NOALLOC_SCRATCH_MB 64
ddm_status ddm_match_noalloc(const ddm_tree* t, const float* upd_lo, const float* upd_hi,
                             uint32_t m, uint64_t* out_pairs, uint64_t capacity,
                             uint64_t* out_count, void* stream);

/* ddm_match_brute -- the same result as ddm_build + ddm_match, computed by
 * Brute-Force Matching (Algorithm 2: every update tested against every
 * subscription, closed predicate in every dimension).  The paper's
 * embarrassingly parallel baseline, for comparison on the same GPU.
 *  sub_lo/sub_hi  device, d*n float32, dimension-major; upd_lo/upd_hi
 *                 device, d*m float32; out_pairs device, capacity uint64
 *                 (may be NULL when capacity is 0); out_count host, always
 *                 receives K on DDM_OK / DDM_E_CAPACITY.
 * Synchronizes the stream once; DDM_E_CAPACITY writes nothing; invalid
 * coordinates give DDM_E_INVALID_INPUT.  Cost O(n m d).                     */
ddm_status ddm_match_brute(const float* sub_lo, const float* sub_hi, uint32_t n,
                           const float* upd_lo, const float* upd_hi, uint32_t m, uint32_t d,
                           uint64_t* out_pairs, uint64_t capacity, uint64_t* out_count,
                           void* stream);

/* ddm_match_sbm -- the same result as ddm_build + ddm_match, computed by
 * Sort-Based Matching (Algorithm 3, Sec. III-D): the endpoints of dimension
 * 0 are sorted and swept; the sweep is cut into segments of 64 subscription
 * lower endpoints whose starting sets of active subscriptions are formed
 * from a prefix, and every update resumes the sweep at its segment's start.
 * The other dimensions are tested on every pair the sweep reports (the
 * combine of Sec. III-A).  The paper's sweep-line comparison system, for
 * comparison on the same GPU.
 *  Arguments, ownership and errors as for ddm_match_brute; n, m < 2^31.
 * Synchronizes the stream twice.  Cost O((n + m) log(n + m)) for the sorts
 * plus, per update, the subscriptions active at its segment's start and the
 * lower endpoints between that start and its upper endpoint.                */
ddm_status ddm_match_sbm(const float* sub_lo, const float* sub_hi, uint32_t n,
                         const float* upd_lo, const float* upd_hi, uint32_t m, uint32_t d,
                         uint64_t* out_pairs, uint64_t capacity, uint64_t* out_count,
                         void* stream);

/* ddm_match_sets -- the result of ddm_build(S) + ddm_match(U) for two sets
 * given together, with the tree built on the smaller set.  Sec. IV assumes
 * n <= m without loss of generality, swapping the roles of S and U
 * otherwise: when swapped, the tree is built on the updates, queried with
 * the subscriptions, and the keys are transposed back on the device (a
 * stable radix sort by update id), so the output is bit-identical to the
 * unswapped one.
 *  sub_lo/sub_hi  device, d*n float32, dimension-major; upd_lo/upd_hi
 *                 device, d*m float32.
 *  swap_policy    DDM_SWAP_AUTO (swap when n > m and d >= 3), DDM_SWAP_NEVER
 *                 or DDM_SWAP_ALWAYS.  AUTO follows measurements on the
 *                 GPU: for d <= 2 the tree on the larger set is as fast or
 *                 faster (per-update work and the transposition outweigh
 *                 the smaller tree), for d >= 3 the tree on the smaller set
 *                 is 1.5x to 11x faster.  A swap transposes on the device
 *                 and needs capacity < 2^32: AUTO does not swap beyond it,
 *                 ALWAYS returns DDM_E_INVALID_ARG.
 *  out_pairs      device, capacity uint64 (may be NULL when capacity is 0).
 *  out_count      host, receives K on DDM_OK / DDM_E_CAPACITY.
 *  out_swapped    host, may be NULL: 1 if the tree was built on the updates.
 * The tree is freed before return.  Synchronizes the stream once (to read
 * K).  DDM_E_CAPACITY writes nothing; invalid coordinates of either set give
 * DDM_E_INVALID_INPUT.  A swap needs 16 bytes of scratch per pair.          */
#define DDM_SWAP_AUTO 0
#define DDM_SWAP_NEVER 1
#define DDM_SWAP_ALWAYS 2
ddm_status ddm_match_sets(const float* sub_lo, const float* sub_hi, uint32_t n,
                          const float* upd_lo, const float* upd_hi, uint32_t m, uint32_t d,
                          int swap_policy, uint64_t* out_pairs, uint64_t capacity,
                          uint64_t* out_count, int* out_swapped, void* stream);

/* ddm_tree_update -- moves `count` subscriptions of a resident tree to new
 * extents (dynamic DDM: extents move between matches, Sec. I, Sec. VI), so
 * that later matches see the moved set without a new ddm_build.
 *  ids            device, count distinct uint32 subscription ids (< n).
 *  new_lo/new_hi  device, [d][count] float32, dimension-major: the new
 *                 extent of subscription ids[c] is column c.
 *  out_rebuilt    host, may be NULL: 0 if every tree kept its (lower bound,
 *                 id) order and was refitted in place (records rewritten,
 *                 maxupper and the search samples recomputed, no sort), 1 if
 *                 the order changed and the tree was rebuilt from its own
 *                 records with the moves applied.
 * Synchronizes the stream once.  DDM_E_INVALID_INPUT (tree unchanged) for
 * an id out of range or an invalid new extent.  The caller must make sure
 * that no match on another stream reads the tree meanwhile.               */
ddm_status ddm_tree_update(ddm_tree* t, const uint32_t* ids, const float* new_lo,
                           const float* new_hi, uint32_t count, void* stream, int* out_rebuilt);

/* ---------------------------------------------------------------------------
 * Dynamic DDM (the paper's dynamic scenario, Sec. IV and Sec. VI): both
 * extent sets, an interval tree over each (T_S over the subscriptions, T_U
 * over the updates) and the current result stay resident on the device;
 * moving extents recomputes only the moved extents' pairs.
 *
 * ddm_dynamic_create -- copies S (n extents) and U (m extents), device,
 *   [d][count] float32 dimension-major, builds both trees and matches
 *   everything once.  Synchronizes the stream.  DDM_E_INVALID_INPUT for a
 *   NaN/inf coordinate or lo > hi in either set.
 * ddm_dynamic_move -- moves `count` extents of one set (set =
 *   DDM_DYNAMIC_SUBSCRIPTIONS or DDM_DYNAMIC_UPDATES) to new extents:
 *   ids device uint32 (distinct, below the set's size), new_lo/new_hi
 *   device [d][count] float32 (column c is the new extent of ids[c]).  The
 *   moved set's tree is refitted or rebuilt (as ddm_tree_update); a moved
 *   update's column of M is recomputed with one query of T_S, a moved
 *   subscription's row with one query of T_U; the resident result drops the
 *   moved ids' old pairs and merges the new ones.  out_count (host, may be
 *   NULL) receives the new K.  Synchronizes the stream a few times.  On
 *   DDM_E_INVALID_INPUT (id out of range or repeated, invalid extent)
 *   nothing changes.  K must stay below 2^32.
 * ddm_dynamic_result -- the current pairs (device pointer, sorted
 *   (update << 32) | subscription keys, valid until the next move or free)
 *   and their number (host pointers).
 * ddm_dynamic_free -- releases everything.                                  */
typedef struct ddm_dynamic ddm_dynamic;
#define DDM_DYNAMIC_SUBSCRIPTIONS 0u
#define DDM_DYNAMIC_UPDATES 1u
ddm_status ddm_dynamic_create(const float* sub_lo, const float* sub_hi, uint32_t n,
                              const float* upd_lo, const float* upd_hi, uint32_t m, uint32_t d,
                              void* stream, ddm_dynamic** out);
ddm_status ddm_dynamic_move(ddm_dynamic* dy, uint32_t set, const uint32_t* ids,
                            const float* new_lo, const float* new_hi, uint32_t count,
                            void* stream, uint64_t* out_count);
ddm_status ddm_dynamic_result(const ddm_dynamic* dy, const uint64_t** pairs, uint64_t* count);
void ddm_dynamic_free(ddm_dynamic* dy);

/* ddm_tree_check -- waits for the build to finish and reports whether the
 * subscription coordinates were valid (DDM_OK or DDM_E_INVALID_INPUT).      */
ddm_status ddm_tree_check(const ddm_tree* t);

/* ddm_tree_info -- host pointers receive n, d and the tree height H (the
 * implicit tree has 2^H - 1 positions, H = 0 for n = 0). Any may be NULL.   */
ddm_status ddm_tree_info(const ddm_tree* t, uint32_t* n, uint32_t* d, uint32_t* height);

/* ddm_tree_export -- copies dimension k's tree to host memory (synchronous),
 * for inspection and tests.  Host pointers, each may be NULL:
 *  lo, hi   n floats: the in-order (sorted by lower bound) segments;
 *  ids      n uint32: subscription id at each in-order position;
 *  maxhi    2^H - 1 floats: maxupper of the subtree rooted at each position
 *           (positions beyond n belong to no subscription).                 */
ddm_status ddm_tree_export(const ddm_tree* t, uint32_t k, float* lo, float* hi,
                           uint32_t* ids, float* maxhi);

/* ddm_tree_free -- releases the tree's device memory, ordered on the stream
 * the tree was built on.  The caller must make sure that work on other
 * streams that reads the tree has finished.  NULL is ignored.               */
void ddm_tree_free(ddm_tree* t);

/* ---------------------------------------------------------------------------
 * Batched matching (an addition to the paper; every instance is the
 * problem of Sec. III, solved as in Algorithm 5 with the trees of Sec. IV).
 *
 * Many independent instances -- each its own subscription set, update set
 * and dimension -- matched by one fixed sequence of kernels: one tree build
 * over all subscription sets, one probe and ordering pass over all updates,
 * a count traversal and a fill traversal over (instance, probe dimension,
 * tile of updates) work items -- one wavefront per item, or with
 * opts.waves_per_cu a persistent grid whose wavefronts take items from an
 * atomic ticket -- one scan and one segment sort.  The sequence allocates
 * nothing and never waits on the host, so it is captured once into a HIP
 * graph and replayed by every ddm_batch_run (opts.use_graph).
 *
 * Output: out_pairs (device, capacity uint64) receives every instance's
 * pairs, instance after instance; instance i owns
 * out_pairs[ranges[i] .. ranges[i+1]) holding keys
 * (update << 32) | subscription with both ids local to instance i, sorted
 * ascending -- the bytes ddm_match returns for that instance alone.
 * --------------------------------------------------------------------------*/
#define DDM_BATCH_MAX_INSTANCES 16383

typedef struct {
  const float* sub_lo;  /* device, [d][n] dimension-major, like ddm_build  */
  const float* sub_hi;
  const float* upd_lo;  /* device, [d][m] dimension-major, like ddm_match  */
  const float* upd_hi;
  uint32_t n;           /* 0 < n < 2^20                                     */
  uint32_t m;           /* m > 0                                            */
  uint32_t d;           /* 1 <= d <= DDM_MAX_D                              */
  uint32_t qpt;         /* updates per traversal work item of this instance:
                           16, 32 or 64; 0 = the batch's opts.qpt          */
} ddm_batch_instance;

typedef struct {
  uint32_t qpt;          /* default updates per traversal work item: 16, 32
                            or 64 (0 = 64)                                  */
  uint32_t waves_per_cu; /* 0: one wavefront per tile of the traversals;
                            1..64: a persistent grid of this many
                            wavefronts per CU taking tiles from a ticket    */
  uint32_t use_graph;    /* nonzero: capture on the first run, then replay  */
  uint32_t reserved[5];  /* must be 0                                       */
} ddm_batch_opts;

typedef struct ddm_batch ddm_batch;

/* ddm_batch_create -- plans a batch on the current device: one device block
 * holds every tree, every intermediate and the work tables (synchronous
 * upload of the tables).  The coordinate arrays are read at every
 * ddm_batch_run, so their contents may change between runs but their
 * addresses and sizes may not.  out_pairs may be NULL when capacity is 0.
 * Errors: DDM_E_INVALID_ARG (count 0 or above DDM_BATCH_MAX_INSTANCES, an
 * instance out of range, bad opts),
 * DDM_E_NOMEM, DDM_E_DEVICE.                                                */
ddm_status ddm_batch_create(const ddm_batch_instance* inst, uint32_t count,
                            uint64_t* out_pairs, uint64_t capacity,
                            const ddm_batch_opts* opts, ddm_batch** out_batch);

/* ddm_batch_run -- enqueues one whole pass on `stream` (graph replay or
 * eager launches); returns without waiting.  Runs of one batch must not
 * overlap in time.                                                           */
ddm_status ddm_batch_run(ddm_batch* b, void* stream);

/* ddm_batch_result -- waits for the last run and reports it: *total
 * receives the number of pairs over all instances, ranges (host, count + 1
 * uint64, may be NULL) the instance offsets -- both also when the result
 * did not fit.  DDM_E_CAPACITY: total > capacity, nothing was written.
 * DDM_E_INVALID_INPUT: an instance has a NaN/inf coordinate or lo > hi;
 * nothing was written.                                                       */
ddm_status ddm_batch_result(ddm_batch* b, uint64_t* total, uint64_t* ranges);

/* Two-step run for batches created without a graph (opts.use_graph = 0),
 * for callers that size the output from the count:
 * ddm_batch_count enqueues everything up to the per-instance offsets on
 * `stream`, waits for it, and returns the total (host) and, if ranges is not
 * NULL, the count + 1 instance offsets (host); DDM_E_INVALID_INPUT if an
 * instance has invalid coordinates.  ddm_batch_fill then writes the pairs
 * into out_pairs (device, capacity uint64; the pointer given at creation is
 * not used) on `stream`; DDM_E_CAPACITY, writing nothing, if capacity is
 * below the total.  Each count is followed by at most one fill.             */
ddm_status ddm_batch_count(ddm_batch* b, void* stream, uint64_t* total, uint64_t* ranges);
ddm_status ddm_batch_fill(ddm_batch* b, uint64_t* out_pairs, uint64_t capacity, void* stream);

/* ddm_batch_free -- waits for the batch's work and releases it; NULL is
 * ignored.                                                                    */
void ddm_batch_free(ddm_batch* b);

/* ---------------------------------------------------------------------------
 * Serving loop (an addition to the paper; every request is the problem of
 * Sec. III, matched as ddm_build + ddm_match / ddm_match_learned_begin do).
 *
 * Requests arrive at any time (ddm_server_submit, thread-safe, returns at
 * once) and are matched concurrently by `workers` host threads, each
 * driving its own HIP stream: a request starts as soon as a worker is free
 * and the device-memory budget admits it, so requests overlap on the device
 * with the ones already running.  Optionally (batch_max > 1) small
 * requests queued together are matched as one batch (the ddm_batch kernels,
 * sized on the device by their exact counts).  Admission is by footprint:
 * inputs + trees + match scratch when a request starts (FIFO order); with
 * learned sizing, the slot arena (4 bytes per predicted slot) plus an
 * output estimate of the same size once the prediction is known and before
 * the arena is allocated; the exact output once known.  A request waits
 * until its bytes fit.  When every request in flight is waiting, the
 * youngest one that has not yet allocated its arena or output gives back
 * everything it holds and goes back to the head of the queue (counted in
 * ddm_server_counters.requeued); only a request alone in flight, or one no
 * waiting request can make room for, goes past the budget, so progress is
 * guaranteed.  With a predictor, requests of d <= 3 use the single-pass
 * learned sizing; results are bit-identical either way.
 *
 * Results are copied into a pinned host pool owned by the server (or stay
 * in device memory with deliver_device) and are announced through a
 * completion queue (ddm_server_wait_any); the caller reads them with
 * ddm_server_result and returns their memory with ddm_server_release.
 * Timestamps are CLOCK_MONOTONIC nanoseconds.
 * --------------------------------------------------------------------------*/
typedef struct {
  uint64_t hbm_budget;     /* device bytes requests in flight may hold
                              (0 = 64 GiB)                                   */
  uint64_t host_pool;      /* pinned host bytes for results (0 = 4 GiB)      */
  uint32_t workers;        /* concurrent requests, 1..64 (0 = 8)             */
  uint32_t tree_cache;     /* keyed trees kept resident after their request
                              (LRU); 0 = none                                */
  uint32_t deliver_device; /* nonzero: results stay in device memory         */
  uint32_t batch_max;      /* up to this many small requests are matched
                              together by one worker (batched kernels);
                              0 or 1 = never batch                          */
  uint32_t batch_small;    /* a request is small if n + m <= batch_small
                              (and n < 2^20, no tree key); 0 = 2^18        */
  uint32_t compact;        /* nonzero: host results as subscription ids
                              (uint32, K) plus update offsets (uint64, m+1)
                              instead of 64-bit keys -- the same pairs in
                              the same order, in about half the bytes       */
  uint32_t reserved[1];    /* must be 0                                      */
} ddm_server_opts;

typedef struct {
  const float* sub_lo;     /* device, [d][n]; may be NULL with a resident
                              tree_key                                        */
  const float* sub_hi;
  const float* upd_lo;     /* device, [d][m]                                  */
  const float* upd_hi;
  uint32_t n, m, d;
  uint32_t reserved;       /* must be 0                                       */
  uint64_t tree_key;       /* nonzero: keep the subscription tree resident
                              under this key / reuse the resident tree        */
} ddm_request;

typedef struct {
  int32_t status;          /* 1 = pending, else the request's ddm_status      */
  uint32_t on_device;      /* pairs is a device pointer                       */
  uint64_t count;          /* K                                               */
  const uint64_t* pairs;   /* K sorted keys, valid until ddm_server_release;
                              NULL for compact results                       */
  int64_t t_arrival_ns;    /* arrival (given to submit, or submit time)       */
  int64_t t_start_ns;      /* admitted onto a worker                          */
  int64_t t_done_ns;       /* result in host (or device) memory               */
  uint64_t slots;          /* learned slot arena of the request (0 if none)   */
  uint32_t overflowed;     /* updates that took the exact fallback            */
  uint32_t m;              /* updates of the request                          */
  const uint32_t* sub_ids;      /* compact results (host): the subscription
                                   of every pair, K entries                  */
  const uint64_t* upd_offsets;  /* compact results (host): update j's pairs
                                   are sub_ids[upd_offsets[j] ..
                                   upd_offsets[j+1]), m + 1 entries          */
} ddm_result;

typedef struct {
  uint64_t submitted, completed, queued, in_flight;
  uint64_t hbm_used, hbm_peak, host_pool_used, trees_resident;
  uint64_t requeued;  /* admissions given back when every request in flight
                         waited for memory (the request started again later) */
} ddm_server_counters;

typedef struct ddm_server ddm_server;

/* Starts the worker threads on the current device.  pred may be NULL (plain
 * two-pass matching); it must outlive the server.                            */
ddm_status ddm_server_create(const ddm_server_opts* opts, ddm_predictor* pred,
                             ddm_server** out);

/* Queues a request.  The coordinate arrays must stay valid until the request
 * completes; the server's streams wait for the work enqueued on `stream`
 * before reading them.  arrival_ns: the request's arrival time (0 = now).   */
ddm_status ddm_server_submit(ddm_server* s, const ddm_request* req, int64_t arrival_ns,
                             void* stream, uint64_t* ticket);

/* Waits up to timeout_ms for completions and moves at most max_tickets
 * completed tickets into `tickets` (host); returns how many.                 */
uint32_t ddm_server_wait_any(ddm_server* s, uint32_t timeout_ms, uint64_t* tickets,
                             uint32_t max_tickets);

/* State and result of a request (host struct).  For a failed request
 * ddm_last_error_detail() holds its detail after this call.                 */
ddm_status ddm_server_result(ddm_server* s, uint64_t ticket, ddm_result* res);

/* Returns a finished request's result memory to the server.                 */
ddm_status ddm_server_release(ddm_server* s, uint64_t ticket);

ddm_status ddm_server_stats(ddm_server* s, ddm_server_counters* out);

/* Waits for queued and running requests, stops the workers and frees
 * everything the server holds (unreleased results included).                */
void ddm_server_destroy(ddm_server* s);

/* Static message for a status code.                                          */
const char* ddm_strerror(ddm_status s);

/* Thread-local detail of the last error returned on this thread ("" if none).*/
const char* ddm_last_error_detail(void);

/* Test hook, for fault injection from the host: caps the device bytes the
 * library's allocator may have handed out at once (blocks in use; freed
 * blocks it keeps cached are not counted), process-wide; 0 lifts the cap.
 * An allocation beyond the cap fails as a failed device allocation does:
 * the call returns DDM_E_NOMEM and frees what it had taken (a server
 * request fails alone with that status).  Returns the bytes in use when
 * called, so that a test can check that a failed call left none behind.
 * Not counted: the predictor's weights and ddm_match_noalloc's static
 * array.                                                                     */
uint64_t ddm_debug_alloc_cap(uint64_t bytes);

/* Kernel timing with HIP events recorded on the launching stream.
 * ddm_prof_enable(1) starts recording every kernel launch of this thread;
 * ddm_prof_read() waits for the recorded events and writes a JSON object
 * {"kernel": [total_ms, launches], ...} into buf (host, size bytes), then
 * clears the records.  Returns the number of bytes needed (excluding NUL). */
void ddm_prof_enable(int on);
uint64_t ddm_prof_read(char* buf, uint64_t size);

/* Restricts recording to launches of the kernel `name` (a key of the JSON
 * report, host string); NULL or "" records every kernel again.              */
void ddm_prof_focus(const char* name);

#ifdef __cplusplus
}
#endif

#endif /* DDM_H_ */
