/*
 * jt.h -- C ABI of the MI355X junction-tree message engine.
 *
 * The engine computes junction-tree belief propagation (Zheng, Mengshoel,
 * Chong, "Belief Propagation by Message Passing in Junction Trees: Computing
 * Each Message Faster Using GPU Parallelization"): every message is the
 * marginalization of a clique table into a separator (eq. (2)), the new/old
 * separator ratio with 0/0 := 0, and the scatter-multiply of that ratio into
 * the neighbouring clique (eq. (3)), driven over the collect and distribute
 * sweeps of Algorithms 2-4.  The cluster-separator index mappings of
 * Sec. 3.1-3.2 are precomputed once, when the tree is compiled.
 *
 * Conventions
 *   - Variables are 0..n_vars-1, variable v has card[v] >= 1 states.
 *   - Clique c lists its variables in clique_vars[clique_off[c] ..
 *     clique_off[c+1]).  The listed order is the table layout: row-major,
 *     last-listed variable fastest.  |phi_X| = product of the cardinalities
 *     (Sec. 3) and must be below 2^31.
 *   - parent[c] is the neighbour towards the root; exactly one clique has
 *     parent -1 (the designated root of Sec. 2.1).  The separator of edge
 *     (c, parent[c]) is the intersection of the two variable sets, ordered by
 *     ascending variable id; separator tables are row-major in that order.
 *   - Potentials are FP32.  Messages are scaled: every new separator table
 *     is rescaled to mean one and the log of the scale is carried in FP64,
 *     so log P(evidence) (more precisely log Z_e, the log of the
 *     evidence-restricted partition function) is exact up to FP32 rounding.
 *   - Evidence is hard: observing variable v in state s zeroes every entry
 *     with x_v != s of the lowest-id clique that contains v.
 *   - n_slots evidence sets ("slots") are propagated together over the same
 *     tree (one query per slot).
 *
 * Memory and threads
 *   - The library never allocates device memory.  jt_compile_index_maps
 *     reports the device workspace size; the caller allocates it (e.g. a
 *     torch uint8 tensor) and hands it to jt_bind.  It must stay valid until
 *     jt_free.  Host arrays passed to any call are copied before it returns.
 *   - A handle is bound to one HIP stream and is not thread-safe.  Distinct
 *     handles are independent.
 *
 * Errors
 *   Every call returns a jt_status: JT_OK (0) or a negative code.  No C++
 *   exception crosses the ABI.  jt_last_error() returns a thread-local
 *   message describing the last failure on the calling thread.
 */
#ifndef JT_H
#define JT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t jt_status;

#define JT_OK 0
#define JT_E_ARG (-1)               /* bad pointer, index, slot, variable or state; conflicting evidence */
#define JT_E_NOT_JUNCTION_TREE (-2) /* not one root, a cycle, or running intersection violated */
#define JT_E_TOO_LARGE (-3)         /* a table with 2^31 or more entries */
#define JT_E_NO_MEM (-4)            /* workspace smaller than required, or host allocation failed */
#define JT_E_HIP (-5)               /* a HIP runtime error (message in jt_last_error) */
#define JT_E_ZERO_EVIDENCE (-6)     /* P(evidence) = 0 for the slot: no posterior exists */
#define JT_E_STATE (-7)             /* call out of order (e.g. propagate before bind) */

/* Propagation schedules (all compute the same messages):
 *   JT_MODE_FUSED  level-scheduled: all cliques of one tree level in one
 *                  launch, marginalize and scatter fused per clique;
 *   JT_MODE_GRAPH  the same launches replayed from one captured HIP graph;
 *   JT_MODE_PLAIN  one message at a time in the paper's depth-first order
 *                  (Algorithms 2-3): marginalize, ratio, scatter launches per
 *                  message, tables updated in place;
 *   JT_MODE_DATAFLOW  reserved for a persistent schedule that overlaps tree
 *                  levels; disabled: jt_propagate and jt_profile return
 *                  JT_E_ARG for it;
 *   JT_MODE_PAPER, JT_MODE_PAPER_GRAPH  the paper's own kernel design (see
 *                  jt_paper_bind).
 * In the first three a message is finalized (new separator table, rescale,
 * ratio, log-scales) inside the pass launch that produces it. */
#define JT_MODE_FUSED 0
#define JT_MODE_GRAPH 1
#define JT_MODE_PLAIN 2
#define JT_MODE_DATAFLOW 3
#define JT_MODE_PAPER 4
#define JT_MODE_PAPER_GRAPH 5

typedef struct jt_tree_s *jt_tree;

/* Shape choices of the fused schedule (all in table entries or blocks; 0
 * selects the built-in default).  They change how the work is cut, never
 * what is computed; results stay within the stated tolerance for every
 * choice and are bit-identical from run to run for a given choice.
 *   group_min, group_max  bounds of a group (the entries one block reduces
 *                         into one partial row), defaults 8192 and 32768;
 *   group_div             a level's entries per slot / group_div is the
 *                         group size before the bounds, default 1024;
 *   target_blocks         blocks per launch aimed for, default 1280 (one
 *                         round of resident blocks);
 *   max_lanes             streams for the root's subtrees (1 = all levels
 *                         on the bound stream); lanes are disabled in this
 *                         version: values above 1 return JT_E_ARG;
 *   task_min              least work of one block (entries, written entries
 *                         counted twice) before it takes a second group,
 *                         default group_min; smaller values spread a small
 *                         launch's groups over more blocks. */
typedef struct {
    int32_t group_min, group_max, group_div, target_blocks, max_lanes, task_min;
} jt_tuning;

typedef struct {
    int32_t n_vars;
    const int32_t *card;        /* [n_vars], each >= 1 */
    int32_t n_cliques;
    const int64_t *clique_off;  /* [n_cliques + 1], clique_off[0] = 0 */
    const int32_t *clique_vars; /* [clique_off[n_cliques]], no repeats within a clique */
    const int32_t *parent;      /* [n_cliques], exactly one -1 */
    int32_t n_slots;            /* evidence sets propagated together, >= 1 */
    const jt_tuning *tuning;    /* NULL: defaults (copied at compile) */
} jt_tree_desc;

/* Validate the tree and precompute every cluster-separator index mapping
 * (Sec. 3.2: the mapping tables are built once, when the junction tree is
 * established).  Host only; touches no GPU.
 *   desc          tree description (host arrays, copied);
 *   out           receives the new handle (caller frees with jt_free);
 *   device_bytes  receives the workspace size jt_bind needs.
 * Errors: JT_E_ARG, JT_E_NOT_JUNCTION_TREE, JT_E_TOO_LARGE, JT_E_NO_MEM. */
jt_status jt_compile_index_maps(const jt_tree_desc *desc, jt_tree *out, size_t *device_bytes);

/* Attach device memory and the initial potentials, and upload the index
 * metadata (Initialization of Algorithm 4 takes the tables from here).
 *   workspace        device pointer, >= device_bytes bytes, 256-byte aligned;
 *   bytes            its size;
 *   init_potentials  device pointer to the FP32 tables concatenated in clique
 *                    order (sum of |phi_X| floats); copied into the
 *                    workspace, so the caller may release it afterwards;
 *   hip_stream       hipStream_t all later work of this handle runs on
 *                    (NULL = the default stream).
 * Enqueues copies on the stream and returns; errors: JT_E_ARG, JT_E_NO_MEM,
 * JT_E_HIP. */
jt_status jt_bind(jt_tree t, void *workspace, size_t bytes, const float *init_potentials,
                  void *hip_stream);

/* Replace the evidence of one slot by n_obs hard observations (Sec. 2.1:
 * evidence is a set of instantiated variables).  n_obs = 0 clears it.
 *   vars, states  host arrays of n_obs entries; a variable may repeat only
 *                 with the same state.
 * Takes effect at the next jt_propagate.  Errors: JT_E_ARG. */
jt_status jt_set_evidence(jt_tree t, int32_t slot, int32_t n_obs, const int32_t *vars,
                          const int32_t *states);

/* Run one full belief propagation for every slot (Algorithm 4): reset
 * every table to the initial potentials with the slot's evidence entered,
 * collect to the root, distribute from it.  Asynchronous on the bound
 * stream; idempotent (always restarts from the initial potentials).
 *   A collect message depends only on the evidence in the subtree it comes
 *   from, so with several active slots the fused schedules compute the
 *   evidence-free collect sweep once (in an extra slot region) and each slot
 *   recomputes only the cliques with some of its evidence below them; the
 *   others read the shared messages.  This is chosen per propagation when it
 *   streams fewer table entries, and every slot's results are bit-identical
 *   either way (and to the same query propagated alone).
 *   mode  JT_MODE_FUSED, JT_MODE_GRAPH, JT_MODE_PLAIN or JT_MODE_DATAFLOW.
 * Errors: JT_E_STATE (not bound), JT_E_ARG (mode), JT_E_HIP (also reported
 * by the next jt_marginal when a dataflow dependency wait gave up). */
jt_status jt_propagate(jt_tree t, int32_t mode);

/* jt_propagate restricted to slots [0, n_active): the other slots are left
 * as they are and their read-out calls return JT_E_STATE until a
 * propagation covers them again.  A serving loop packs the queries of one
 * batch into the first n_active slots.  Errors: as jt_propagate, and JT_E_ARG
 * for n_active outside [1, n_slots]. */
jt_status jt_propagate_n(jt_tree t, int32_t mode, int32_t n_active);

/* Posterior of one clique, P(X_C | e) (Sec. 2.1: marginals are read from the
 * calibrated tables), normalized to sum 1, and log Z_e.  Synchronizes the
 * bound stream.
 *   out    |phi_X| floats in the clique's table layout; host or device
 *          pointer; may be NULL to read only log_z;
 *   log_z  host pointer, may be NULL.
 * Errors: JT_E_ARG, JT_E_STATE (nothing propagated yet), JT_E_HIP,
 * JT_E_ZERO_EVIDENCE (then *log_z = -inf and out is left untouched). */
jt_status jt_marginal(jt_tree t, int32_t slot, int32_t clique, float *out, double *log_z);

/* All clique posteriors of one slot, concatenated in clique order
 * (sum of |phi_X| floats, host or device pointer).  Same errors as
 * jt_marginal. */
jt_status jt_marginals_all(jt_tree t, int32_t slot, float *out, double *log_z);

/* The paper's own kernel design, kept as an ablation of the tiled engine
 * (Sec. 3.2 Algorithm 1, Sec. 4.5 Fig. 8): jt_propagate with
 * JT_MODE_PAPER (or JT_MODE_PAPER_GRAPH, the same launches replayed from a
 * captured graph) runs one message at a time in the order of Algorithms 2-3
 * on the caller's root, children ascending, each evidence set after the
 * other; a message is three launches with one thread per separator entry j:
 * marginalize through the explicit mapping list mu(j), normalize (sigma,
 * log-scales, new/old with 0/0 := 0) and scatter-multiply through mu(j) of
 * the receiving table.  The mapping lists live in a second caller workspace:
 *   jt_paper_bytes    its size;
 *   jt_paper_bind     build the lists on the host (after jt_bind) in
 *                     `layout`: JT_LAYOUT_NAIVE (list j contiguous) or
 *                     JT_LAYOUT_INTERLEAVED (entry n of all lists contiguous,
 *                     Fig. 8's improved layout), upload them and set the
 *                     threads per block (1..1024) of the per-entry kernels;
 *                     synchronizes the bound stream.  May be called again
 *                     to switch layout or block size.
 * Results equal the other schedules' within the stated tolerance, and are
 * bit-identical between the two layouts and across block sizes.
 * Errors: JT_E_ARG, JT_E_STATE (jt_bind missing), JT_E_NO_MEM, JT_E_HIP;
 * jt_propagate with a paper mode before jt_paper_bind returns JT_E_STATE. */
#define JT_LAYOUT_NAIVE 0
#define JT_LAYOUT_INTERLEAVED 1
jt_status jt_paper_bytes(jt_tree t, size_t *bytes);
jt_status jt_paper_bind(jt_tree t, void *workspace, size_t bytes, int32_t layout, int32_t threads_per_block);

/* Bayesian-network front end (Sec. 2.1: a junction tree is compiled from a
 * Bayesian network by moralization and triangulation; Algorithm 4's
 * Initialization multiplies the conditional tables into the cliques).
 *   jt_bn_desc      variables 0..n_vars-1 with card[v] states; variable v's
 *                   parents are parents[parent_off[v] .. parent_off[v+1]) and
 *                   its conditional table P(v | parents) is laid out as
 *                   (parents in that order..., v), last fastest, |table| =
 *                   product of the cards; the tables of all variables are
 *                   concatenated in variable order.
 *   jt_compile_bn   validate (parents in range, no cycle), moralize,
 *                   triangulate (greedy elimination, fewest fill-in edges,
 *                   ties to fewer neighbours, then the lower id), keep the
 *                   maximal cliques (each lists its variables ascending), join
 *                   them by a maximum-weight spanning tree over separator
 *                   sizes (ties to the lower clique ids; components joined by
 *                   empty separators), root at clique 0, assign each family
 *                   to the lowest-id clique holding it, and compile the tree
 *                   as jt_compile_index_maps does (n_slots, tuning as there).
 *                   *n_cliques receives the clique count.
 *   jt_bn_structure the compiled tree: clique_off [n_cliques + 1],
 *                   clique_vars [clique_off[n_cliques]], parent [n_cliques],
 *                   family_clique [n_vars] (host arrays, caller-sized: query
 *                   the clique count first, then JT_Q_TOTAL_CLIQUE_VARS).
 *   jt_bind_bn      jt_bind, with the initial tables computed on the device
 *                   from the conditional tables (`cpts`, device pointer, read
 *                   during the call: it synchronizes the stream): each
 *                   clique's table is the product, in ascending variable
 *                   order, of the tables of the families assigned to it (1
 *                   where none is).
 *   jt_bn_expected_counts  after a propagation of slots [0, n_active): for
 *                   every variable the expected counts of its family,
 *                   sum over the slots of P(v, parents | e_slot), in the
 *                   conditional table's layout, concatenated like the
 *                   tables (`counts`, device pointer, FP32; each entry summed
 *                   in FP64, slots in order).  Asynchronous on the bound
 *                   stream.  The E-step of EM over a batch of evidence sets.
 *   jt_bn_m_step    the M-step: every row of every conditional table (the
 *                   card[v] entries of one parent configuration) becomes
 *                   (counts + alpha) / sum over the row of (counts + alpha),
 *                   into `cpts` (device pointers; alpha >= 0 is a Dirichlet
 *                   pseudo-count; a row with zero sum becomes uniform).
 *                   Asynchronous.
 *   jt_bn_set_cpts  recompute the initial tables from new conditional tables
 *                   (device pointer, read by the stream before the next
 *                   propagation); asynchronous, like jt_bind_bn's product.
 * Errors: JT_E_ARG, JT_E_NOT_JUNCTION_TREE (a cycle among the parents),
 * JT_E_TOO_LARGE (a clique table of 2^31 entries or more), JT_E_NO_MEM,
 * JT_E_STATE (not a network tree, or nothing propagated), JT_E_HIP. */
typedef struct {
    int32_t n_vars;
    const int32_t *card;
    const int64_t *parent_off;  /* [n_vars + 1] */
    const int32_t *parents;     /* [parent_off[n_vars]] */
    int32_t n_slots;
    const jt_tuning *tuning;
} jt_bn_desc;
jt_status jt_compile_bn(const jt_bn_desc *bn, jt_tree *out, size_t *device_bytes, int32_t *n_cliques);
jt_status jt_bn_structure(jt_tree t, int64_t *clique_off, int32_t *clique_vars, int32_t *parent,
                          int32_t *family_clique);
jt_status jt_bind_bn(jt_tree t, void *workspace, size_t bytes, const float *cpts, void *hip_stream);
jt_status jt_bn_expected_counts(jt_tree t, int32_t n_active, float *counts);
jt_status jt_bn_m_step(jt_tree t, const float *counts, float alpha, float *cpts);
jt_status jt_bn_set_cpts(jt_tree t, const float *cpts);

/* Merging small separators (the paper's Sec. 5 future work: fewer, larger
 * messages for trees of many small cliques).  jt_compile_merged validates
 * the caller's tree and contracts, bottom-up from its root (children before
 * parents, ascending ids), every edge whose separator has at most max_sep
 * entries while the merged clique's table stays within max_entries entries;
 * a merged clique lists the union of its cliques' variables ascending.  The
 * handle keeps the caller's cliques as its interface: jt_bind takes their
 * tables (concatenated in their order) and the device multiplies them into
 * the merged cliques; jt_marginal / jt_marginals_all return the caller's
 * cliques' posteriors, marginalized from their merged cliques on the device
 * (FP64 sums; they synchronize the stream); evidence, propagation and the
 * schedules are unchanged.  Exact results equal those of the unmerged tree
 * (within the stated tolerance).  *n_compiled receives the merged clique
 * count; jt_read_out, the mapping queries and the paper schedule refer to the
 * merged cliques.  Errors: as jt_compile_index_maps, and JT_E_ARG for bounds
 * below 1. */
jt_status jt_compile_merged(const jt_tree_desc *desc, int32_t max_sep, int64_t max_entries, jt_tree *out,
                            size_t *device_bytes, int32_t *n_compiled);

/* Asynchronous read-out on the bound stream: the posteriors of slots
 * [slot0, slot0 + n) packed in clique order, slot after slot
 * (n * sum |phi_X| floats), and their log Z_e (n doubles, -inf where the
 * evidence has probability zero; the posteriors of such a slot are
 * undefined).  Both outputs are device pointers.  Ordered after the last
 * propagation; a serving loop records an event after it to know when a
 * query's result is complete.  Errors: JT_E_ARG, JT_E_STATE (a slot not
 * active in the last propagation), JT_E_HIP. */
jt_status jt_read_out(jt_tree t, int32_t slot0, int32_t n, float *posteriors, double *log_z);

/* The cluster-separator mapping of Sec. 3.2 in its single-table form (CSM):
 * for edge (child, parent[child]), side 0 = the child's table, side 1 = the
 * parent's table, host_out[r] = index of the separator entry that table
 * entry r maps to.  host_out has |phi_X| entries.  Host only.
 * Errors: JT_E_ARG. */
jt_status jt_get_index_map(jt_tree t, int32_t child, int32_t side, int32_t *host_out);

/* The same mapping as the paper's |phi_S| lists mu_{X, phi_S(j)}: list j
 * holds the table entries that map to separator entry j, in ascending
 * order, stored at host_out[j * m .. (j+1) * m) with m = |phi_X| / |phi_S|.
 * Host only.  Errors: JT_E_ARG. */
jt_status jt_get_mu_lists(jt_tree t, int32_t child, int32_t side, int32_t *host_out);

/* Scalar facts about a compiled tree (host only), selected by `what`:
 *   JT_Q_N_SLOTS, JT_Q_TOTAL_ENTRIES (sum |phi_X|),
 *   JT_Q_TABLE_SIZE (clique = arg), JT_Q_SEP_SIZE (edge child = arg),
 *   JT_Q_ENTRIES_PER_SWEEP (sum over the n-1 messages of one sweep of
 *     |phi_Xi| + |phi_Xk|, eq. (4)'s numerator, per slot),
 *   JT_Q_BYTES_FUSED (FP32 table bytes one fused propagation reads and
 *     writes, all slots), JT_Q_BYTES_PLAIN (same for JT_MODE_PLAIN),
 *   JT_Q_N_LAUNCHES_FUSED, JT_Q_N_LAUNCHES_PLAIN (kernel launches per
 *     propagation), JT_Q_HEIGHT (levels of the collect sweep),
 *   JT_Q_DEPTH (levels of the distribute sweep),
 *   JT_Q_FUSED_LAUNCH_KIND (arg = launch index: 1, a pass launch -- every
 *     launch of the fused schedule is one),
 *   JT_Q_FUSED_LAUNCH_BYTES (arg = launch index: FP32 table bytes of that
 *     pass launch),
 *   JT_Q_SLOT_BYTES (workspace bytes each slot adds),
 *   JT_Q_SHARED_BYTES (workspace bytes independent of the slot count),
 *   JT_Q_ROOT (the clique the schedules collect to and distribute from: a
 *     center of the tree, i.e. the middle of a longest path, so the sweeps
 *     have the fewest levels; the caller's root only orients the edges),
 *   JT_Q_N_LANES (streams the fused schedule spreads the root's subtrees
 *     over, 0 when everything runs on the bound stream),
 *   JT_Q_CLIQUE_LANE (arg = clique: its lane, -1 for the root or without lanes),
 *   JT_Q_FUSED_LAUNCH_LANE (arg = launch index: the lane it runs on, -1 for
 *     the bound stream),
 *   JT_Q_BYTES_LAST (FP32 table bytes the last propagation moved: shared
 *     tables -- initial tables, evidence-free collect tables read by several
 *     slots -- counted once per launch, every slot's own tables per slot),
 *   JT_Q_LAST_SHARED (1 when the last propagation computed the evidence-free
 *     collect messages once and shared them, see jt_propagate),
 *   JT_Q_LAST_COLLECT_PASSES ((clique, slot) collect passes it ran, the
 *     evidence-free slot included),
 *   JT_Q_TOTAL_CLIQUE_VARS (sum of the cliques' variable counts),
 *   JT_Q_CPT_TOTAL (network trees: floats of the concatenated conditional
 *     tables, 0 otherwise),
 *   JT_Q_N_COMPILED_CLIQUES, JT_Q_COMPILED_TABLE_SIZE (arg = clique): the
 *     cliques the schedules run on (for a merged tree its merged cliques;
 *     JT_Q_TABLE_SIZE and JT_Q_TOTAL_ENTRIES describe the caller's),
 *   JT_Q_LAST_LAUNCH_BYTES (arg = launch index, as for
 *     JT_Q_FUSED_LAUNCH_BYTES: FP32 table bytes that launch moved in the last
 *     JT_MODE_FUSED / JT_MODE_GRAPH propagation, counted as for
 *     JT_Q_BYTES_LAST; a shared source table read by both of a level's
 *     distribute launches is counted in the multi-slot one),
 *   JT_Q_FUSED_LAUNCH_MULTI (arg = launch index: 1 for a multi-slot
 *     distribute launch, which runs on the handle's side stream beside the
 *     level's one-slot launch, 0 otherwise),
 *   JT_Q_FUSED_LAUNCH_BLOCKS (arg = launch index: its blocks per evidence
 *     set, i.e. its tasks; a launch over all slots runs that many per slot,
 *     a listed one the (task, slot) pairs the evidence needs),
 *   JT_Q_ALG_BYTES (arg = slot count, 0 = all: the FP32 table bytes a fused
 *     propagation must move when every slot is computed on its own -- per
 *     clique and entry 12 B for a leaf (initial table read twice, posterior
 *     written), 16 B for an inner clique (its absorbed table written and read
 *     back too), 8 B for the schedule's root (read once, written once) -- the
 *     algorithmic count the roofline is priced on; shared evidence-free
 *     collect messages make the executed schedule move fewer, JT_Q_BYTES_LAST).
 * JT_Q_BYTES_LAST, JT_Q_LAST_SHARED and JT_Q_LAST_COLLECT_PASSES return
 * JT_E_STATE before the first propagation, JT_Q_LAST_LAUNCH_BYTES before the
 * first fused or graph propagation.  Other errors: JT_E_ARG. */
#define JT_Q_N_SLOTS 0
#define JT_Q_TOTAL_ENTRIES 1
#define JT_Q_TABLE_SIZE 2
#define JT_Q_SEP_SIZE 3
#define JT_Q_ENTRIES_PER_SWEEP 4
#define JT_Q_BYTES_FUSED 5
#define JT_Q_BYTES_PLAIN 6
#define JT_Q_N_LAUNCHES_FUSED 7
#define JT_Q_N_LAUNCHES_PLAIN 8
#define JT_Q_HEIGHT 9
#define JT_Q_DEPTH 10
#define JT_Q_FUSED_LAUNCH_KIND 11
#define JT_Q_FUSED_LAUNCH_BYTES 12
#define JT_Q_SLOT_BYTES 13
#define JT_Q_SHARED_BYTES 14
#define JT_Q_ROOT 15
#define JT_Q_N_LANES 16
#define JT_Q_CLIQUE_LANE 17
#define JT_Q_FUSED_LAUNCH_LANE 18
#define JT_Q_BYTES_LAST 19
#define JT_Q_LAST_SHARED 20
#define JT_Q_LAST_COLLECT_PASSES 21
#define JT_Q_TOTAL_CLIQUE_VARS 22
#define JT_Q_CPT_TOTAL 23
#define JT_Q_N_COMPILED_CLIQUES 24
#define JT_Q_COMPILED_TABLE_SIZE 25
#define JT_Q_LAST_LAUNCH_BYTES 26
#define JT_Q_ALG_BYTES 27
#define JT_Q_FUSED_LAUNCH_MULTI 28
#define JT_Q_FUSED_LAUNCH_BLOCKS 29
jt_status jt_query(jt_tree t, int32_t what, int64_t arg, int64_t *out);

/* Run one propagation with a HIP event pair around every kernel launch and
 * report the device time spent in the pass launches (which finalize their
 * messages too) and in the other launches -- the set-up kernel of
 * JT_MODE_PLAIN -- (milliseconds, summed over the propagation) and how many
 * of each ran.  Synchronizes the bound stream.  For measurement only; the
 * results it leaves are those of a normal jt_propagate.
 *   mode  JT_MODE_FUSED or JT_MODE_PLAIN;
 *   pass_ms, finalize_ms, n_pass, n_finalize  host pointers (any may be NULL);
 *     finalize_ms and n_finalize count the launches other than passes.
 * Errors: JT_E_STATE, JT_E_ARG, JT_E_HIP. */
jt_status jt_profile(jt_tree t, int32_t mode, double *pass_ms, double *finalize_ms, int32_t *n_pass,
                     int32_t *n_finalize);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): one propagation of every slot of a compiled tree in a static device
 * scratch array owned by the library (128 MiB per GPU, held until the
 * process ends) instead of a caller workspace; no jt_bind is
 * needed and the handle's own binding, if any, is left untouched.  The
 * library calls no device allocator here.
 *   init_potentials  device pointer, FP32 tables concatenated in clique order;
 *   posteriors       device pointer, n_slots * sum |phi_X| floats: every
 *                    slot's normalized clique posteriors, clique order, slot
 *                    after slot (undefined for a slot whose evidence has
 *                    probability zero);
 *   log_z            device pointer, n_slots doubles: log Z_e per slot, -inf
 *                    when the evidence has probability zero;
 *   mode             JT_MODE_FUSED or JT_MODE_PLAIN;
 *   hip_stream       stream the work is enqueued on (asynchronous).
 * The evidence is the handle's (jt_set_evidence).  Every call on one GPU
 * uses that GPU's one scratch array, which keeps the last call's contents:
 * calls that overlap on one GPU (different streams, or a second call before
 * the first has finished reading its inputs) race, and the handle must stay
 * alive, with its evidence unchanged, until the stream has run the call.
 * Results are bit-identical to jt_bind + jt_propagate in the same mode.
 * Errors: JT_E_ARG, JT_E_NO_MEM (the tree's workspace exceeds the scratch;
 * nothing is launched), JT_E_HIP. */
jt_status jt_propagate_scratch(jt_tree t, const float *init_potentials, float *posteriors, double *log_z,
                               int32_t mode, void *hip_stream);

/* Release the handle and its host-side objects (captured graphs included),
 * after the work queued on its bound stream has finished.  Device memory
 * stays the caller's.  NULL is ignored. */
void jt_free(jt_tree t);

/* Thread-local text of the last failure on this thread ("" if none). */
const char *jt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* JT_H */
