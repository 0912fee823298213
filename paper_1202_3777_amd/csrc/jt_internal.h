// jt_internal.h -- plan structures shared by the host planner and the HIP
// kernels of the junction-tree message engine.  Plain structs of fixed-width
// integers so the same bytes are valid on host and device.
//
// Index mapping in factored form.  A clique table phi_X is cut into tiles of
// T consecutive entries, T being the product of the innermost (fastest)
// variables' cardinalities (an innermost variable may be split into a high
// and a low digit when a divisor of its cardinality fits).  Entry r = o*T + i
// then has its state string split into the tile's (outer) digits and the
// in-tile (inner) digits, and the separator index of Sec. 3.1's mapping rule
// is a sum of two parts:
//     j(r) = Jin[i] + Jout[o].
// Jin has T entries and Jout |phi_X|/T entries, so the cluster-separator
// mapping (the single table of CSM, or the paper's |phi_S| lists) costs no
// per-entry index storage and no per-entry division on the device.
#pragma once
#include <stdint.h>

#define JT_WAVE 64
#define JT_BLOCK 256
#define JT_WAVES_PER_BLOCK (JT_BLOCK / JT_WAVE)
#define JT_TILE_MAX 256           /* one wave covers a tile: 64 lanes x 4 entries */
#define JT_NG_REG 4               /* gathers whose Jin values live in registers */
#define JT_LDS_RATIO_FLOATS 8192  /* at most 32 KiB of LDS for staged ratio tables */
#define JT_FIN_LDS_FLOATS 64      /* smallest dynamic LDS of a pass launch */
#define JT_FIN_STAGE_FLOATS 4096  /* separators up to this size are finalized through LDS */
#ifndef JT_UNROLL
#define JT_UNROLL 2               /* tiles (paired: tile pairs) per batch; two batches in flight per wave */
#endif
#ifndef JT_MAX_LANES
#define JT_MAX_LANES 4            /* streams the fused schedule could spread the root's subtrees over */
#endif
/* Lanes are switched off: the first GPU run with them ended in a host-side
 * segmentation fault inside a graph propagation (cause not found), so
 * max_lanes must stay 1 and every level runs on the bound stream.  (Only the
 * sanitized host build of the planner turns them on, to check their
 * planning.) */
#ifndef JT_LANES_ENABLED
#define JT_LANES_ENABLED 0
#endif
#ifndef JT_WAVE_GROUP_TILES
#define JT_WAVE_GROUP_TILES 28    /* output views with at most this many tiles per kept-outer configuration use wave groups */
#endif
#ifndef JT_PAIR_TILES
#define JT_PAIR_TILES 1           /* tiles of at most JT_TILE_MAX / 2 entries are streamed two per wave load */
#endif

// One clique table seen through one separator (or through the empty
// separator, for the table's total).
typedef struct {
    int64_t jin_off;        // int32 meta: Jin[T]
    int64_t jout_off;       // int32 meta: Jout[n_tiles]
    int64_t kout_tile_off;  // int32 meta: tile offset of each kept-outer configuration
    int64_t kout_j_off;     // int32 meta: separator offset of each kept-outer configuration
    int64_t rout_tile_off;  // int32 meta: tile offset of each reduced-outer configuration
    int64_t perm_off;       // int32 meta: in-tile positions grouped by class, ascending
    int64_t clsj_off;       // int32 meta: separator offset of each class
    int32_t n_kout, n_rout, n_cls, m_in;
    int32_t ssize, clique;
} JtView;

// A separator table multiplied into the entries of a pass.
typedef struct {
    int32_t view;     // view of the pass's clique through that separator
    int32_t sep_off;  // float offset of the table inside the per-slot separator region
    int32_t ssize;
    int32_t lds_off;  // float offset of its LDS copy, -1 = read from global memory
    int32_t jin_off, jout_off;   // the view's Jin / Jout tables (int32 meta offsets)
    int32_t src_clique;          // collect message of this (child) clique: read from the slot that
                                 // holds that clique's collect data (see JtDev::csrc); -1: the
                                 // launch's own slot (distribute ratios)
} JtGather;

enum { JT_SRC_INIT = 0, JT_SRC_COLL = 1, JT_SRC_OUT = 2 };

// Launch flags of the pass kernel.
#define JT_PF_SHARE 1     // collect data are read through the per-slot collect sources
enum { JT_DST_NONE = -1, JT_DST_COLL = 1, JT_DST_OUT = 2 };

// One streaming pass over one clique table (per slot):
//   v = src[r] * [evidence] * prod_g ratio_g[j_g(r)] * scale
//   if dst: dst[r] = v;   if out_view: partial[j_out(r)] += v
typedef struct {
    int32_t clique, T, vec, n_tiles;
    int32_t src_kind, dst_kind;
    int64_t src_off, dst_off;   // float offsets (init region, or per-slot region)
    int32_t n_gather, gather_base;
    int32_t n_gather_lds, lds_floats;
    int32_t scale_clique;       // -1: no scaling
    int32_t ev;                 // 1: enter this slot's evidence of `clique`
    int32_t out_view;           // -1: no reduction output
    int32_t tpg;                // tiles per group (a group is streamed by one block, its
                                // tiles shared out over the block's waves)
    int32_t nsplit;             // groups per kept-outer configuration
    int32_t n_groups;           // per slot; one partial row of the output view per group
    int64_t partial_off;        // float offset in the per-slot partial region
    // the output view's reduction tables, copied here to keep the kernel
    // prologue short (meta offsets stay below 2^30)
    int32_t o_kout_tile, o_kout_j, o_rout_tile, o_perm, o_clsj;
    int32_t o_n_rout, o_n_cls, o_m_in, o_ssize;
    int32_t n_tasks;            // blocks per slot that make up the pass
    int32_t msg;                // message this pass produces and finalizes, -1 none
    int32_t wave_groups;        // 1: short groups (one kept-outer configuration each,
                                // all its tiles), each streamed whole by one wave
    int32_t pair;               // 1: T <= JT_TILE_MAX / 2 with 4-entry lanes, block
                                // groups: a wave load covers two tiles, one per half-wave
} JtItem;

// A block's share of an item: groups [g0, g1), one after the other.
typedef struct {
    int32_t item, g0, g1, pad;
} JtTask;

// What one block of a pass launch reads first, in one record: its task, a
// copy of the item and of the item's first gathers (one dependent load
// instead of three).
typedef struct {
    JtItem it;
    JtGather g[JT_NG_REG];
    int32_t item, g0, g1, pad;
} JtBlock;

enum {
    JT_MSG_COLLECT = 0,   // child -> parent, collect sweep
    JT_MSG_TOTAL = 1,     // root table total: log Z and the root's output scale
    JT_MSG_DIST = 2,      // parent -> child, distribute sweep
    JT_MSG_PLAIN = 3,     // one message of the one-at-a-time schedule
    JT_MSG_PLAIN_TOTAL = 4 // total of a calibrated table, one-at-a-time schedule
};

// Finalization of one message: sum the split partials into the new
// separator table, rescale it to mean one, form the ratio, update log-scales.
typedef struct {
    int32_t kind;
    int32_t edge;           // separator id (= child clique), -1 for a total
    int32_t from, to;
    int32_t ssize, nsplit;
    int64_t partial_off;
    int32_t child_base, n_children;  // children edges of `from` (collect log-scale sum)
    int32_t sepc_off, sepd_off;      // separator tables in the per-slot region
    int32_t item, pad;               // the pass item whose partials this message sums
} JtMsg;

// One digit condition of hard evidence: entry kept iff
// (index / stride) % card == digit, index being the tile index for outer
// digits and the in-tile position for inner ones.
typedef struct {
    int32_t outer, stride, card, digit;
} JtEv;

// Per-slot log-scale layout (doubles): [0,nc) collect separators, [nc,2nc)
// distribute separators, [2nc,3nc) clique collect scales, [3nc] log Z.
#define JT_LAM_SC(nc) 0
#define JT_LAM_SD(nc) (nc)
#define JT_LAM_COLL(nc) (2 * (nc))
#define JT_LAM_LOGZ(nc) (3 * (nc))

// One entry of a listed launch: block-task `task` (relative to the launch's
// first task) of slot `slot`; in a multi-slot launch `slot` indexes a
// JtChunk instead.  task = -1: padding, the block returns at once.
typedef struct {
    int32_t task, slot;
} JtWork;

// Up to JT_MS slots that read the same (evidence-free) source table in one
// multi-slot distribute pass; unused entries are -1 (the used ones first).
#define JT_MS 4
// A level whose sets of JT_MS slots number fewer than one round of resident
// multi-slot blocks (four per CU on a 256-CU GPU) is cut into sets of JT_MS / 2.
#ifndef JT_MULTI_ROUND
#define JT_MULTI_ROUND 1024
#endif
typedef struct {
    int32_t s[JT_MS];
} JtChunk;

// Paper-faithful schedule (the ablation of the paper's own kernel design):
// one message at a time in Algorithm 2-3 order, one thread per separator
// entry reading explicit mapping lists (Algorithm 1), in the naive layout
// (list j contiguous) or the interleaved one (entry n of every list
// contiguous, Fig. 8).
#define JT_LAYOUT_NAIVE_ 0
#define JT_LAYOUT_INTERLEAVED_ 1
typedef struct {
    int64_t mu_from, mu_to;     // int32 offsets of the two mapping-list sets in the paper workspace
    int64_t from_off, to_off;   // float offsets of the two tables in a slot's posterior region
    int32_t m_from, m_to;       // list lengths |phi_X| / |phi_S|
    int32_t ssize, edge, from, to;
    int32_t sepc_off, sepd_off; // old table and new/ratio table of the edge
} JtPaperMsg;

// A block of the paper schedule's per-entry kernels: entries [start, end) of
// one clique's table.
typedef struct {
    int32_t clique, T;          // the clique and its tile (for the evidence digits)
    int64_t start, end;
    int64_t init_off, out_off;  // float offsets of its initial table and of its posterior in a slot
} JtPaperBlk;

// Bayesian-network front end: one job per variable v multiplies its
// conditional table P(v | parents) into the clique that holds the family
// (Algorithm 4's Initialization).  The family's entry index of clique entry
// r = o*T + i is Jin[i] + Jout[o] (the family laid out as parents..., v).
typedef struct {
    int64_t jin_off, jout_off;  // int32 meta offsets
    int64_t cpt_off;            // float offset of the table in the caller's concatenated tables
    int64_t mu_off;             // int32 offset of the family's mapping lists (expected counts)
    int32_t clique, fsize;      // clique holding the family; |P(v | parents)|
    int32_t var, pad;
} JtFamily;

// Per-clique shape for the network front end's kernels.
typedef struct {
    int64_t init_off, n_tiles, size;
    int32_t T, pad;
} JtCliqueShape;

// Everything a kernel needs, passed by value.
typedef struct {
    const int32_t *meta;
    const JtView *views;
    const JtGather *gathers;
    const JtItem *items;
    const JtTask *tasks;
    const JtBlock *blocks;
    const JtMsg *msgs;
    const int32_t *child_edges;
    const float *init;
    float *coll;
    float *out;
    float *sep;
    float *partial;
    double *lam;
    float *scale;
    int32_t *flag;
    int32_t *icnt;                 // per-slot arrival counters of the pass items
    const int32_t *ev_idx;
    const JtEv *ev_ent;
    // Collect source of every (slot, clique): the slot whose collect data
    // (absorbed table, collect message to the schedule parent, collect
    // log-scales) hold this clique's.  A clique whose subtree carries none
    // of the slot's evidence sends the same collect message as with no
    // evidence at all, so batched trees compute that message once, in an
    // extra evidence-free slot, and every such slot reads it from there.
    const int32_t *csrc;
    const JtWork *work;            // entries of the listed launches
    const int32_t *work_count;     // entries per listed launch
    const JtChunk *chunks;         // slot sets of the multi-slot entries
    const int64_t *cltab;          // per clique: posterior offset, size, packed offset
    int64_t coll_stride, out_stride, sep_stride, partial_stride;
    int64_t lam_stride, scale_stride, ev_idx_stride, ev_ent_stride;
    int64_t icnt_stride, csrc_stride;
    int32_t n_cliques, n_msgs;
} JtDev;
