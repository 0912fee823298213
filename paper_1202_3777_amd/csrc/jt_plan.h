// jt_plan.h -- host-side compiled junction tree (C++ only, no HIP).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "jt.h"
#include "jt_internal.h"

namespace jt {

// A digit of the table index.  A variable is one digit, or two when the
// tile boundary falls inside it (high digit outer, low digit inner); the
// variable's state is sum(sub_digit * w).
struct VDigit {
    int32_t var;
    int32_t card;
    int64_t stride;   // in table entries
    int64_t w;        // weight of this digit inside the variable's state
    bool outer;
    int64_t ostride;  // in tiles (outer digits only)
};

struct CliqueInfo {
    std::vector<int32_t> vars;       // listed order = table layout
    int64_t size = 0;
    std::vector<VDigit> digits;
    int32_t T = 1, vec = 1;
    int64_t n_tiles = 1;
    int64_t init_off = 0, coll_off = -1, out_off = 0;
    int32_t height = 0, depth = 0;
    std::vector<int32_t> children;   // ascending id, schedule orientation
    int32_t total_view = -1;
    int32_t parent_view = -1;        // this clique through the separator to its schedule parent
};

struct EdgeInfo {                    // edge (c, parent[c]); id = c
    std::vector<int32_t> vars;       // ascending id
    std::vector<int64_t> sst;        // separator stride of each variable
    int64_t ssize = 1;
    int32_t sepc_off = 0, sepd_off = 0;
    int32_t view_child = -1, view_parent = -1;
};

struct Launch {
    int32_t is_pass;        // 1 = pass kernel over tasks, 2 = one-at-a-time set-up
    int32_t begin, count;   // tasks (per slot)
    int64_t bytes = 0;      // FP32 table bytes a pass launch reads and writes (all slots)
    int32_t lds_floats = 0; // dynamic LDS of a pass launch (staged ratio tables, finalize scratch)
    int32_t lane = -1;      // stream: -1 the bound stream, else the lane of a root subtree
    int32_t join_before = 0;  // the bound stream first waits for every lane
    int32_t fork_after = 0;   // every lane then waits for the bound stream
    // Listed launch (batched collect): the blocks walk a list of (task, slot)
    // entries written per propagation, instead of every task of every slot.
    int32_t listed = 0;
    int64_t work_off = 0;   // first entry in the work region
    int32_t work_cap = 0;   // entries the list can hold: count * (slots + 1)
    int32_t work_idx = 0;   // its counter in the work-count array
    int32_t collect = 0;    // 1: a collect-sweep launch of the fused schedule
    int32_t multi = 0;      // 1: multi-slot distribute launch (entries index JtChunk sets)
    int64_t chunk_off = 0;  // its first chunk in the chunk region
    int32_t chunk_cap = 0;
    // One-slot distribute launch that may read what an earlier multi-slot
    // launch wrote: it holds an item a multi-slot launch cannot take, so a
    // slot whose parent pass ran in a multi-slot set can land here.  Without
    // the flag every pair it runs has evidence below its clique, and so has
    // the pair's parent pass, which then ran in a one-slot launch too.
    int32_t after_multi = 0;
};

// A family (variable and parents) to be mapped into a clique: the index of
// clique entry r in the family's table laid out as vars (last fastest).
struct FamilyReq {
    int32_t clique;
    int32_t var;
    std::vector<int32_t> vars;   // parents..., var
    int64_t cpt_off;             // in the concatenated conditional tables
};

struct Plan {
    // shape choices (defaults filled in)
    jt_tuning tune{};
    // tree
    int32_t n_vars = 0, n_cliques = 0, n_slots = 1, root = -1;
    std::vector<int32_t> card, parent;
    std::vector<CliqueInfo> cl;
    std::vector<EdgeInfo> edge;
    std::vector<int32_t> home;       // lowest clique id holding each variable
    // The schedules run on the tree re-rooted at a center clique (fewest
    // levels); edges keep the caller's ids (the child clique of the caller's
    // orientation).  iparent / iedge: parent in the schedule's orientation and
    // the id of the edge to it; user_root: the caller's root.
    std::vector<int32_t> iparent, iedge;
    int32_t user_root = -1;
    // Lanes: the root's subtrees, grouped into at most JT_MAX_LANES sets of
    // about equal work; each lane's levels run on a stream of their own, so
    // one subtree's launch tail overlaps another's streaming.
    std::vector<int32_t> lane;       // per clique, -1 for the root
    int32_t n_lanes = 0;
    int32_t height = 0, depth = 0;

    // device metadata (host copies)
    std::vector<int32_t> meta;
    std::vector<JtView> views;
    std::vector<JtGather> gathers;
    std::vector<JtItem> items;
    std::vector<JtTask> tasks;
    std::vector<JtBlock> blocks;     // device records of the tasks (same order)
    std::vector<JtMsg> msgs;
    std::vector<int32_t> child_edges;   // pairs (edge id, schedule child clique)
    std::vector<Launch> fused;       // launch list of one fused propagation (finalize inside the passes)
    std::vector<Launch> plain;       // launch list of one one-at-a-time propagation
    int32_t plain_reset_task_begin = 0, plain_reset_task_count = 0;

    // Batched trees (n_slots >= 2) keep one extra, evidence-free slot (index
    // n_slots) whose collect messages every slot without evidence below an
    // edge reads instead of computing its own; the collect launches are then
    // listed launches.
    int32_t share = 0;
    int32_t n_regions = 1;           // slot regions: n_slots + share
    int32_t n_listed = 0;            // listed launches (work counters)
    int64_t work_total = 0;          // entries of all listed launches
    int64_t chunk_total = 0;         // slot sets of all multi-slot launches
    std::vector<char> item_multi;    // per item: eligible for multi-slot passes
    // per-slot region sizes (elements)
    int64_t csrc_stride = 0;
    int64_t init_floats = 0, coll_stride = 0, out_stride = 0, sep_stride = 0,
            partial_stride = 0, lam_stride = 0, scale_stride = 0, ev_idx_stride = 0,
            ev_ent_stride = 0, icnt_stride = 0;
    // byte offsets of every region inside the workspace
    size_t off_meta = 0, off_views = 0, off_gathers = 0, off_items = 0, off_tasks = 0, off_blocks = 0,
           off_msgs = 0, off_child = 0, off_init = 0, off_coll = 0, off_out = 0, off_sep = 0,
           off_partial = 0, off_lam = 0, off_scale = 0, off_flag = 0, off_ev_idx = 0,
           off_ev_ent = 0, off_icnt = 0, off_csrc = 0, off_work = 0, off_work_count = 0, off_cltab = 0,
           off_chunks = 0,
           total_bytes = 0;
    // the part of the workspace rewritten when evidence or the active slot
    // count change (evidence tables, collect sources, work lists): one range
    size_t off_dyn = 0, dyn_bytes = 0;
    std::vector<int64_t> cltab;      // per clique: posterior offset, size, packed offset
    // Bayesian-network trees: the families, sorted by clique, and each
    // clique's range of them; the mapping lists of each family
    std::vector<JtFamily> fam;
    std::vector<int32_t> fam_rng;    // [n_cliques + 1]
    int64_t fam_mu_total = 0, cpt_total = 0;
    std::vector<JtCliqueShape> cshape;   // per clique (network trees)
    int64_t max_tiles = 0, max_fsize = 0;
    size_t off_fam = 0, off_fam_rng = 0, off_fam_mu = 0, off_cshape = 0, off_card = 0;
    // merged trees: read-out staging of one slot's original-clique posteriors
    int64_t stage_floats = 0;
    size_t off_stage = 0;
    size_t slot_bytes = 0;           // workspace bytes that scale with the slot count (per slot)

    // statistics
    int64_t total_entries = 0, entries_per_sweep = 0;
    int64_t bytes_fused = 0, bytes_plain = 0;   // all slots; shared initial tables counted once
};

// Paper-faithful schedule of a compiled tree (host side): messages in the
// order of Algorithms 2-3 on the caller's root, children ascending, and the
// per-entry blocks of the reset and normalization kernels.
struct PaperPlan {
    std::vector<JtPaperMsg> msgs;
    std::vector<JtPaperBlk> blocks;
    int64_t mu_total = 0;                 // int32 entries of all mapping lists
    size_t off_msgs = 0, off_blocks = 0, off_mu = 0, bytes = 0;
};
void build_paper_plan(const Plan &plan, PaperPlan &pp);
// The mapping lists of every message's two tables in `layout`
// (JT_LAYOUT_NAIVE_ or JT_LAYOUT_INTERLEAVED_), concatenated as the
// messages' mu_from / mu_to offsets say.
void paper_mu_lists(const Plan &plan, const PaperPlan &pp, int32_t layout, int32_t *out);

// Build the plan; returns JT_OK or an error code with `err` filled in.
// `families` (Bayesian-network trees only): the conditional tables to map
// into their cliques; cpt_total their concatenated size.
// The host-side checks compile_plan runs on every plan (index ranges, layouts
// and the fused schedule's dataflow order); false with `why` on a failure.
bool check_plan(const Plan &plan, std::string &why);
jt_status compile_plan(const jt_tree_desc *desc, Plan &plan, std::string &err,
                       const std::vector<FamilyReq> *families = nullptr, int64_t cpt_total = 0);

// The family mapping lists of a Bayesian-network tree (list j of family k:
// the entries of its clique whose family index is j, ascending), at each
// family's mu_off: fam_mu_total int32.
void family_mu_lists(const Plan &plan, int32_t *out);

// Bayesian network -> junction tree (host): moralize, triangulate by greedy
// min-fill elimination, keep the maximal cliques (variables ascending), join
// them by a maximum-weight spanning tree over separator sizes, root at
// clique 0, and give every family the lowest-id clique that holds it.
struct BnTree {
    std::vector<int32_t> card;
    std::vector<std::vector<int32_t>> cliques;
    std::vector<int32_t> parent;
    std::vector<FamilyReq> families;
    int64_t cpt_total = 0;
};
jt_status compile_bn(const jt_bn_desc *bn, BnTree &out, std::string &err);

// Merging small separators (the paper's Sec. 5): contract every edge whose
// separator has at most max_sep entries, bottom-up from the caller's
// root, while the merged clique's table stays within max_entries.  Each
// merged clique lists the union of its cliques' variables ascending; the
// original cliques become its "families" (their tables multiplied into it,
// their posteriors read back out of it).  The caller's tree is validated.
struct MergedTree {
    std::vector<int32_t> card;
    std::vector<std::vector<int32_t>> cliques;
    std::vector<int32_t> parent;
    std::vector<FamilyReq> families;     // var = original clique id
    std::vector<int64_t> orig_size;      // per original clique
    int64_t total = 0;                   // sum of the original table sizes
};
jt_status merge_tree(const jt_tree_desc *desc, int32_t max_sep, int64_t max_entries, MergedTree &out,
                     std::string &err);

// Per-propagation schedule of a batched tree: which (clique, slot) pairs the
// collect sweep computes and where every slot reads collect data from.
struct Dynamic {
    std::vector<int32_t> csrc;          // [n_regions][csrc_stride]
    std::vector<JtWork> work;           // [work_total]
    std::vector<JtChunk> chunks;        // [chunk_total]
    std::vector<int32_t> count;         // [n_listed]
    std::vector<int32_t> grid;          // [n_listed] blocks launched: the count rounded up to a power of
                                        // two (at most the list's capacity), so few graphs cover many counts
    int64_t bytes = 0;                  // FP32 table bytes of the fused propagation it describes
    std::vector<int64_t> launch_bytes;  // [fused launches] the same per launch
    int32_t shared = 0;                 // 1: the evidence-free slot is computed and read
    int64_t collect_pairs = 0;          // (clique, slot) collect passes, evidence-free slot included
};

// Build the dynamic schedule for slots [0, n_active) with the given
// evidence (one variable list per slot).  Sharing is used when it moves
// fewer bytes than computing every slot's collect sweep.
void build_dynamic(const Plan &plan, const std::vector<std::vector<int32_t>> &ev_vars, int32_t n_active,
                   Dynamic &dyn);

// Evidence of one slot as device digit conditions (host side).
// idx gets n_cliques + 1 offsets into ent; ent gets the conditions.
void evidence_tables(const Plan &plan, const std::vector<int32_t> &vars,
                     const std::vector<int32_t> &states, int32_t *idx, JtEv *ent);

// Separator index of every entry of clique `c` seen through view `v`
// (reconstructed from the factored tables).
void expand_map(const Plan &plan, int32_t view, int32_t *out);

}  // namespace jt
