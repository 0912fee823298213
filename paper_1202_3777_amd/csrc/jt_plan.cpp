// jt_plan.cpp -- compile a junction tree into the engine's device plan.
//
// Host only.  Validates the tree (Sec. 2.1: cliques, separators
// S_ij = X_i intersect X_j, one designated root), derives every
// cluster-separator index mapping of Sec. 3.1-3.2 once (the paper
// precomputes them when the tree is established) in factored tile form, and
// lays out the level schedule of the collect / distribute sweeps
// (Algorithms 2-4) plus the one-message-at-a-time schedule.
#include "jt_plan.h"

#include <algorithm>
#include <cstring>
#include <limits>
#include <functional>
#include <map>
#include <set>
#include <stdexcept>

namespace jt {

namespace {

constexpr int64_t kAlignFloats = 64;       // 256-byte alignment of every table
// Tuning constants (overridable at build time for sweeps).
#ifndef JT_TARGET_BLOCKS
#define JT_TARGET_BLOCKS 1280
#endif
#ifndef JT_PARTIAL_MAX
#define JT_PARTIAL_MAX 16384
#endif
#ifndef JT_GROUP_MIN
#define JT_GROUP_MIN 8192
#endif
#ifndef JT_GROUP_MAX
#define JT_GROUP_MAX 32768
#endif
#ifndef JT_WRITE_WEIGHT
#define JT_WRITE_WEIGHT 1          // work of a stored entry relative to a read-only one
#endif
#ifndef JT_GROUP_DIV
#define JT_GROUP_DIV 1024
#endif
constexpr int64_t kPartialMax = JT_PARTIAL_MAX;       // cap on split partial floats per message
constexpr int64_t kMaxMeta = int64_t(1) << 30;

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

jt_status fail(std::string &err, jt_status code, const std::string &msg) {
    err = msg;
    return code;
}

bool has_var(const std::vector<int32_t> &sorted_vars, int32_t v) {
    return std::binary_search(sorted_vars.begin(), sorted_vars.end(), v);
}

// Choose the tile of a clique: the largest product of the innermost
// cardinalities that fits JT_TILE_MAX, splitting the next variable into a
// high and a low digit when a divisor of its cardinality still fits.
void shape_clique(const std::vector<int32_t> &card, CliqueInfo &C) {
    const int m = (int)C.vars.size();
    std::vector<int64_t> st(m);
    int64_t s = 1;
    for (int i = m - 1; i >= 0; --i) {
        st[i] = s;
        s *= card[C.vars[i]];
    }
    C.size = s;
    int64_t prod = 1;
    int i = m - 1;
    while (i >= 0 && prod * card[C.vars[i]] <= JT_TILE_MAX) {
        prod *= card[C.vars[i]];
        --i;
    }
    int split = -1;
    int64_t f = 1;
    if (i >= 0) {
        int64_t k = card[C.vars[i]];
        for (int64_t d = k - 1; d >= 2; --d)
            if (k % d == 0 && prod * d <= JT_TILE_MAX) {
                f = d;
                break;
            }
        if (f > 1) split = i;
    }
    C.T = (int32_t)(prod * f);
    C.n_tiles = C.size / C.T;
    C.vec = (C.T % 4 == 0) ? 4 : 1;
    C.digits.clear();
    for (int a = 0; a < m; ++a) {
        const int32_t v = C.vars[a];
        const int32_t k = card[v];
        if (a == split) {
            VDigit hi{v, (int32_t)(k / f), st[a] * f, f, true, (st[a] * f) / C.T};
            VDigit lo{v, (int32_t)f, st[a], 1, false, 0};
            C.digits.push_back(hi);
            C.digits.push_back(lo);
        } else {
            const bool outer = (a <= i);
            VDigit d{v, k, st[a], 1, outer, outer ? st[a] / C.T : 0};
            C.digits.push_back(d);
        }
    }
}

// Build the factored mapping tables of clique c through edge e (or through
// the empty separator when e < 0) and return the view index.
int32_t build_view(Plan &P, int32_t c, int32_t e) {
    const CliqueInfo &C = P.cl[c];
    JtView V;
    std::memset(&V, 0, sizeof(V));
    V.clique = c;
    V.ssize = (int32_t)(e >= 0 ? P.edge[e].ssize : 1);
    const size_t nd = C.digits.size();
    std::vector<int64_t> ws(nd, 0);
    if (e >= 0) {
        const EdgeInfo &E = P.edge[e];
        for (size_t k = 0; k < nd; ++k)
            for (size_t p = 0; p < E.vars.size(); ++p)
                if (E.vars[p] == C.digits[k].var) ws[k] = E.sst[p] * C.digits[k].w;
    }
    std::vector<int32_t> &M = P.meta;
    // Jin: separator contribution of the in-tile digits
    V.jin_off = (int64_t)M.size();
    for (int64_t i = 0; i < C.T; ++i) {
        int64_t j = 0;
        for (size_t k = 0; k < nd; ++k)
            if (!C.digits[k].outer) j += ((i / C.digits[k].stride) % C.digits[k].card) * ws[k];
        M.push_back((int32_t)j);
    }
    // Jout: separator contribution of the tile digits
    V.jout_off = (int64_t)M.size();
    for (int64_t o = 0; o < C.n_tiles; ++o) {
        int64_t j = 0;
        for (size_t k = 0; k < nd; ++k)
            if (C.digits[k].outer) j += ((o / C.digits[k].ostride) % C.digits[k].card) * ws[k];
        M.push_back((int32_t)j);
    }
    // kept / reduced outer digits and kept inner digits, listed order
    std::vector<size_t> ko, ro, ki;
    for (size_t k = 0; k < nd; ++k) {
        if (C.digits[k].outer)
            (ws[k] ? ko : ro).push_back(k);
        else if (ws[k])
            ki.push_back(k);
    }
    auto count = [&](const std::vector<size_t> &ds) {
        int64_t n = 1;
        for (size_t k : ds) n *= C.digits[k].card;
        return n;
    };
    const int64_t n_kout = count(ko), n_rout = count(ro), n_cls = count(ki);
    V.n_kout = (int32_t)n_kout;
    V.n_rout = (int32_t)n_rout;
    V.n_cls = (int32_t)n_cls;
    V.m_in = (int32_t)(C.T / n_cls);
    // decode a mixed-radix index over a digit list (last listed fastest)
    auto decode = [&](int64_t x, const std::vector<size_t> &ds, int64_t &tile, int64_t &j) {
        tile = 0;
        j = 0;
        for (size_t a = ds.size(); a-- > 0;) {
            const VDigit &d = C.digits[ds[a]];
            const int64_t dig = x % d.card;
            x /= d.card;
            tile += dig * d.ostride;
            j += dig * ws[ds[a]];
        }
    };
    V.kout_tile_off = (int64_t)M.size();
    for (int64_t k = 0; k < n_kout; ++k) {
        int64_t t, j;
        decode(k, ko, t, j);
        M.push_back((int32_t)t);
    }
    V.kout_j_off = (int64_t)M.size();
    for (int64_t k = 0; k < n_kout; ++k) {
        int64_t t, j;
        decode(k, ko, t, j);
        M.push_back((int32_t)j);
    }
    V.rout_tile_off = (int64_t)M.size();
    for (int64_t q = 0; q < n_rout; ++q) {
        int64_t t, j;
        decode(q, ro, t, j);
        M.push_back((int32_t)t);
    }
    // in-tile positions grouped by class (kept inner digits), ascending
    V.perm_off = (int64_t)M.size();
    M.resize(M.size() + C.T);
    std::vector<int64_t> fill(n_cls, 0);
    for (int64_t i = 0; i < C.T; ++i) {
        int64_t cls = 0;
        for (size_t k : ki) cls = cls * C.digits[k].card + (i / C.digits[k].stride) % C.digits[k].card;
        M[V.perm_off + cls * V.m_in + fill[cls]++] = (int32_t)i;
    }
    V.clsj_off = (int64_t)M.size();
    for (int64_t cls = 0; cls < n_cls; ++cls) M.push_back(M[V.jin_off + M[V.perm_off + cls * V.m_in]]);
    P.views.push_back(V);
    return (int32_t)P.views.size() - 1;
}

// Jin / Jout tables of clique c seen through an arbitrary variable list
// `vars` laid out row-major, last fastest (a conditional table's layout):
// entry o*T + i of the clique has index Jin[i] + Jout[o] in that table.
// Returns false when a variable of the list is not in the clique.
bool build_projection(Plan &P, int32_t c, const std::vector<int32_t> &vars, int64_t &jin_off, int64_t &jout_off) {
    const CliqueInfo &C = P.cl[c];
    const size_t nd = C.digits.size();
    std::vector<int64_t> ws(nd, 0);
    int64_t stride = 1;
    for (size_t q = vars.size(); q-- > 0;) {
        bool found = false;
        for (size_t k = 0; k < nd; ++k)
            if (C.digits[k].var == vars[q]) {
                ws[k] = stride * C.digits[k].w;
                found = true;
            }
        if (!found) return false;
        stride *= P.card[vars[q]];
    }
    std::vector<int32_t> &M = P.meta;
    jin_off = (int64_t)M.size();
    for (int64_t i = 0; i < C.T; ++i) {
        int64_t j = 0;
        for (size_t k = 0; k < nd; ++k)
            if (!C.digits[k].outer) j += ((i / C.digits[k].stride) % C.digits[k].card) * ws[k];
        M.push_back((int32_t)j);
    }
    jout_off = (int64_t)M.size();
    for (int64_t o = 0; o < C.n_tiles; ++o) {
        int64_t j = 0;
        for (size_t k = 0; k < nd; ++k)
            if (C.digits[k].outer) j += ((o / C.digits[k].ostride) % C.digits[k].card) * ws[k];
        M.push_back((int32_t)j);
    }
    return true;
}

struct GatherSpec {
    int32_t edge;
    bool dist;   // ratio of the distribute sweep (else the collect table)
};

// Entries of one group (the tiles one block streams and reduces to one
// partial row) in a launch that streams `level_entries` table entries per
// slot: small levels are cut finer (to spread over the chip), large ones
// coarser (to amortize a block's set-up and its reduction).  It depends on
// one slot's work only, so a query's summation order -- and hence its bits --
// do not depend on how many other queries share the launch.
int64_t group_entries_for(const Plan &P, int64_t level_entries) {
    return std::min<int64_t>(P.tune.group_max, std::max<int64_t>(P.tune.group_min, level_entries / P.tune.group_div));
}

// Blocks over the items [i0, i1) of one launch: each block takes
// consecutive groups of one item, one after the other, so that every block
// moves about the same number of bytes (entries read, plus entries written
// when the pass stores its table) and the launch has about
// `target_blocks` blocks (one round of resident blocks: each block's set-up
// latency is paid once per launch, not once per small group).  Groups per
// block change no summation order.
void emit_tasks(Plan &P, int32_t i0, int32_t i1, int64_t target_blocks) {
    const int64_t tb = std::max<int64_t>(1, target_blocks);
    // work of an entry: its read, plus its write when the pass stores the table
    auto weight = [&](int32_t i) { return P.items[i].dst_kind != JT_DST_NONE ? JT_WRITE_WEIGHT : 1; };
    int64_t entries = 0;
    for (int32_t i = i0; i < i1; ++i) entries += (int64_t)P.items[i].T * P.items[i].n_tiles * weight(i);
    entries *= P.n_slots;
    // Entries per block, rounded up per item: each item adds at most one
    // partly filled block per slot, which the budget leaves room for.  With
    // many (item, slot) pairs every pair is a block anyway; then blocks are
    // rounded down instead.
    const int64_t extra = (int64_t)(i1 - i0) * P.n_slots;
    const bool few = extra < tb / 2;
    const int64_t budget = few ? tb - extra : tb;
    const int64_t floor_ = P.tune.task_min > 0 ? P.tune.task_min : P.tune.group_min;
    int64_t target = std::max<int64_t>(floor_, few ? (entries + budget - 1) / budget : entries / budget);
    // groups per block of item i for a target of entries per block
    auto gpb_for = [&](int32_t i, int64_t tgt) {
        const int64_t ge = (int64_t)P.items[i].tpg * P.items[i].T * weight(i);   // work of a full group
        const int64_t want = few ? (tgt + ge - 1) / ge : tgt / ge;
        return (int32_t)std::max<int64_t>(1, std::min<int64_t>(P.items[i].n_groups, want));
    };
    auto blocks_for = [&](int64_t tgt) {
        int64_t n = 0;
        for (int32_t i = i0; i < i1; ++i) n += (P.items[i].n_groups + gpb_for(i, tgt) - 1) / gpb_for(i, tgt);
        return n * P.n_slots;
    };
    // The floor on a block's work can push a launch past its block target,
    // and the blocks of a second round of resident blocks take about as long
    // again: when the count is up to 2x over, the work per block grows by the
    // overshoot ratio (up to eight times).  A launch only a few blocks over
    // keeps its blocks: doubling every block's work (the next step the
    // groups allow) measured slower than the few extra blocks.
    for (int k = 0; k < 8; ++k) {
        const int64_t n = blocks_for(target);
        if (n <= tb || n >= 2 * tb) break;
        target = target * n / tb + 1;
    }
    for (int32_t i = i0; i < i1; ++i) {
        const int32_t gpb = gpb_for(i, target);
        for (int32_t g0 = 0; g0 < P.items[i].n_groups; g0 += gpb) {
            P.items[i].n_tasks++;
            JtTask t;
            t.item = i;
            t.g0 = g0;
            t.g1 = std::min<int32_t>(P.items[i].n_groups, g0 + gpb);
            t.pad = 0;
            P.tasks.push_back(t);
        }
    }
}

// An output view whose kept-outer configurations hold few tiles each is
// reduced in wave groups (one wave streams a configuration's tiles whole).
bool wave_group_view(int64_t n_rout) { return n_rout <= JT_WAVE_GROUP_TILES; }

int32_t add_item(Plan &P, int32_t c, int32_t src_kind, int64_t src_off, int32_t dst_kind,
                 int64_t dst_off, const std::vector<GatherSpec> &gs, int32_t scale_clique,
                 int32_t out_view, int64_t partial_off, int64_t &bytes_acc, int64_t group_entries) {
    const CliqueInfo &C = P.cl[c];
    JtItem it;
    std::memset(&it, 0, sizeof(it));
    it.clique = c;
    it.T = C.T;
    it.vec = C.vec;
    it.n_tiles = (int32_t)C.n_tiles;
    it.src_kind = src_kind;
    it.src_off = src_off;
    it.dst_kind = dst_kind;
    it.dst_off = dst_off;
    it.gather_base = (int32_t)P.gathers.size();
    it.n_gather = (int32_t)gs.size();
    int32_t lds = 0, n_lds = 0;
    bool lds_open = true;
    for (const GatherSpec &g : gs) {
        const EdgeInfo &E = P.edge[g.edge];
        JtGather G;
        G.view = (c == g.edge) ? E.view_child : E.view_parent;
        G.sep_off = g.dist ? E.sepd_off : E.sepc_off;
        G.ssize = (int32_t)E.ssize;
        G.jin_off = (int32_t)P.views[G.view].jin_off;
        G.jout_off = (int32_t)P.views[G.view].jout_off;
        // a collect message is read through the collect source of the clique
        // that sent it (the edge's other end); a distribute ratio belongs to
        // the launch's slot
        G.src_clique = g.dist ? -1 : (c == g.edge ? P.parent[g.edge] : g.edge);
        // LDS slots start 16-byte aligned: the kernels stage a table with
        // 16-byte global->LDS loads, whose last lane may fill up to three
        // floats of the slot's padding
        if (lds_open && lds + align_up(E.ssize, 4) <= JT_LDS_RATIO_FLOATS) {
            G.lds_off = lds;
            lds += (int32_t)align_up(E.ssize, 4);
            ++n_lds;
        } else {
            lds_open = false;
            G.lds_off = -1;
        }
        P.gathers.push_back(G);
    }
    it.n_gather_lds = n_lds;
    it.lds_floats = lds;
    it.scale_clique = scale_clique;
    it.ev = (src_kind == JT_SRC_INIT) ? 1 : 0;
    it.out_view = out_view;
    it.partial_off = partial_off;
    it.msg = -1;
    const int64_t tiles_per_group = std::max<int64_t>(1, group_entries / C.T);
    if (out_view >= 0) {
        const JtView &V = P.views[out_view];
        it.o_kout_tile = (int32_t)V.kout_tile_off;
        it.o_kout_j = (int32_t)V.kout_j_off;
        it.o_rout_tile = (int32_t)V.rout_tile_off;
        it.o_perm = (int32_t)V.perm_off;
        it.o_clsj = (int32_t)V.clsj_off;
        it.o_n_rout = V.n_rout;
        it.o_n_cls = V.n_cls;
        it.o_m_in = V.m_in;
        it.o_ssize = V.ssize;
        // split partials (nsplit x |phi_S| floats) stay below 1/32 of the
        // table, or one separator table when that is larger
        const int64_t cap = std::max<int64_t>(V.ssize, std::min<int64_t>(kPartialMax, C.size / 32));
        if (wave_group_view(V.n_rout) && V.n_kout > 1) {
            // short groups: one per kept-outer configuration, a wave each,
            // streamed back to back (one partial row, nsplit = 1)
            it.wave_groups = 1;
            it.tpg = V.n_rout;
            it.nsplit = 1;
            it.n_groups = V.n_kout;
        }
        int64_t tpg = std::min<int64_t>(V.n_rout, tiles_per_group);
        int64_t nsplit = (V.n_rout + tpg - 1) / tpg;
        while (nsplit * V.ssize > cap && tpg < V.n_rout) {
            tpg *= 2;
            nsplit = (V.n_rout + tpg - 1) / tpg;
        }
        if (!it.wave_groups) {
            it.tpg = (int32_t)tpg;
            it.nsplit = (int32_t)nsplit;
            it.n_groups = (int32_t)(V.n_kout * nsplit);
        }
    } else {
        const int64_t tpg = std::min<int64_t>(C.n_tiles, tiles_per_group);
        it.tpg = (int32_t)tpg;
        it.nsplit = 1;
        it.n_groups = (int32_t)((C.n_tiles + tpg - 1) / tpg);
    }
    it.pair = (JT_PAIR_TILES && C.T <= JT_TILE_MAX / 2 && C.vec == 4 && !it.wave_groups) ? 1 : 0;
    P.items.push_back(it);
    const int32_t idx = (int32_t)P.items.size() - 1;
    // FP32 table bytes: shared initial tables are read once for all slots
    const int64_t tb = 4 * C.size;
    bytes_acc += (src_kind == JT_SRC_INIT) ? tb : tb * P.n_slots;
    if (dst_kind != JT_DST_NONE) bytes_acc += tb * P.n_slots;
    return idx;
}

int32_t item_nsplit(const Plan &P, int32_t item) { return P.items[item].nsplit; }


// Check, on the host, that every index the kernels derive from the plan
// stays inside its buffer and that the fused schedule's launches respect the
// messages' dataflow.  Run once per compiled tree; a failure here is a
// planner bug and is reported instead of launching anything.
bool verify_plan(const Plan &P, std::string &why) {
    auto bad = [&](const std::string &m) {
        why = "plan check failed: " + m;
        return false;
    };
    const int64_t nm = (int64_t)P.meta.size();
    auto in_meta = [&](int64_t off, int64_t n) { return off >= 0 && n >= 0 && off + n <= nm; };
    auto mmax = [&](int64_t off, int64_t n) {
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i) m = std::max<int64_t>(m, P.meta[off + i]);
        return m;
    };
    auto mmin = [&](int64_t off, int64_t n) {
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i) m = std::min<int64_t>(m, P.meta[off + i]);
        return m;
    };
    for (size_t vi = 0; vi < P.views.size(); ++vi) {
        const JtView &V = P.views[vi];
        if (V.clique < 0 || V.clique >= P.n_cliques) return bad("view clique");
        const CliqueInfo &C = P.cl[V.clique];
        if (C.T < 1 || C.T > JT_TILE_MAX || C.T * C.n_tiles != C.size) return bad("tile shape");
        if ((int64_t)V.n_kout * V.n_rout != C.n_tiles || (int64_t)V.n_cls * V.m_in != C.T) return bad("view counts");
        if (!in_meta(V.jin_off, C.T) || !in_meta(V.jout_off, C.n_tiles) || !in_meta(V.kout_tile_off, V.n_kout) ||
            !in_meta(V.kout_j_off, V.n_kout) || !in_meta(V.rout_tile_off, V.n_rout) || !in_meta(V.perm_off, C.T) ||
            !in_meta(V.clsj_off, V.n_cls))
            return bad("view tables outside metadata");
        if (mmin(V.jin_off, C.T) < 0 || mmin(V.jout_off, C.n_tiles) < 0 || mmin(V.kout_j_off, V.n_kout) < 0 ||
            mmin(V.clsj_off, V.n_cls) < 0 || mmin(V.kout_tile_off, V.n_kout) < 0 || mmin(V.rout_tile_off, V.n_rout) < 0 ||
            mmin(V.perm_off, C.T) < 0)
            return bad("negative index in view");
        if (mmax(V.jin_off, C.T) + mmax(V.jout_off, C.n_tiles) >= V.ssize) return bad("separator index range");
        if (mmax(V.kout_j_off, V.n_kout) + mmax(V.clsj_off, V.n_cls) >= V.ssize) return bad("class index range");
        if (mmax(V.kout_tile_off, V.n_kout) + mmax(V.rout_tile_off, V.n_rout) >= C.n_tiles) return bad("tile range");
        if (mmax(V.perm_off, C.T) >= C.T) return bad("perm range");
    }
    for (size_t ii = 0; ii < P.items.size(); ++ii) {
        const JtItem &it = P.items[ii];
        if (it.clique < 0 || it.clique >= P.n_cliques) return bad("item clique");
        const CliqueInfo &C = P.cl[it.clique];
        if (it.T != C.T || it.n_tiles != C.n_tiles || (it.vec != 1 && it.vec != 4) || (it.vec == 4 && it.T % 4))
            return bad("item shape");
        const int64_t src_lim = it.src_kind == JT_SRC_INIT ? P.init_floats
                                : it.src_kind == JT_SRC_COLL ? P.coll_stride : P.out_stride;
        if (it.src_off < 0 || it.src_off + C.size > src_lim || it.src_off % 4) return bad("item source range");
        if (it.dst_kind != JT_DST_NONE) {
            const int64_t dst_lim = it.dst_kind == JT_DST_COLL ? P.coll_stride : P.out_stride;
            if (it.dst_off < 0 || it.dst_off + C.size > dst_lim || it.dst_off % 4) return bad("item destination range");
        }
        if (it.gather_base < 0 || it.gather_base + it.n_gather > (int32_t)P.gathers.size()) return bad("gather range");
        if (it.n_gather_lds > it.n_gather || it.lds_floats > JT_LDS_RATIO_FLOATS) return bad("LDS budget");
        for (int g = 0; g < it.n_gather; ++g) {
            const JtGather &G = P.gathers[it.gather_base + g];
            if (G.view < 0 || G.view >= (int32_t)P.views.size() || P.views[G.view].clique != it.clique) return bad("gather view");
            if (P.views[G.view].ssize != G.ssize) return bad("gather size");
            if (G.jin_off != P.views[G.view].jin_off || G.jout_off != P.views[G.view].jout_off)
                return bad("gather tables");
            if (G.sep_off < 0 || G.sep_off + (int64_t)G.ssize > P.sep_stride) return bad("gather separator range");
            if ((g < it.n_gather_lds) != (G.lds_off >= 0)) return bad("gather LDS order");
            if (G.src_clique < -1 || G.src_clique >= P.n_cliques) return bad("gather source clique");
            if (G.lds_off >= 0 && (G.lds_off % 4 != 0 || G.lds_off + align_up(G.ssize, 4) > it.lds_floats))
                return bad("gather LDS range");
        }
        if (it.scale_clique >= P.n_cliques) return bad("scale clique");
        if (it.tpg < 1 || it.nsplit < 1 || it.n_groups < 1) return bad("grouping");
        if (it.wave_groups && (it.out_view < 0 || it.nsplit != 1 || it.tpg != it.o_n_rout || !wave_group_view(it.tpg)))
            return bad("wave groups");
        if (it.pair && (it.T > JT_TILE_MAX / 2 || it.vec != 4 || it.wave_groups)) return bad("paired tiles");
        if (it.out_view >= 0) {
            if (it.out_view >= (int32_t)P.views.size()) return bad("output view");
            const JtView &V = P.views[it.out_view];
            if (V.clique != it.clique) return bad("output view clique");
            if (it.o_kout_tile != V.kout_tile_off || it.o_kout_j != V.kout_j_off || it.o_rout_tile != V.rout_tile_off ||
                it.o_perm != V.perm_off || it.o_clsj != V.clsj_off || it.o_n_rout != V.n_rout ||
                it.o_n_cls != V.n_cls || it.o_m_in != V.m_in || it.o_ssize != V.ssize)
                return bad("output view copy");
            if ((int64_t)it.tpg * it.nsplit < V.n_rout || (int64_t)it.tpg * (it.nsplit - 1) >= V.n_rout)
                return bad("split cover");
            if ((int64_t)it.n_groups != (int64_t)V.n_kout * it.nsplit) return bad("group count");
            if (it.partial_off < 0 || it.partial_off + (int64_t)it.nsplit * V.ssize > P.partial_stride)
                return bad("partial range");
        } else {
            if ((int64_t)it.tpg * it.n_groups < C.n_tiles || (int64_t)it.tpg * (it.n_groups - 1) >= C.n_tiles)
                return bad("tile cover");
        }
    }
    for (size_t ii = 0; ii < P.items.size(); ++ii) {
        const JtItem &it = P.items[ii];
        if (it.n_tasks < 1) return bad("item without tasks");
        if (it.msg < -1 || it.msg >= (int32_t)P.msgs.size()) return bad("item message");
        if ((it.msg >= 0) != (it.out_view >= 0)) return bad("item output without message");
        if (it.msg >= 0) {
            const JtMsg &m = P.msgs[it.msg];
            if (m.item != (int32_t)ii || m.partial_off != it.partial_off || m.nsplit != it.nsplit ||
                m.ssize != it.o_ssize)
                return bad("item message fields");
        }
    }
    for (const JtTask &t : P.tasks) {
        if (t.item < 0 || t.item >= (int32_t)P.items.size()) return bad("task item");
        if (t.g0 < 0 || t.g1 > P.items[t.item].n_groups || t.g0 >= t.g1) return bad("task groups");
    }
    if (P.blocks.size() != P.tasks.size()) return bad("block records");
    for (size_t k = 0; k < P.tasks.size(); ++k) {
        const JtTask &t = P.tasks[k];
        const JtBlock &b = P.blocks[k];
        if (b.item != t.item || b.g0 != t.g0 || b.g1 != t.g1 ||
            std::memcmp(&b.it, &P.items[t.item], sizeof(JtItem)) != 0)
            return bad("block record copy");
        for (int g = 0; g < JT_NG_REG && g < b.it.n_gather; ++g)
            if (std::memcmp(&b.g[g], &P.gathers[b.it.gather_base + g], sizeof(JtGather)) != 0)
                return bad("block gather copy");
    }
    {
        int64_t wt = 0, ct = 0;
        int32_t nl = 0;
        for (const Launch &l : P.fused) {
            if (!l.listed) {
                if (l.multi) return bad("multi-slot launch not listed");
                continue;
            }
            if (!P.share) return bad("listed launch outside a batched tree");
            const int64_t cap = l.multi ? 8 * (int64_t)l.chunk_cap
                                        : 8 * (int64_t)l.count * (l.collect ? P.n_regions : P.n_slots);
            if (l.work_off != wt || l.work_cap != cap || l.work_idx != nl || (l.multi && l.collect))
                return bad("listed launch layout");
            if (!l.collect && !l.multi && !l.after_multi)
                for (int32_t t = l.begin; t < l.begin + l.count; ++t)
                    if (!P.item_multi[P.tasks[t].item]) return bad("one-slot launch not ordered after multi-slot launches");
            if (l.multi) {
                if (l.chunk_off != ct || l.chunk_cap < 1) return bad("chunk layout");
                ct += l.chunk_cap;
                for (int32_t t = l.begin; t < l.begin + l.count; ++t) {
                    const int32_t i = P.tasks[t].item;
                    if (!P.item_multi[i]) continue;
                    const JtItem &it = P.items[i];
                    const JtGather &G = P.gathers[it.gather_base];
                    if (it.n_gather != 1 || G.src_clique != -1 || G.lds_off != 0 ||
                        JT_MS * align_up(G.ssize, 4) > l.lds_floats || it.src_kind == JT_SRC_OUT)
                        return bad("multi-slot item");
                }
            }
            wt += l.work_cap;
            ++nl;
        }
        if (wt != P.work_total || nl != P.n_listed || ct != P.chunk_total) return bad("work totals");
    }
    for (const JtMsg &m : P.msgs) {
        if (m.ssize < 1 || m.nsplit < 1) return bad("message shape");
        if (m.partial_off < 0 || m.partial_off + (int64_t)m.nsplit * m.ssize > P.partial_stride) return bad("message partial");
        if (m.from < 0 || m.from >= P.n_cliques) return bad("message source");
        if (m.kind == JT_MSG_COLLECT || m.kind == JT_MSG_DIST || m.kind == JT_MSG_PLAIN) {
            if (m.edge < 0 || m.edge >= P.n_cliques || P.parent[m.edge] < 0) return bad("message edge");
            if (m.ssize != P.edge[m.edge].ssize) return bad("message separator size");
            if (m.sepc_off + (int64_t)m.ssize > P.sep_stride || m.sepd_off + (int64_t)m.ssize > P.sep_stride)
                return bad("message separator range");
            if (m.to < 0 || m.to >= P.n_cliques) return bad("message target");
        }
        if (m.child_base < 0 || 2 * ((int64_t)m.child_base + m.n_children) > (int64_t)P.child_edges.size())
            return bad("children range");
        for (int32_t k = 0; k < m.n_children; ++k) {
            const int32_t e = P.child_edges[2 * (m.child_base + k)], ch = P.child_edges[2 * (m.child_base + k) + 1];
            if (e < 0 || e >= P.n_cliques || ch < 0 || ch >= P.n_cliques || P.iedge[ch] != e) return bad("child pair");
        }
    }
    for (const std::vector<Launch> *L : {&P.fused, &P.plain})
        for (const Launch &l : *L) {
            if (l.is_pass == 1 && (l.begin < 0 || l.begin + l.count > (int32_t)P.tasks.size())) return bad("launch tasks");
            if (l.is_pass == 1) {
                if (l.lds_floats < JT_FIN_LDS_FLOATS || l.lds_floats > JT_LDS_RATIO_FLOATS) return bad("launch LDS");
                for (int32_t t = l.begin; t < l.begin + l.count; ++t)
                    if (P.items[P.tasks[t].item].lds_floats > l.lds_floats) return bad("launch LDS of an item");
            }
        }
    for (int32_t c = 0; c < P.n_cliques; ++c)
        for (const VDigit &d : P.cl[c].digits)
            if (d.card < 1 || (d.outer ? d.ostride : d.stride) < 1) return bad("digit shape");
    // lanes: every launch's items belong to the launch's lane; the root's
    // launches are on the bound stream, the collect one joins, the distribute
    // one forks
    if (P.n_lanes < 0 || P.n_lanes > JT_MAX_LANES || (int32_t)P.lane.size() != P.n_cliques) return bad("lanes");
    for (const Launch &l : P.fused) {
        if (l.lane < -1 || l.lane >= std::max(1, P.n_lanes) || (P.n_lanes == 0 && l.lane != -1)) return bad("launch lane");
        for (int32_t t = l.begin; t < l.begin + l.count; ++t)
            if (P.lane[P.items[P.tasks[t].item].clique] != l.lane) return bad("item lane");
        const bool root = l.count > 0 && P.items[P.tasks[l.begin].item].clique == P.root;
        if (P.n_lanes > 0 && root != (l.join_before || l.fork_after)) return bad("lane sync");
    }
    for (const Launch &l : P.plain)
        if (l.lane != -1 || l.join_before || l.fork_after) return bad("plain lanes");
    // dataflow of the fused schedule, in launch order: a pass reads only
    // messages finalized by an earlier launch; a clique's collect passes
    // (pre-passes, then its own) run one per launch, the one reading its
    // initial table first; a distribute pass reading the collect table runs
    // after the last of them
    {
        std::map<int32_t, int32_t> by_sepc, by_sepd;   // separator table -> message writing it
        for (size_t mi = 0; mi < P.msgs.size(); ++mi) {
            const JtMsg &m = P.msgs[mi];
            if (m.kind == JT_MSG_COLLECT) by_sepc[m.sepc_off] = (int32_t)mi;
            if (m.kind == JT_MSG_DIST) by_sepd[m.sepd_off] = (int32_t)mi;
        }
        std::vector<int32_t> fin(P.msgs.size(), -1);        // launch finalizing each message
        std::vector<int32_t> coll_last(P.n_cliques, -1);    // launch of a clique's latest collect pass
        for (size_t li = 0; li < P.fused.size(); ++li) {
            const Launch &l = P.fused[li];
            if (l.is_pass != 1) continue;
            std::set<int32_t> seen;
            for (int32_t t = l.begin; t < l.begin + l.count; ++t) {
                const int32_t i = P.tasks[t].item;
                if (!seen.insert(i).second) continue;
                const JtItem &it = P.items[i];
                for (int32_t g = 0; g < it.n_gather; ++g) {
                    const JtGather &G = P.gathers[it.gather_base + g];
                    const std::map<int32_t, int32_t> &mp = G.src_clique < 0 ? by_sepd : by_sepc;
                    const auto f = mp.find(G.sep_off);
                    if (f == mp.end()) return bad("gathered table without a message");
                    if (fin[f->second] < 0 || fin[f->second] >= (int32_t)li) return bad("message read before it is finalized");
                }
                if (l.collect && it.dst_kind == JT_DST_COLL) {
                    const int32_t prev = coll_last[it.clique];
                    if ((it.src_kind == JT_SRC_INIT) != (prev < 0)) return bad("collect passes out of order");
                    if (prev >= (int32_t)li) return bad("two collect passes of a clique in one launch");
                    coll_last[it.clique] = (int32_t)li;
                }
                if (!l.collect && it.src_kind == JT_SRC_COLL &&
                    (coll_last[it.clique] < 0 || coll_last[it.clique] >= (int32_t)li))
                    return bad("collect table read before it is complete");
            }
            for (int32_t i : seen)
                if (P.items[i].msg >= 0) fin[P.items[i].msg] = (int32_t)li;
        }
    }
    return true;
}

}  // namespace

bool check_plan(const Plan &P, std::string &why) { return verify_plan(P, why); }

jt_status compile_plan(const jt_tree_desc *desc, Plan &P, std::string &err, const std::vector<FamilyReq> *families,
                       int64_t cpt_total) {
    if (!desc) return fail(err, JT_E_ARG, "desc is NULL");
    const int32_t nv = desc->n_vars, nc = desc->n_cliques;
    if (nv < 0) return fail(err, JT_E_ARG, "n_vars < 0");
    if (nc < 1) return fail(err, JT_E_ARG, "n_cliques < 1");
    if (desc->n_slots < 1 || desc->n_slots > (1 << 20)) return fail(err, JT_E_ARG, "n_slots out of range");
    if ((nv > 0 && !desc->card) || !desc->clique_off || !desc->clique_vars || !desc->parent)
        return fail(err, JT_E_ARG, "NULL array in desc");
    P = Plan();
    {
        jt_tuning d{JT_GROUP_MIN, JT_GROUP_MAX, JT_GROUP_DIV, JT_TARGET_BLOCKS, JT_LANES_ENABLED ? JT_MAX_LANES : 1, 0};
        if (desc->tuning) {
            const jt_tuning &u = *desc->tuning;
            if (u.group_min < 0 || u.group_max < 0 || u.group_div < 0 || u.target_blocks < 0 || u.max_lanes < 0 ||
                u.max_lanes > JT_MAX_LANES || u.group_div > (1 << 20) || u.target_blocks > (1 << 20) || u.task_min < 0)
                return fail(err, JT_E_ARG, "tuning value out of range");
            if (u.group_min) d.group_min = u.group_min;
            if (u.group_max) d.group_max = u.group_max;
            if (u.group_div) d.group_div = u.group_div;
            if (u.target_blocks) d.target_blocks = u.target_blocks;
            if (u.max_lanes) d.max_lanes = u.max_lanes;
            if (u.task_min) d.task_min = u.task_min;
        }
        if (d.group_min > d.group_max) return fail(err, JT_E_ARG, "tuning: group_min above group_max");
        if (!JT_LANES_ENABLED && d.max_lanes > 1)
            return fail(err, JT_E_ARG, "tuning: lanes are disabled (max_lanes must be 1)");
        P.tune = d;
    }
    P.n_vars = nv;
    P.n_cliques = nc;
    P.n_slots = desc->n_slots;
    P.share = P.n_slots >= 2 ? 1 : 0;
    P.n_regions = P.n_slots + P.share;
    P.card.assign(desc->card, desc->card + nv);
    P.parent.assign(desc->parent, desc->parent + nc);
    for (int32_t v = 0; v < nv; ++v)
        if (P.card[v] < 1) return fail(err, JT_E_ARG, "card[" + std::to_string(v) + "] < 1");
    if (desc->clique_off[0] != 0) return fail(err, JT_E_ARG, "clique_off[0] != 0");
    P.cl.resize(nc);
    std::vector<std::vector<int32_t>> sorted_vars(nc);
    std::vector<int32_t> stamp(nv, -1);
    for (int32_t c = 0; c < nc; ++c) {
        const int64_t a = desc->clique_off[c], b = desc->clique_off[c + 1];
        if (b < a || b - a > 64) return fail(err, JT_E_ARG, "clique " + std::to_string(c) + ": bad variable count");
        int64_t size = 1;
        for (int64_t k = a; k < b; ++k) {
            const int32_t v = desc->clique_vars[k];
            if (v < 0 || v >= nv) return fail(err, JT_E_ARG, "clique " + std::to_string(c) + ": variable out of range");
            if (stamp[v] == c) return fail(err, JT_E_ARG, "clique " + std::to_string(c) + ": repeated variable");
            stamp[v] = c;
            size *= P.card[v];
            if (size > std::numeric_limits<int32_t>::max())
                return fail(err, JT_E_TOO_LARGE, "clique " + std::to_string(c) + ": table has 2^31 or more entries");
            P.cl[c].vars.push_back(v);
        }
        sorted_vars[c] = P.cl[c].vars;
        std::sort(sorted_vars[c].begin(), sorted_vars[c].end());
    }
    // one root, parents in range, every clique reachable from the root
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t p = P.parent[c];
        if (p == -1) {
            if (P.root >= 0) return fail(err, JT_E_NOT_JUNCTION_TREE, "more than one root");
            P.root = c;
        } else if (p < 0 || p >= nc || p == c) {
            return fail(err, JT_E_NOT_JUNCTION_TREE, "parent of clique " + std::to_string(c) + " out of range");
        }
    }
    if (P.root < 0) return fail(err, JT_E_NOT_JUNCTION_TREE, "no root (parent == -1)");
    for (int32_t c = 0; c < nc; ++c)
        if (P.parent[c] >= 0) P.cl[P.parent[c]].children.push_back(c);
    std::vector<int32_t> bfs;
    bfs.reserve(nc);
    bfs.push_back(P.root);
    for (size_t h = 0; h < bfs.size(); ++h)
        for (int32_t ch : P.cl[bfs[h]].children) {
            P.cl[ch].depth = P.cl[bfs[h]].depth + 1;
            bfs.push_back(ch);
        }
    if ((int32_t)bfs.size() != nc) return fail(err, JT_E_NOT_JUNCTION_TREE, "parent links contain a cycle");
    // running intersection: the cliques holding a variable are connected
    {
        std::vector<std::vector<int32_t>> holders(nv);
        for (int32_t c = 0; c < nc; ++c)
            for (int32_t v : P.cl[c].vars) holders[v].push_back(c);
        std::vector<int32_t> seen(nc, -1), queue;
        for (int32_t v = 0; v < nv; ++v) {
            if (holders[v].empty()) continue;
            queue.assign(1, holders[v][0]);
            seen[holders[v][0]] = v;
            for (size_t h = 0; h < queue.size(); ++h) {
                const int32_t x = queue[h];
                auto visit = [&](int32_t y) {
                    if (y >= 0 && seen[y] != v && has_var(sorted_vars[y], v)) {
                        seen[y] = v;
                        queue.push_back(y);
                    }
                };
                visit(P.parent[x]);
                for (int32_t ch : P.cl[x].children) visit(ch);
            }
            if (queue.size() != holders[v].size())
                return fail(err, JT_E_NOT_JUNCTION_TREE,
                            "running intersection violated for variable " + std::to_string(v));
        }
    }
    // Re-root at a center of the tree (the middle of a longest path): the
    // collect / distribute sweeps then have the fewest levels.  Any clique
    // may serve as the root of Algorithms 2-4; the messages between two
    // cliques, the posteriors and P(e) do not depend on the choice.
    {
        std::vector<std::vector<int32_t>> adj(nc);
        for (int32_t c = 0; c < nc; ++c)
            if (P.parent[c] >= 0) {
                adj[c].push_back(P.parent[c]);
                adj[P.parent[c]].push_back(c);
            }
        for (auto &a : adj) std::sort(a.begin(), a.end());
        std::vector<int32_t> dist(nc), from(nc);
        auto farthest = [&](int32_t s0) {
            std::fill(dist.begin(), dist.end(), -1);
            std::vector<int32_t> q{s0};
            dist[s0] = 0;
            from[s0] = -1;
            int32_t best = s0;
            for (size_t h = 0; h < q.size(); ++h) {
                const int32_t x = q[h];
                if (dist[x] > dist[best]) best = x;
                for (int32_t y : adj[x])
                    if (dist[y] < 0) {
                        dist[y] = dist[x] + 1;
                        from[y] = x;
                        q.push_back(y);
                    }
            }
            return best;
        };
        const int32_t a = farthest(P.root);
        const int32_t b = farthest(a);
        int32_t center = b;
        for (int32_t k = 0; k < dist[b] / 2; ++k) center = from[center];
        P.user_root = P.root;
        P.root = center;
        P.iparent.assign(nc, -1);
        P.iedge.assign(nc, -1);
        for (int32_t c = 0; c < nc; ++c) {
            P.cl[c].children.clear();
            P.cl[c].depth = 0;
            P.cl[c].height = 0;
        }
        bfs.assign(1, P.root);
        std::vector<char> seen(nc, 0);
        seen[P.root] = 1;
        for (size_t h = 0; h < bfs.size(); ++h) {
            const int32_t x = bfs[h];
            for (int32_t y : adj[x]) {
                if (seen[y]) continue;
                seen[y] = 1;
                P.iparent[y] = x;
                P.iedge[y] = (P.parent[y] == x) ? y : x;   // the caller's child end of the edge
                P.cl[x].children.push_back(y);
                P.cl[y].depth = P.cl[x].depth + 1;
                bfs.push_back(y);
            }
        }
    }
    for (size_t h = bfs.size(); h-- > 0;) {
        const int32_t c = bfs[h];
        const int32_t p = P.iparent[c];
        if (p >= 0) P.cl[p].height = std::max(P.cl[p].height, P.cl[c].height + 1);
    }
    P.height = P.cl[P.root].height;
    for (int32_t c = 0; c < nc; ++c) P.depth = std::max(P.depth, P.cl[c].depth);
    P.home.assign(nv, -1);
    for (int32_t c = nc - 1; c >= 0; --c)
        for (int32_t v : P.cl[c].vars) P.home[v] = c;

    // tiles, table regions
    for (int32_t c = 0; c < nc; ++c) {
        shape_clique(P.card, P.cl[c]);
        P.total_entries += P.cl[c].size;
        if (P.cl[c].n_tiles > (int64_t(1) << 26))
            return fail(err, JT_E_TOO_LARGE, "clique " + std::to_string(c) + ": too many tiles");
    }
    for (int32_t c = 0; c < nc; ++c) {
        CliqueInfo &C = P.cl[c];
        C.init_off = P.init_floats;
        P.init_floats += align_up(C.size, kAlignFloats);
        C.out_off = P.out_stride;
        P.out_stride += align_up(C.size, kAlignFloats);
        if (!C.children.empty()) {
            C.coll_off = P.coll_stride;
            P.coll_stride += align_up(C.size, kAlignFloats);
        }
    }
    // lanes: the root's subtrees, largest first, each to the lane with the
    // least work so far (ties to the lower lane)
    {
        P.lane.assign(nc, -1);
        const std::vector<int32_t> &rk = P.cl[P.root].children;
        std::vector<int64_t> sub(nc, 0);
        for (size_t h = bfs.size(); h-- > 0;) {
            const int32_t c = bfs[h];
            sub[c] += P.cl[c].size;
            if (P.iparent[c] >= 0) sub[P.iparent[c]] += sub[c];
        }
        P.n_lanes = (rk.size() >= 2 && P.tune.max_lanes >= 2)
                        ? (int32_t)std::min<size_t>((size_t)P.tune.max_lanes, rk.size())
                        : 0;
        if (P.n_lanes > 0) {
            std::vector<int32_t> order(rk.begin(), rk.end());
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return sub[a] > sub[b]; });
            std::vector<int64_t> load(P.n_lanes, 0);
            for (int32_t ch : order) {
                const int32_t l = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
                load[l] += sub[ch];
                P.lane[ch] = l;
            }
            for (int32_t c : bfs)
                if (c != P.root && P.lane[c] < 0) P.lane[c] = P.lane[P.iparent[c]];
        }
    }
    // separators: ascending variable id, row-major, last fastest
    P.edge.resize(nc);
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t p = P.parent[c];
        if (p < 0) continue;
        EdgeInfo &E = P.edge[c];
        std::set_intersection(sorted_vars[c].begin(), sorted_vars[c].end(), sorted_vars[p].begin(),
                              sorted_vars[p].end(), std::back_inserter(E.vars));
        E.sst.assign(E.vars.size(), 1);
        int64_t s = 1;
        for (size_t k = E.vars.size(); k-- > 0;) {
            E.sst[k] = s;
            s *= P.card[E.vars[k]];
        }
        E.ssize = s;
        E.sepc_off = (int32_t)P.sep_stride;
        P.sep_stride += align_up(s, kAlignFloats);
        E.sepd_off = (int32_t)P.sep_stride;
        P.sep_stride += align_up(s, kAlignFloats);
        if (P.sep_stride > std::numeric_limits<int32_t>::max())
            return fail(err, JT_E_TOO_LARGE, "separator tables exceed 2^31 floats");
        P.entries_per_sweep += P.cl[c].size + P.cl[p].size;
    }
    // views: every clique through each incident separator and through nothing
    for (int32_t c = 0; c < nc; ++c) {
        if (P.parent[c] >= 0) {
            P.edge[c].view_child = build_view(P, c, c);
            P.edge[c].view_parent = build_view(P, P.parent[c], c);
        }
        P.cl[c].total_view = build_view(P, c, -1);
        if ((int64_t)P.meta.size() > kMaxMeta) return fail(err, JT_E_TOO_LARGE, "index metadata too large");
    }
    // families of a Bayesian-network tree: their mapping into their cliques,
    // sorted by clique (stable: ascending variable within a clique)
    if (families) {
        std::vector<FamilyReq> fr(*families);
        std::stable_sort(fr.begin(), fr.end(), [](const FamilyReq &a, const FamilyReq &b) { return a.clique < b.clique; });
        P.fam_rng.assign((size_t)nc + 1, 0);
        for (const FamilyReq &f : fr) {
            if (f.clique < 0 || f.clique >= nc) return fail(err, JT_E_ARG, "family clique out of range");
            JtFamily F;
            std::memset(&F, 0, sizeof(F));
            if (!build_projection(P, f.clique, f.vars, F.jin_off, F.jout_off))
                return fail(err, JT_E_ARG, "family of variable " + std::to_string(f.var) + " not in its clique");
            int64_t fs = 1;
            for (int32_t v : f.vars) fs *= P.card[v];
            F.cpt_off = f.cpt_off;
            F.mu_off = P.fam_mu_total;
            F.clique = f.clique;
            F.fsize = (int32_t)fs;
            F.var = f.var;
            P.fam_mu_total += P.cl[f.clique].size;
            P.fam.push_back(F);
            P.fam_rng[f.clique + 1]++;
        }
        for (int32_t c = 0; c < nc; ++c) P.fam_rng[c + 1] += P.fam_rng[c];
        P.cpt_total = cpt_total;
        for (int32_t c = 0; c < nc; ++c) {
            JtCliqueShape sh;
            sh.init_off = P.cl[c].init_off;
            sh.n_tiles = P.cl[c].n_tiles;
            sh.size = P.cl[c].size;
            sh.T = P.cl[c].T;
            sh.pad = 0;
            P.cshape.push_back(sh);
            P.max_tiles = std::max<int64_t>(P.max_tiles, sh.n_tiles);
        }
        for (const JtFamily &F : P.fam) P.max_fsize = std::max<int64_t>(P.max_fsize, F.fsize);
        if ((int64_t)P.meta.size() > kMaxMeta) return fail(err, JT_E_TOO_LARGE, "index metadata too large");
    }
    // clique c seen through edge e (c is one of its two ends)
    auto view_of = [&](int32_t c, int32_t e) { return c == e ? P.edge[e].view_child : P.edge[e].view_parent; };
    for (int32_t c = 0; c < nc; ++c)
        if (P.iparent[c] >= 0) P.cl[c].parent_view = view_of(c, P.iedge[c]);
    // ---------------- fused level schedule ----------------
    auto add_partial = [&](int64_t floats) {
        const int64_t off = P.partial_stride;
        P.partial_stride += align_up(floats, kAlignFloats);
        return off;
    };
    std::vector<std::vector<int32_t>> by_height(P.height + 1), by_depth(P.depth + 1);
    for (int32_t c = 0; c < nc; ++c) {
        by_height[P.cl[c].height].push_back(c);
        by_depth[P.cl[c].depth].push_back(c);
    }
    int64_t bytes = 0;
    // cliques of one level, lane by lane (the root is alone on its level)
    auto split_lanes = [&](const std::vector<int32_t> &level) {
        std::vector<std::vector<int32_t>> out(std::max(1, P.n_lanes) + 1);
        for (int32_t c : level) out[P.lane[c] + 1].push_back(c);
        return out;   // [0]: the root; [l + 1]: lane l
    };
    // a launch of a lane gets its share of one round of resident blocks
    auto lane_target = [&](int64_t part, int64_t level_total) {
        const int64_t tb = P.tune.target_blocks;
        if (P.n_lanes == 0 || level_total <= 0) return tb;
        return std::max<int64_t>(tb / 8, tb * part / level_total);
    };
    auto push_launch = [&](int32_t t0, int32_t lane, int32_t join, int32_t fork) {
        Launch l;
        l.is_pass = 1;
        l.begin = t0;
        l.count = (int32_t)P.tasks.size() - t0;
        l.lane = lane;
        l.join_before = join;
        l.fork_after = fork;
        P.fused.push_back(l);
    };
    // A pass multiplies up to JT_NG_REG ratio tables with indices held in
    // registers; further ones are looked up tile by tile (a chain of
    // dependent loads per tile).  A clique with more children therefore
    // absorbs the messages of its earliest-finished children in pre-passes at
    // earlier collect levels: JT_NG_REG messages each, the first reading the
    // initial table (evidence entered), every one writing the collect table,
    // each at a level after its children's and the previous pre-pass's and
    // before the clique's own pass, which multiplies the rest and sums into
    // the separator.  Only for tables of at most 2^22 entries: a pre-pass
    // reads and writes the whole table once more, which on larger tables
    // costs more than the lookups it saves (measured on a 2^23-entry root).
    // (Not with lanes: a pre-pass would join them early.)
    struct PrePass {
        int32_t clique;
        bool first;
        std::vector<int32_t> children;
    };
    std::vector<std::vector<PrePass>> pre_at((size_t)P.height + 1);
    std::vector<std::vector<int32_t>> final_children(nc);
    std::vector<char> absorbed_before(nc, 0);
    for (int32_t c = 0; c < nc; ++c) {
        const std::vector<int32_t> &kids = P.cl[c].children;
        final_children[c] = kids;
        if ((int32_t)kids.size() <= JT_NG_REG || P.n_lanes > 0 || P.cl[c].size > (int64_t(1) << 22)) continue;
        std::vector<int32_t> by_h = kids;
        std::stable_sort(by_h.begin(), by_h.end(),
                         [&](int32_t a, int32_t b) { return P.cl[a].height < P.cl[b].height; });
        const size_t n_pre = kids.size() - JT_NG_REG;   // at most this many absorbed early
        std::vector<char> early(nc, 0);
        int32_t prev = -1;
        for (size_t k0 = 0; k0 < n_pre; k0 += JT_NG_REG) {
            const size_t k1 = std::min(n_pre, k0 + JT_NG_REG);
            const int32_t level = std::max(prev + 1, P.cl[by_h[k1 - 1]].height + 1);
            if (level >= P.cl[c].height) break;
            PrePass pp;
            pp.clique = c;
            pp.first = prev < 0;
            pp.children.assign(by_h.begin() + (std::ptrdiff_t)k0, by_h.begin() + (std::ptrdiff_t)k1);
            for (int32_t ch : pp.children) early[ch] = 1;
            pre_at[level].push_back(std::move(pp));
            prev = level;
        }
        if (prev < 0) continue;
        absorbed_before[c] = 1;
        final_children[c].clear();
        for (int32_t ch : kids)
            if (!early[ch]) final_children[c].push_back(ch);
    }
    for (int32_t h = 0; h <= P.height; ++h) {
        int64_t level_entries = 0;
        for (int32_t c : by_height[h]) level_entries += P.cl[c].size;
        for (const PrePass &pp : pre_at[h]) level_entries += P.cl[pp.clique].size;
        const int64_t ge = group_entries_for(P, level_entries);
        const auto parts = split_lanes(by_height[h]);
        for (size_t li = 0; li < parts.size(); ++li) {
        std::vector<const PrePass *> pre_here;
        for (const PrePass &pp : pre_at[h])
            if ((size_t)(P.lane[pp.clique] + 1) == li) pre_here.push_back(&pp);
        if (parts[li].empty() && pre_here.empty()) continue;
        const int32_t t0 = (int32_t)P.tasks.size(), m0 = (int32_t)P.msgs.size(), i0 = (int32_t)P.items.size();
        int64_t part_entries = 0;
        for (int32_t c : parts[li]) part_entries += P.cl[c].size;
        for (const PrePass *pp : pre_here) part_entries += P.cl[pp->clique].size;
        for (const PrePass *pp : pre_here) {
            const CliqueInfo &C = P.cl[pp->clique];
            std::vector<GatherSpec> gs;
            for (int32_t ch : pp->children) gs.push_back({P.iedge[ch], false});
            add_item(P, pp->clique, pp->first ? JT_SRC_INIT : JT_SRC_COLL, pp->first ? C.init_off : C.coll_off,
                     JT_DST_COLL, C.coll_off, gs, -1, -1, 0, bytes, ge);
        }
        std::vector<JtMsg> level_msgs;
        for (int32_t c : parts[li]) {
            const CliqueInfo &C = P.cl[c];
            std::vector<GatherSpec> gs;
            for (int32_t ch : final_children[c]) gs.push_back({P.iedge[ch], false});
            const bool is_root = (c == P.root);
            const int32_t view = is_root ? C.total_view : C.parent_view;
            // partial size is known once the item's split is chosen: add the
            // item first with a placeholder, then patch its offset.
            const int32_t it = absorbed_before[c]
                                   ? add_item(P, c, JT_SRC_COLL, C.coll_off, JT_DST_COLL, C.coll_off, gs, -1, view, 0,
                                              bytes, ge)
                                   : add_item(P, c, JT_SRC_INIT, C.init_off,
                                              C.children.empty() ? JT_DST_NONE : JT_DST_COLL, C.coll_off, gs, -1, view,
                                              0, bytes, ge);
            const int64_t ss = P.views[view].ssize;
            const int64_t poff = add_partial(ss * item_nsplit(P, it));
            P.items[it].partial_off = poff;
            JtMsg m;
            std::memset(&m, 0, sizeof(m));
            m.item = it;
            P.items[it].msg = m0 + (int32_t)level_msgs.size();
            m.kind = is_root ? JT_MSG_TOTAL : JT_MSG_COLLECT;
            m.edge = is_root ? -1 : P.iedge[c];
            m.from = c;
            m.to = is_root ? -1 : P.iparent[c];
            m.ssize = (int32_t)ss;
            m.nsplit = P.items[it].nsplit;
            m.partial_off = poff;
            m.child_base = (int32_t)P.child_edges.size() / 2;
            m.n_children = (int32_t)C.children.size();
            for (int32_t ch : C.children) {
                P.child_edges.push_back(P.iedge[ch]);
                P.child_edges.push_back(ch);
            }
            m.sepc_off = is_root ? 0 : P.edge[P.iedge[c]].sepc_off;
            m.sepd_off = is_root ? 0 : P.edge[P.iedge[c]].sepd_off;
            level_msgs.push_back(m);
        }
        emit_tasks(P, i0, (int32_t)P.items.size(), lane_target(part_entries, level_entries));
        for (const JtMsg &m : level_msgs) P.msgs.push_back(m);
        // the root's collect pass first joins every lane
        push_launch(t0, (int32_t)li - 1, li == 0 && P.n_lanes > 0 ? 1 : 0, 0);
        P.fused.back().collect = 1;
        }
    }
    for (int32_t d = 0; d <= P.depth; ++d) {
        int64_t level_entries = 0;
        for (int32_t c : by_depth[d])
            level_entries += P.cl[c].size * std::max<int64_t>(1, (int64_t)P.cl[c].children.size());
        const int64_t ge = group_entries_for(P, level_entries);
        const auto parts = split_lanes(by_depth[d]);
        for (size_t li = 0; li < parts.size(); ++li) {
        if (parts[li].empty()) continue;
        const int32_t t0 = (int32_t)P.tasks.size(), m0 = (int32_t)P.msgs.size(), i0 = (int32_t)P.items.size();
        int64_t part_entries = 0;
        for (int32_t c : parts[li])
            part_entries += P.cl[c].size * std::max<int64_t>(1, (int64_t)P.cl[c].children.size());
        std::vector<JtMsg> level_msgs;
        for (int32_t c : parts[li]) {
            const CliqueInfo &C = P.cl[c];
            std::vector<GatherSpec> gs;
            if (c != P.root) gs.push_back({P.iedge[c], true});
            const bool leaf = C.children.empty();
            const int32_t src_kind = leaf ? JT_SRC_INIT : JT_SRC_COLL;
            const int64_t src_off = leaf ? C.init_off : C.coll_off;
            if (leaf) {
                add_item(P, c, src_kind, src_off, JT_DST_OUT, C.out_off, gs, c, -1, 0, bytes, ge);
                continue;
            }
            for (size_t k = 0; k < C.children.size(); ++k) {
                const int32_t ch = C.children[k];
                const int32_t e = P.iedge[ch];
                const int32_t view = view_of(c, e);
                const int32_t it = add_item(P, c, src_kind, src_off, k == 0 ? JT_DST_OUT : JT_DST_NONE,
                                            C.out_off, gs, c, view, 0, bytes, ge);
                const int64_t ss = P.views[view].ssize;
                const int64_t poff = add_partial(ss * item_nsplit(P, it));
                P.items[it].partial_off = poff;
                JtMsg m;
                std::memset(&m, 0, sizeof(m));
                m.item = it;
                P.items[it].msg = m0 + (int32_t)level_msgs.size();
                m.kind = JT_MSG_DIST;
                m.edge = e;
                m.from = c;
                m.to = ch;
                m.ssize = (int32_t)ss;
                m.nsplit = P.items[it].nsplit;
                m.partial_off = poff;
                m.sepc_off = P.edge[e].sepc_off;
                m.sepd_off = P.edge[e].sepd_off;
                level_msgs.push_back(m);
            }
        }
        emit_tasks(P, i0, (int32_t)P.items.size(), lane_target(part_entries, level_entries));
        for (const JtMsg &m : level_msgs) P.msgs.push_back(m);
        // after the root's distribute pass every lane waits for it
        push_launch(t0, (int32_t)li - 1, 0, li == 0 && P.n_lanes > 0 ? 1 : 0);
        }
    }
    P.bytes_fused = bytes;
    // Batched trees: every fused launch walks a per-propagation work list.
    //  * collect: the evidence-free slot's tasks plus the (task, slot) pairs
    //    whose clique has evidence of that slot below it;
    //  * distribute: a multi-slot launch over sets of up to JT_MS slots that
    //    read the same evidence-free source table (one tile load serves them
    //    all), then a launch over the remaining (task, slot) pairs.
    // Lists are sized for the worst case (every task of every region; a
    // multi-slot list also for its per-XCD padding).
    P.item_multi.assign(P.items.size(), 0);
    if (P.share) {
        for (const Launch &l : P.fused) {
            if (l.collect || l.count == 0) continue;
            for (int32_t t = l.begin; t < l.begin + l.count; ++t) {
                const int32_t i = P.tasks[t].item;
                const JtItem &it = P.items[i];
                if (it.n_gather != 1) continue;
                const JtGather &G = P.gathers[it.gather_base];
                if (G.src_clique != -1 || JT_MS * align_up(G.ssize, 4) > JT_LDS_RATIO_FLOATS) continue;
                P.item_multi[i] = 1;
            }
        }
        std::vector<Launch> L2;
        // sets of JT_MS / 2 slots on short levels
        const int64_t per_task_chunks = (P.n_slots + JT_MS / 2 - 1) / (JT_MS / 2);
        for (Launch l : P.fused) {
            if (l.count == 0) {
                L2.push_back(l);
                continue;
            }
            l.listed = 1;
            // lists hold 8 x the entries: room for the per-XCD padding
            if (l.collect) {
                l.work_cap = (int32_t)std::min<int64_t>(8 * (int64_t)l.count * P.n_regions, INT32_MAX);
                if (8 * (int64_t)l.count * P.n_regions > l.work_cap) return fail(err, JT_E_TOO_LARGE, "work list too long");
                L2.push_back(l);
                continue;
            }
            int64_t eligible = 0;
            for (int32_t t = l.begin; t < l.begin + l.count; ++t) eligible += P.item_multi[P.tasks[t].item];
            if (eligible > 0) {
                Launch m = l;
                m.multi = 1;
                if (eligible * per_task_chunks * 8 > INT32_MAX) return fail(err, JT_E_TOO_LARGE, "work list too long");
                m.chunk_cap = (int32_t)(eligible * per_task_chunks);
                m.work_cap = 8 * m.chunk_cap;
                L2.push_back(m);
            }
            l.work_cap = (int32_t)std::min<int64_t>(8 * (int64_t)l.count * P.n_slots, INT32_MAX);
            if (8 * (int64_t)l.count * P.n_slots > l.work_cap) return fail(err, JT_E_TOO_LARGE, "work list too long");
            L2.push_back(l);
        }
        P.fused = L2;
        for (Launch &l : P.fused) {
            if (!l.collect && !l.multi)
                for (int32_t t = l.begin; t < l.begin + l.count; ++t)
                    if (!P.item_multi[P.tasks[t].item]) l.after_multi = 1;
            if (!l.listed) continue;
            l.work_off = P.work_total;
            l.work_idx = P.n_listed++;
            P.work_total += l.work_cap;
            if (l.multi) {
                l.chunk_off = P.chunk_total;
                P.chunk_total += l.chunk_cap;
            }
        }
    }

    // Tables live in the output region and are updated in place.
    bytes = 0;
    {
        const int32_t t0 = (int32_t)P.tasks.size();
        const int32_t i0 = (int32_t)P.items.size();
        const int64_t ge = group_entries_for(P, P.total_entries);
        for (int32_t c = 0; c < nc; ++c)
            add_item(P, c, JT_SRC_INIT, P.cl[c].init_off, JT_DST_OUT, P.cl[c].out_off, {}, -1, -1, 0, bytes, ge);
        emit_tasks(P, i0, (int32_t)P.items.size(), P.tune.target_blocks);
        P.plain_reset_task_begin = t0;
        P.plain_reset_task_count = (int32_t)P.tasks.size() - t0;
        P.plain.push_back({2, 0, 0});   // separators := 1, log-scales := 0
        P.plain.push_back({1, t0, P.plain_reset_task_count});
    }
    auto plain_message = [&](int32_t e, int32_t from, int32_t to) {
        const int32_t view_from = (from == e) ? P.edge[e].view_child : P.edge[e].view_parent;
        const int32_t t0 = (int32_t)P.tasks.size();
        const int32_t it = add_item(P, from, JT_SRC_OUT, P.cl[from].out_off, JT_DST_NONE, 0, {}, -1,
                                    view_from, 0, bytes, group_entries_for(P, P.cl[from].size));
        emit_tasks(P, it, it + 1, P.tune.target_blocks);
        const int64_t ss = P.edge[e].ssize;
        const int64_t poff = add_partial(ss * item_nsplit(P, it));
        P.items[it].partial_off = poff;
        P.plain.push_back({1, t0, (int32_t)P.tasks.size() - t0});
        JtMsg m;
        std::memset(&m, 0, sizeof(m));
        m.kind = JT_MSG_PLAIN;
        m.item = it;
        m.edge = e;
        m.from = from;
        m.to = to;
        m.ssize = (int32_t)ss;
        m.nsplit = P.items[it].nsplit;
        m.partial_off = poff;
        m.sepc_off = P.edge[e].sepc_off;
        m.sepd_off = P.edge[e].sepd_off;
        P.msgs.push_back(m);
        P.items[it].msg = (int32_t)P.msgs.size() - 1;
        const int32_t t1 = (int32_t)P.tasks.size();
        const int32_t it2 = add_item(P, to, JT_SRC_OUT, P.cl[to].out_off, JT_DST_OUT, P.cl[to].out_off, {{e, true}},
                                     -1, -1, 0, bytes, group_entries_for(P, P.cl[to].size));
        emit_tasks(P, it2, it2 + 1, P.tune.target_blocks);
        P.plain.push_back({1, t1, (int32_t)P.tasks.size() - t1});
    };
    // Algorithm 2 (post-order) and Algorithm 3 (pre-order), children ascending
    {
        std::vector<std::pair<int32_t, size_t>> stack{{P.root, 0}};
        while (!stack.empty()) {
            auto &top = stack.back();
            const CliqueInfo &C = P.cl[top.first];
            if (top.second < C.children.size()) {
                const int32_t ch = C.children[top.second++];
                stack.push_back({ch, 0});
            } else {
                const int32_t c = top.first;
                stack.pop_back();
                if (P.iparent[c] >= 0) plain_message(P.iedge[c], c, P.iparent[c]);
            }
        }
        std::vector<std::pair<int32_t, size_t>> st2{{P.root, 0}};
        while (!st2.empty()) {
            auto &top = st2.back();
            const CliqueInfo &C = P.cl[top.first];
            if (top.second < C.children.size()) {
                const int32_t ch = C.children[top.second++];
                plain_message(P.iedge[ch], top.first, ch);
                st2.push_back({ch, 0});
            } else {
                st2.pop_back();
            }
        }
    }
    {
        // read-out: totals of every calibrated table, then normalize in place
        const int32_t t0 = (int32_t)P.tasks.size();
        const int32_t i0 = (int32_t)P.items.size();
        const int64_t ge = group_entries_for(P, P.total_entries);
        for (int32_t c = 0; c < nc; ++c) {
            const int32_t view = P.cl[c].total_view;
            const int32_t it = add_item(P, c, JT_SRC_OUT, P.cl[c].out_off, JT_DST_NONE, 0, {}, -1, view, 0, bytes, ge);
            const int64_t poff = add_partial(item_nsplit(P, it));
            P.items[it].partial_off = poff;
            JtMsg m;
            std::memset(&m, 0, sizeof(m));
            m.kind = JT_MSG_PLAIN_TOTAL;
            m.edge = -1;
            m.from = c;
            m.to = (c == P.root) ? -2 : -1;   // -2 marks the root: log Z is read there
            m.ssize = 1;
            m.nsplit = P.items[it].nsplit;
            m.partial_off = poff;
            m.item = it;
            P.msgs.push_back(m);
            P.items[it].msg = (int32_t)P.msgs.size() - 1;
        }
        emit_tasks(P, i0, (int32_t)P.items.size(), P.tune.target_blocks);
        P.plain.push_back({1, t0, (int32_t)P.tasks.size() - t0});
        const int32_t t1 = (int32_t)P.tasks.size();
        const int32_t i1 = (int32_t)P.items.size();
        for (int32_t c = 0; c < nc; ++c)
            add_item(P, c, JT_SRC_OUT, P.cl[c].out_off, JT_DST_OUT, P.cl[c].out_off, {}, c, -1, 0, bytes, ge);
        emit_tasks(P, i1, (int32_t)P.items.size(), P.tune.target_blocks);
        P.plain.push_back({1, t1, (int32_t)P.tasks.size() - t1});
    }
    P.bytes_plain = bytes;
    for (std::vector<Launch> *L : {&P.fused, &P.plain})
        for (Launch &l : *L) {
            if (l.is_pass != 1) continue;
            l.lds_floats = JT_FIN_LDS_FLOATS;
            for (int32_t t = l.begin; t < l.begin + l.count; ++t) {
                const JtItem &it = P.items[P.tasks[t].item];
                l.lds_floats = std::max<int32_t>(l.lds_floats, it.lds_floats);
                // a multi-slot pass stages one ratio table per slot of its set
                if (l.multi && P.item_multi[P.tasks[t].item])
                    l.lds_floats = std::max<int32_t>(
                        l.lds_floats, JT_MS * (int32_t)align_up(P.gathers[it.gather_base].ssize, 4));
                // room to stage a finalized separator of up to JT_FIN_STAGE_FLOATS entries
                if (it.msg >= 0)
                    l.lds_floats = std::max<int32_t>(l.lds_floats, std::min<int32_t>(JT_FIN_STAGE_FLOATS, it.o_ssize));
            }
            l.lds_floats = (int32_t)align_up(l.lds_floats, 64);
        }
    for (std::vector<Launch> *L : {&P.fused, &P.plain})
        for (Launch &l : *L) {
            if (l.is_pass != 1 || l.count == 0 || l.multi) continue;
            int32_t last = -1;
            for (int32_t t = l.begin; t < l.begin + l.count; ++t) {
                const int32_t i = P.tasks[t].item;
                if (i == last) continue;
                last = i;
                const JtItem &it = P.items[i];
                const int64_t tb = 4 * P.cl[it.clique].size;
                l.bytes += (it.src_kind == JT_SRC_INIT) ? tb : tb * P.n_slots;
                if (it.dst_kind != JT_DST_NONE) l.bytes += tb * P.n_slots;
            }
        }
    if (P.partial_stride > std::numeric_limits<int32_t>::max() * int64_t(4))
        return fail(err, JT_E_TOO_LARGE, "partial region too large");

    // per-block records: the task, its item and the item's first gathers
    P.blocks.resize(P.tasks.size());
    for (size_t k = 0; k < P.tasks.size(); ++k) {
        JtBlock &b = P.blocks[k];
        std::memset(&b, 0, sizeof(b));
        const JtTask &t = P.tasks[k];
        b.it = P.items[t.item];
        for (int g = 0; g < JT_NG_REG && g < b.it.n_gather; ++g) b.g[g] = P.gathers[b.it.gather_base + g];
        b.item = t.item;
        b.g0 = t.g0;
        b.g1 = t.g1;
    }

    // ---------------- workspace layout ----------------
    P.lam_stride = align_up(3 * (int64_t)nc + 1, 32);
    P.scale_stride = align_up(nc, kAlignFloats);
    P.ev_idx_stride = align_up((int64_t)nc + 1, kAlignFloats);
    P.ev_ent_stride = align_up(2 * (int64_t)nv + 1, 16);
    size_t off = 0;
    auto region = [&](size_t bytes_) {
        const size_t o = off;
        off = (size_t)align_up((int64_t)(off + bytes_), 256);
        return o;
    };
    const size_t S = (size_t)P.n_regions;   // slot regions, the evidence-free one included
    P.csrc_stride = align_up(nc, kAlignFloats);
    P.cltab.assign(3 * (size_t)nc, 0);
    {
        int64_t packed = 0;
        for (int32_t c = 0; c < nc; ++c) {
            P.cltab[3 * c] = P.cl[c].out_off;
            P.cltab[3 * c + 1] = P.cl[c].size;
            P.cltab[3 * c + 2] = packed;
            packed += P.cl[c].size;
        }
    }
    P.off_meta = region(P.meta.size() * sizeof(int32_t));
    P.off_views = region(P.views.size() * sizeof(JtView));
    P.off_gathers = region(std::max<size_t>(1, P.gathers.size()) * sizeof(JtGather));
    P.off_items = region(P.items.size() * sizeof(JtItem));
    P.off_tasks = region(P.tasks.size() * sizeof(JtTask));
    P.off_blocks = region(std::max<size_t>(1, P.blocks.size()) * sizeof(JtBlock));
    P.off_msgs = region(P.msgs.size() * sizeof(JtMsg));
    P.off_child = region(std::max<size_t>(1, P.child_edges.size()) * sizeof(int32_t));
    P.off_init = region((size_t)P.init_floats * sizeof(float));
    P.off_coll = region(S * (size_t)P.coll_stride * sizeof(float));
    P.off_out = region(S * (size_t)P.out_stride * sizeof(float));
    if ((int64_t)S * P.sep_stride > std::numeric_limits<int32_t>::max())
        return fail(err, JT_E_TOO_LARGE, "separator tables of all slots exceed 2^31 floats");
    P.off_sep = region(S * (size_t)P.sep_stride * sizeof(float));
    P.off_partial = region(S * (size_t)P.partial_stride * sizeof(float));
    P.off_lam = region(S * (size_t)P.lam_stride * sizeof(double));
    P.off_scale = region(S * (size_t)P.scale_stride * sizeof(float));
    P.off_flag = region(S * sizeof(int32_t));
    P.off_ev_idx = region(S * (size_t)P.ev_idx_stride * sizeof(int32_t));
    P.off_ev_ent = region(S * (size_t)P.ev_ent_stride * sizeof(JtEv));
    P.off_csrc = region(S * (size_t)P.csrc_stride * sizeof(int32_t));
    P.off_work_count = region(std::max<size_t>(1, (size_t)P.n_listed) * sizeof(int32_t));
    P.off_work = region(std::max<size_t>(1, (size_t)P.work_total) * sizeof(JtWork));
    P.off_chunks = region(std::max<size_t>(1, (size_t)P.chunk_total) * sizeof(JtChunk));
    P.off_dyn = P.off_ev_idx;
    P.dyn_bytes = off - P.off_ev_idx;
    P.icnt_stride = align_up(std::max<int64_t>(1, (int64_t)P.items.size()), kAlignFloats);
    P.off_icnt = region(S * (size_t)P.icnt_stride * sizeof(int32_t));
    P.off_cltab = region(P.cltab.size() * sizeof(int64_t));
    if (!P.fam.empty()) {
        P.off_fam = region(P.fam.size() * sizeof(JtFamily));
        P.off_fam_rng = region(P.fam_rng.size() * sizeof(int32_t));
        P.off_fam_mu = region((size_t)P.fam_mu_total * sizeof(int32_t));
        P.off_cshape = region(P.cshape.size() * sizeof(JtCliqueShape));
        P.off_card = region(std::max<size_t>(1, P.card.size()) * sizeof(int32_t));
        P.stage_floats = cpt_total;
        P.off_stage = region((size_t)std::max<int64_t>(1, cpt_total) * sizeof(float));
    }
    P.total_bytes = off;
    P.slot_bytes = (size_t)P.coll_stride * sizeof(float) + (size_t)P.out_stride * sizeof(float) +
                   (size_t)P.sep_stride * sizeof(float) + (size_t)P.partial_stride * sizeof(float) +
                   (size_t)P.lam_stride * sizeof(double) + (size_t)P.scale_stride * sizeof(float) + sizeof(int32_t) +
                   (size_t)P.ev_idx_stride * sizeof(int32_t) + (size_t)P.ev_ent_stride * sizeof(JtEv) +
                   (size_t)P.icnt_stride * sizeof(int32_t) + (size_t)P.csrc_stride * sizeof(int32_t);
    std::string why;
    if (!verify_plan(P, why)) return fail(err, JT_E_ARG, why);
    return JT_OK;
}

namespace {

// Deal groups of work entries to the 8 XCDs (blocks go to the XCDs round
// robin, so entry e of a list runs on XCD e % 8): a group's entries share a
// table (the same clique's source or absorbed table), so keeping them on one
// XCD keeps that table in one L2.  Groups are taken largest first onto the
// least-loaded XCD; a group above an eighth of the launch's work is cut so
// that one large clique still spreads over the chip.  Returns the list
// length (8 x the longest queue); shorter queues are padded with task -1.
int32_t place_on_xcds(std::vector<std::vector<JtWork>> &groups, const std::vector<int64_t> &weight, JtWork *out) {
    int64_t total = 0;
    for (int64_t w : weight) total += std::max<int64_t>(1, w);
    const int64_t cap = std::max<int64_t>(1, (total + 7) / 8);
    struct G { int64_t w; size_t g, lo, hi; };
    std::vector<G> parts;
    for (size_t g = 0; g < groups.size(); ++g) {
        const size_t n = groups[g].size();
        if (n == 0) continue;
        const int64_t w = std::max<int64_t>(1, weight[g]);
        const size_t pieces = (size_t)std::min<int64_t>((int64_t)n, (w + cap - 1) / cap);
        for (size_t k = 0; k < pieces; ++k)
            parts.push_back({w / (int64_t)pieces, g, n * k / pieces, n * (k + 1) / pieces});
    }
    std::stable_sort(parts.begin(), parts.end(), [](const G &a, const G &b) { return a.w > b.w; });
    std::vector<std::vector<JtWork>> q(8);
    std::vector<int64_t> load(8, 0);
    for (const G &p : parts) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        for (size_t i = p.lo; i < p.hi; ++i) q[x].push_back(groups[p.g][i]);
        load[x] += p.w;
    }
    size_t len = 0;
    for (const auto &v : q) len = std::max(len, v.size());
    for (size_t k = 0; k < len; ++k)
        for (int x = 0; x < 8; ++x) out[8 * k + x] = k < q[x].size() ? q[x][k] : JtWork{-1, 0};
    return (int32_t)(8 * len);
}

}  // namespace

void build_dynamic(const Plan &P, const std::vector<std::vector<int32_t>> &ev_vars, int32_t n_active, Dynamic &D) {
    const int32_t nc = P.n_cliques, S = P.n_slots, N = P.n_slots;   // N: the evidence-free slot
    D.csrc.assign((size_t)P.n_regions * P.csrc_stride, 0);
    for (int32_t r = 0; r < P.n_regions; ++r)
        for (int32_t c = 0; c < nc; ++c) D.csrc[(size_t)r * P.csrc_stride + c] = r;
    D.work.assign((size_t)std::max<int64_t>(1, P.work_total), JtWork{0, 0});
    D.count.assign((size_t)std::max<int32_t>(1, P.n_listed), 0);
    D.grid.assign((size_t)std::max<int32_t>(1, P.n_listed), 1);
    D.shared = 0;
    D.collect_pairs = 0;
    // dirty[s][c]: the subtree of c (schedule orientation) holds the home
    // clique of one of slot s's observed variables; the root always is
    std::vector<std::vector<char>> dirty((size_t)n_active, std::vector<char>(nc, 0));
    for (int32_t s = 0; s < n_active; ++s) {
        std::vector<char> &d = dirty[s];
        d[P.root] = 1;
        if (s < (int32_t)ev_vars.size())
            for (int32_t v : ev_vars[s]) {
                for (int32_t c = P.home[v]; c >= 0 && !d[c]; c = P.iparent[c]) d[c] = 1;
            }
    }
    // share when the evidence-free slot plus the dirty passes stream fewer
    // entries than every active slot's whole collect sweep
    int64_t full = 0, dirty_sum = 0;
    for (int32_t c = 0; c < nc; ++c) full += P.cl[c].size;
    for (int32_t s = 0; s < n_active; ++s)
        for (int32_t c = 0; c < nc; ++c)
            if (dirty[s][c]) dirty_sum += P.cl[c].size;
    const bool share = P.share && full + dirty_sum < (int64_t)n_active * full;
    D.shared = share ? 1 : 0;
    if (share)
        for (int32_t s = 0; s < n_active; ++s)
            for (int32_t c = 0; c < nc; ++c)
                if (!dirty[s][c]) D.csrc[(size_t)s * P.csrc_stride + c] = N;
    auto runs = [&](int32_t s, int32_t c) { return share ? (s == N || dirty[s][c]) : s < n_active; };
    // a distribute pass of slot s reads the evidence-free slot's table
    auto shared_src = [&](int32_t s, int32_t c) { return D.csrc[(size_t)s * P.csrc_stride + c] != s; };
    JtChunk none;
    for (int k = 0; k < JT_MS; ++k) none.s[k] = -1;
    D.chunks.assign((size_t)std::max<int64_t>(1, P.chunk_total), none);
    int64_t bytes = 0;
    D.launch_bytes.assign(P.fused.size(), 0);
    for (size_t li = 0; li < P.fused.size(); ++li) {
        const Launch &l = P.fused[li];
        if (l.count == 0) continue;
        int64_t bytes0 = bytes;
        // the level's multi-slot launch directly precedes its other distribute launch
        const int32_t mli = (li > 0 && P.fused[li - 1].multi && P.fused[li - 1].begin == l.begin) ? (int32_t)li - 1 : -1;
        if (l.listed && l.multi) {
            // sets of up to JT_MS slots per (task, clique without evidence of
            // them); all sets of one task go to one XCD (blocks are dealt to
            // the XCDs round robin, so entry e runs on XCD e % 8), which keeps
            // the shared source table in that XCD's L2; tasks are spread over
            // the XCDs by their work, the lists padded to equal length
            struct Ent { int32_t task, chunk; };
            std::vector<std::vector<Ent>> xl(8);
            std::vector<int64_t> load(8, 0);
            int64_t nch = 0;
            std::vector<std::pair<int64_t, int32_t>> order;
            for (int32_t t = 0; t < l.count; ++t) {
                const int32_t i = P.tasks[l.begin + t].item;
                if (!P.item_multi[i]) continue;
                const JtTask &T = P.tasks[l.begin + t];
                order.push_back({-(16384 + (int64_t)(T.g1 - T.g0) * P.items[i].tpg * P.items[i].T), t});
            }
            std::stable_sort(order.begin(), order.end());
            std::vector<std::pair<int64_t, std::vector<int32_t>>> sets;   // (order index, slots)
            int64_t n_full = 0;
            for (size_t oi = 0; oi < order.size(); ++oi) {
                const int32_t c = P.items[P.tasks[l.begin + order[oi].second].item].clique;
                std::vector<int32_t> sl;
                if (share)
                    for (int32_t s = 0; s < n_active; ++s)
                        if (shared_src(s, c)) sl.push_back(s);
                if (sl.empty()) continue;
                n_full += ((int64_t)sl.size() + JT_MS - 1) / JT_MS;
                sets.push_back({(int64_t)oi, std::move(sl)});
            }
            // sets of JT_MS slots, or of JT_MS / 2 when the level's sets of
            // JT_MS would not fill one round of resident multi-slot blocks:
            // more, shorter blocks then end a short level sooner
            const size_t m = n_full < JT_MULTI_ROUND ? JT_MS / 2 : JT_MS;
            for (const auto &ts : sets) {
                const int32_t t = order[ts.first].second;
                const std::vector<int32_t> &sl = ts.second;
                const int32_t x = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
                for (size_t k0 = 0; k0 < sl.size(); k0 += m) {
                    JtChunk ch;
                    for (size_t k = 0; k < JT_MS; ++k) ch.s[k] = (k < m && k0 + k < sl.size()) ? sl[k0 + k] : -1;
                    D.chunks[l.chunk_off + nch] = ch;
                    xl[x].push_back({t, (int32_t)nch});
                    ++nch;
                }
                load[x] += -order[ts.first].first * (int64_t)((sl.size() + m - 1) / m);
            }
            size_t len = 0;
            for (const auto &v : xl) len = std::max(len, v.size());
            for (size_t k = 0; k < len; ++k)
                for (int x = 0; x < 8; ++x)
                    D.work[l.work_off + 8 * k + x] = k < xl[x].size() ? JtWork{xl[x][k].task, (int32_t)l.chunk_off + xl[x][k].chunk}
                                                                     : JtWork{-1, 0};
            const int32_t k = (int32_t)(8 * len);
            D.count[l.work_idx] = k;
            int64_t g = 1;
            while (g < k) g *= 2;
            D.grid[l.work_idx] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(g, l.work_cap));
            continue;   // its bytes are counted with the level's other launch
        }
        if (l.listed) {
            // groups: collect -- every pass of one clique (they read its
            // initial table); distribute -- the passes of one (clique, slot)
            // (the items of its children read its table once each)
            std::map<std::pair<int32_t, int32_t>, size_t> gid;
            std::vector<std::vector<JtWork>> groups;
            std::vector<int64_t> weight;
            auto put = [&](int32_t c, int32_t key, int32_t t, int32_t s) {
                auto it = gid.emplace(std::make_pair(c, key), groups.size());
                if (it.second) {
                    groups.emplace_back();
                    weight.push_back(0);
                }
                groups[it.first->second].push_back(JtWork{t, s});
                // a block costs its set-up and finalize latency plus its
                // streaming: weigh it as a fixed 16K entries plus its entries
                const JtTask &T = P.tasks[l.begin + t];
                weight[it.first->second] += 16384 + (int64_t)(T.g1 - T.g0) * P.items[T.item].tpg * P.items[T.item].T;
            };
            for (int32_t t = 0; t < l.count; ++t) {
                const int32_t i = P.tasks[l.begin + t].item;
                const int32_t c = P.items[i].clique;
                if (l.collect) {
                    if (share) put(c, -1, t, N);
                    for (int32_t s = 0; s < n_active; ++s)
                        if (runs(s, c)) put(c, -1, t, s);
                } else {
                    // the pairs no multi-slot set took
                    for (int32_t s = 0; s < n_active; ++s)
                        if (!(share && P.item_multi[i] && shared_src(s, c))) put(c, s, t, s);
                }
            }
            const int32_t k = place_on_xcds(groups, weight, &D.work[l.work_off]);
            if (k > l.work_cap) throw std::logic_error("work list overflow");
            D.count[l.work_idx] = k;
            int64_t g = 1;
            while (g < k) g *= 2;
            D.grid[l.work_idx] = (int32_t)std::max<int64_t>(1, std::min<int64_t>(g, l.work_cap));
        }
        // FP32 table bytes: shared tables (initial tables, evidence-free
        // absorbed tables) once per level, slot tables per slot
        int32_t last = -1;
        for (int32_t t = l.begin; t < l.begin + l.count; ++t) {
            const int32_t i = P.tasks[t].item;
            if (i == last) continue;
            last = i;
            const JtItem &it = P.items[i];
            const int32_t c = it.clique;
            const int64_t tb = 4 * P.cl[c].size;
            if (l.collect) {
                int64_t n = 0;
                for (int32_t s = 0; s < n_active; ++s) n += runs(s, c) ? 1 : 0;
                if (share) n += 1;
                D.collect_pairs += n;
                // the initial table once, or a pre-absorbed collect table per slot
                if (n > 0) bytes += it.src_kind == JT_SRC_INIT ? tb : tb * n;
                if (it.dst_kind != JT_DST_NONE) bytes += tb * n;  // absorbed tables
            } else {
                // slots reading the shared source run in the level's
                // multi-slot launch when the item is eligible, else here
                // (shared source: the initial table, or the evidence-free
                // slot's absorbed table; read once per launch that reads it)
                int64_t own = 0, sh = 0;
                for (int32_t s = 0; s < n_active; ++s) {
                    if (!shared_src(s, c)) ++own;
                    else ++sh;
                }
                const bool in_multi = share && P.item_multi[i] && sh > 0 && mli >= 0;
                int64_t b_here = 0, b_multi = 0;
                if (it.src_kind == JT_SRC_INIT) {
                    if (own > 0 || !in_multi) b_here += tb;
                    if (in_multi) b_multi += tb;
                } else {
                    b_here += tb * own;
                    (in_multi ? b_multi : b_here) += sh > 0 ? tb : 0;
                }
                if (it.dst_kind != JT_DST_NONE) {
                    b_here += tb * (in_multi ? own : n_active);
                    if (in_multi) b_multi += tb * sh;
                }
                bytes += b_here + b_multi;
                if (mli >= 0) D.launch_bytes[mli] += b_multi;
                bytes0 += b_multi;
            }
        }
        D.launch_bytes[li] = bytes - bytes0;
    }
    D.bytes = bytes;
    (void)S;
}

void build_paper_plan(const Plan &P, PaperPlan &pp) {
    pp = PaperPlan();
    const int32_t nc = P.n_cliques;
    // the caller's orientation: children ascending
    std::vector<std::vector<int32_t>> ch(nc);
    for (int32_t c = 0; c < nc; ++c)
        if (P.parent[c] >= 0) ch[P.parent[c]].push_back(c);
    std::vector<int64_t> mu_off_side(2 * (size_t)nc, -1);   // per edge: child-side and parent-side lists
    auto lists = [&](int32_t e, int side) {
        int64_t &o = mu_off_side[2 * (size_t)e + side];
        if (o < 0) {
            o = pp.mu_total;
            pp.mu_total += P.cl[side == 0 ? e : P.parent[e]].size;
        }
        return o;
    };
    auto add = [&](int32_t e, int32_t from, int32_t to) {
        JtPaperMsg m;
        std::memset(&m, 0, sizeof(m));
        const int fs = from == e ? 0 : 1, ts = to == e ? 0 : 1;
        m.mu_from = lists(e, fs);
        m.mu_to = lists(e, ts);
        m.ssize = (int32_t)P.edge[e].ssize;
        m.m_from = (int32_t)(P.cl[from].size / m.ssize);
        m.m_to = (int32_t)(P.cl[to].size / m.ssize);
        m.from_off = P.cl[from].out_off;
        m.to_off = P.cl[to].out_off;
        m.edge = e;
        m.from = from;
        m.to = to;
        m.sepc_off = P.edge[e].sepc_off;
        m.sepd_off = P.edge[e].sepd_off;
        pp.msgs.push_back(m);
    };
    // Algorithm 2: a child's subtree is collected, then the child sends to
    // its parent (post-order); Algorithm 3: a parent sends to each child,
    // then the child distributes (pre-order)
    {
        std::vector<std::pair<int32_t, size_t>> st{{P.user_root, 0}};
        while (!st.empty()) {
            auto &top = st.back();
            if (top.second < ch[top.first].size()) {
                const int32_t c = ch[top.first][top.second++];
                st.push_back({c, 0});
            } else {
                const int32_t c = top.first;
                st.pop_back();
                if (P.parent[c] >= 0) add(c, c, P.parent[c]);
            }
        }
        std::vector<std::pair<int32_t, size_t>> st2{{P.user_root, 0}};
        while (!st2.empty()) {
            auto &top = st2.back();
            if (top.second < ch[top.first].size()) {
                const int32_t c = ch[top.first][top.second++];
                add(c, top.first, c);
                st2.push_back({c, 0});
            } else {
                st2.pop_back();
            }
        }
    }
    for (int32_t c = 0; c < nc; ++c)
        for (int64_t a = 0; a < P.cl[c].size; a += 4096) {
            JtPaperBlk b;
            b.clique = c;
            b.T = P.cl[c].T;
            b.start = a;
            b.end = std::min<int64_t>(P.cl[c].size, a + 4096);
            b.init_off = P.cl[c].init_off;
            b.out_off = P.cl[c].out_off;
            pp.blocks.push_back(b);
        }
    size_t off = 0;
    auto region = [&](size_t bytes) {
        const size_t o = off;
        off = (size_t)align_up((int64_t)(off + bytes), 256);
        return o;
    };
    pp.off_msgs = region(std::max<size_t>(1, pp.msgs.size()) * sizeof(JtPaperMsg));
    pp.off_blocks = region(std::max<size_t>(1, pp.blocks.size()) * sizeof(JtPaperBlk));
    pp.off_mu = region(std::max<int64_t>(1, pp.mu_total) * sizeof(int32_t));
    pp.bytes = off;
}

void paper_mu_lists(const Plan &P, const PaperPlan &pp, int32_t layout, int32_t *out) {
    std::vector<char> done((size_t)std::max<int64_t>(1, pp.mu_total), 0);
    std::vector<int32_t> map;
    for (const JtPaperMsg &m : pp.msgs) {
        for (int side = 0; side < 2; ++side) {
            const int64_t base = side == 0 ? m.mu_from : m.mu_to;
            if (done[base]) continue;
            done[base] = 1;
            const int32_t c = side == 0 ? m.from : m.to;
            const int32_t e = m.edge;
            const int32_t view = c == e ? P.edge[e].view_child : P.edge[e].view_parent;
            const int64_t n = P.cl[c].size, S = m.ssize, len = n / S;
            map.resize(n);
            expand_map(P, view, map.data());
            std::vector<int64_t> fill(S, 0);
            for (int64_t r = 0; r < n; ++r) {   // ascending r: every list in ascending order
                const int64_t j = map[r], k = fill[j]++;
                out[base + (layout == JT_LAYOUT_INTERLEAVED_ ? k * S + j : j * len + k)] = (int32_t)r;
            }
        }
    }
}

void family_mu_lists(const Plan &P, int32_t *out) {
    for (const JtFamily &F : P.fam) {
        const CliqueInfo &C = P.cl[F.clique];
        const int32_t *jin = P.meta.data() + F.jin_off;
        const int32_t *jout = P.meta.data() + F.jout_off;
        const int64_t m = C.size / F.fsize;
        std::vector<int64_t> fill(F.fsize, 0);
        for (int64_t o = 0; o < C.n_tiles; ++o)
            for (int64_t i = 0; i < C.T; ++i) {
                const int64_t j = jin[i] + jout[o];
                out[F.mu_off + j * m + fill[j]++] = (int32_t)(o * C.T + i);
            }
    }
}

jt_status compile_bn(const jt_bn_desc *bn, BnTree &T, std::string &err) {
    T = BnTree();
    if (!bn || bn->n_vars < 1 || !bn->card || !bn->parent_off || (bn->parent_off[bn->n_vars] > 0 && !bn->parents))
        return fail(err, JT_E_ARG, "bad network description");
    const int32_t n = bn->n_vars;
    T.card.assign(bn->card, bn->card + n);
    std::vector<std::vector<int32_t>> pa(n);
    if (bn->parent_off[0] != 0) return fail(err, JT_E_ARG, "parent_off[0] != 0");
    for (int32_t v = 0; v < n; ++v) {
        if (T.card[v] < 1) return fail(err, JT_E_ARG, "card < 1");
        if (bn->parent_off[v + 1] < bn->parent_off[v] || bn->parent_off[v + 1] - bn->parent_off[v] > 63)
            return fail(err, JT_E_ARG, "bad parent count");
        for (int64_t k = bn->parent_off[v]; k < bn->parent_off[v + 1]; ++k) {
            const int32_t p = bn->parents[k];
            if (p < 0 || p >= n || p == v) return fail(err, JT_E_ARG, "parent out of range");
            if (std::find(pa[v].begin(), pa[v].end(), p) != pa[v].end()) return fail(err, JT_E_ARG, "repeated parent");
            pa[v].push_back(p);
        }
    }
    // acyclic: Kahn's order over parent -> child
    {
        std::vector<int32_t> indeg(n, 0);
        std::vector<std::vector<int32_t>> ch(n);
        for (int32_t v = 0; v < n; ++v)
            for (int32_t p : pa[v]) {
                ch[p].push_back(v);
                ++indeg[v];
            }
        std::vector<int32_t> q;
        for (int32_t v = 0; v < n; ++v)
            if (!indeg[v]) q.push_back(v);
        for (size_t h = 0; h < q.size(); ++h)
            for (int32_t c : ch[q[h]])
                if (--indeg[c] == 0) q.push_back(c);
        if ((int32_t)q.size() != n) return fail(err, JT_E_NOT_JUNCTION_TREE, "the parent links contain a cycle");
    }
    // moral graph (a bit matrix for adjacency tests, sets for neighbours)
    std::vector<std::vector<char>> adj(n, std::vector<char>(n, 0));
    std::vector<std::set<int32_t>> nbs(n);
    auto link = [&](int32_t a, int32_t b) {
        if (a != b && !adj[a][b]) {
            adj[a][b] = adj[b][a] = 1;
            nbs[a].insert(b);
            nbs[b].insert(a);
        }
    };
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t p : pa[v]) link(v, p);
        for (size_t a = 0; a < pa[v].size(); ++a)
            for (size_t b = a + 1; b < pa[v].size(); ++b) link(pa[v][a], pa[v][b]);
    }
    // greedy elimination, fewest fill-in edges, then fewest neighbours, then
    // the lower id; each eliminated variable with its neighbours is a
    // candidate clique
    std::vector<char> gone(n, 0);
    std::vector<std::vector<int32_t>> cand;
    for (int32_t step = 0; step < n; ++step) {
        int32_t best = -1;
        int64_t bf = 0, bd = 0;
        for (int32_t v = 0; v < n; ++v) {
            if (gone[v]) continue;
            const std::vector<int32_t> nb(nbs[v].begin(), nbs[v].end());
            int64_t fill = 0;
            for (size_t a = 0; a < nb.size(); ++a)
                for (size_t b = a + 1; b < nb.size(); ++b) fill += adj[nb[a]][nb[b]] ? 0 : 1;
            if (best < 0 || fill < bf || (fill == bf && (int64_t)nb.size() < bd)) {
                best = v;
                bf = fill;
                bd = (int64_t)nb.size();
            }
        }
        std::vector<int32_t> cl{best};
        for (int32_t u : nbs[best]) cl.push_back(u);
        for (size_t a = 1; a < cl.size(); ++a)
            for (size_t b = a + 1; b < cl.size(); ++b) link(cl[a], cl[b]);
        gone[best] = 1;
        for (int32_t u : nbs[best]) nbs[u].erase(best);
        nbs[best].clear();
        std::sort(cl.begin(), cl.end());
        int64_t size = 1;
        for (int32_t v : cl) {
            size *= T.card[v];
            if (size > std::numeric_limits<int32_t>::max())
                return fail(err, JT_E_TOO_LARGE, "a clique of the triangulated network has 2^31 or more entries");
        }
        cand.push_back(cl);
    }
    // maximal candidates, in elimination order
    for (size_t a = 0; a < cand.size(); ++a) {
        bool sub = false;
        for (size_t b = 0; b < cand.size() && !sub; ++b) {
            if (a == b) continue;
            const bool incl = std::includes(cand[b].begin(), cand[b].end(), cand[a].begin(), cand[a].end());
            // equal sets: keep the first
            if (incl && (cand[b].size() > cand[a].size() || b < a)) sub = true;
        }
        if (!sub) T.cliques.push_back(cand[a]);
    }
    const int32_t nc = (int32_t)T.cliques.size();
    // maximum-weight spanning tree over separator sizes (Kruskal)
    struct E { int32_t w, a, b; };
    std::vector<E> es;
    for (int32_t a = 0; a < nc; ++a)
        for (int32_t b = a + 1; b < nc; ++b) {
            std::vector<int32_t> x;
            std::set_intersection(T.cliques[a].begin(), T.cliques[a].end(), T.cliques[b].begin(), T.cliques[b].end(),
                                  std::back_inserter(x));
            es.push_back({(int32_t)x.size(), a, b});
        }
    std::stable_sort(es.begin(), es.end(), [](const E &x, const E &y) { return x.w > y.w; });
    std::vector<int32_t> uf(nc);
    for (int32_t c = 0; c < nc; ++c) uf[c] = c;
    std::function<int32_t(int32_t)> root = [&](int32_t x) { return uf[x] == x ? x : (uf[x] = root(uf[x])); };
    std::vector<std::vector<int32_t>> nbr(nc);
    for (const E &e : es) {
        const int32_t ra = root(e.a), rb = root(e.b);
        if (ra == rb) continue;
        uf[ra] = rb;
        nbr[e.a].push_back(e.b);
        nbr[e.b].push_back(e.a);
    }
    T.parent.assign(nc, -1);
    {
        std::vector<char> seen(nc, 0);
        std::vector<int32_t> q{0};
        seen[0] = 1;
        for (size_t h = 0; h < q.size(); ++h) {
            std::vector<int32_t> nb = nbr[q[h]];
            std::sort(nb.begin(), nb.end());
            for (int32_t y : nb)
                if (!seen[y]) {
                    seen[y] = 1;
                    T.parent[y] = q[h];
                    q.push_back(y);
                }
        }
    }
    // families
    int64_t off = 0;
    for (int32_t v = 0; v < n; ++v) {
        std::vector<int32_t> fam(pa[v]);
        fam.push_back(v);
        std::vector<int32_t> fs(fam);
        std::sort(fs.begin(), fs.end());
        int32_t home = -1;
        for (int32_t c = 0; c < nc && home < 0; ++c)
            if (std::includes(T.cliques[c].begin(), T.cliques[c].end(), fs.begin(), fs.end())) home = c;
        if (home < 0) return fail(err, JT_E_ARG, "internal: a family is in no clique");
        int64_t size = 1;
        for (int32_t u : fam) size *= T.card[u];
        T.families.push_back({home, v, fam, off});
        off += size;
    }
    T.cpt_total = off;
    return JT_OK;
}

jt_status merge_tree(const jt_tree_desc *desc, int32_t max_sep, int64_t max_entries, MergedTree &M,
                     std::string &err) {
    M = MergedTree();
    {
        // the caller's tree must be a junction tree
        Plan check;
        jt_tree_desc d1 = *desc;
        d1.n_slots = 1;
        d1.tuning = nullptr;
        const jt_status rc = compile_plan(&d1, check, err);
        if (rc != JT_OK) return rc;
    }
    if (max_sep < 1 || max_entries < 1) return fail(err, JT_E_ARG, "merge bounds must be positive");
    const int32_t nc = desc->n_cliques, nv = desc->n_vars;
    M.card.assign(desc->card, desc->card + nv);
    std::vector<std::vector<int32_t>> vars(nc);
    for (int32_t c = 0; c < nc; ++c) {
        vars[c].assign(desc->clique_vars + desc->clique_off[c], desc->clique_vars + desc->clique_off[c + 1]);
        int64_t sz = 1;
        for (int32_t v : vars[c]) sz *= M.card[v];
        M.orig_size.push_back(sz);
    }
    int32_t root = -1;
    std::vector<std::vector<int32_t>> ch(nc);
    for (int32_t c = 0; c < nc; ++c) {
        if (desc->parent[c] < 0) root = c;
        else ch[desc->parent[c]].push_back(c);
    }
    // post-order (children ascending)
    std::vector<int32_t> post;
    {
        std::vector<std::pair<int32_t, size_t>> st{{root, 0}};
        while (!st.empty()) {
            auto &top = st.back();
            if (top.second < ch[top.first].size()) {
                const int32_t c = ch[top.first][top.second++];
                st.push_back({c, 0});
            } else {
                post.push_back(top.first);
                st.pop_back();
            }
        }
    }
    std::vector<int32_t> grp(nc);
    std::vector<std::vector<int32_t>> gvars(nc);   // sorted union of each group's variables
    for (int32_t c = 0; c < nc; ++c) {
        grp[c] = c;
        gvars[c] = vars[c];
        std::sort(gvars[c].begin(), gvars[c].end());
    }
    std::function<int32_t(int32_t)> find = [&](int32_t x) { return grp[x] == x ? x : (grp[x] = find(grp[x])); };
    for (int32_t c : post) {
        const int32_t p = desc->parent[c];
        if (p < 0) continue;
        std::vector<int32_t> sc(vars[c]), sp(vars[p]), sep;
        std::sort(sc.begin(), sc.end());
        std::sort(sp.begin(), sp.end());
        std::set_intersection(sc.begin(), sc.end(), sp.begin(), sp.end(), std::back_inserter(sep));
        int64_t ss = 1;
        for (int32_t v : sep) ss *= M.card[v];
        if (ss > max_sep) continue;
        const int32_t a = find(c), b = find(p);
        std::vector<int32_t> un;
        std::set_union(gvars[a].begin(), gvars[a].end(), gvars[b].begin(), gvars[b].end(), std::back_inserter(un));
        int64_t sz = 1;
        for (int32_t v : un) {
            sz *= M.card[v];
            if (sz > max_entries) break;
        }
        if (sz > max_entries) continue;
        grp[a] = b;
        gvars[b] = un;
    }
    // merged cliques in order of their smallest original id (the caller's
    // root's group first)
    std::vector<int32_t> id(nc, -1), rep;
    const int32_t r0 = find(root);
    id[r0] = 0;
    rep.push_back(r0);
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t g = find(c);
        if (id[g] < 0) {
            id[g] = (int32_t)rep.size();
            rep.push_back(g);
        }
    }
    const int32_t nm = (int32_t)rep.size();
    M.cliques.resize(nm);
    M.parent.assign(nm, -1);
    for (int32_t k = 0; k < nm; ++k) M.cliques[k] = gvars[rep[k]];
    for (int32_t c = 0; c < nc; ++c) {
        const int32_t p = desc->parent[c];
        if (p >= 0 && find(c) != find(p)) M.parent[id[find(c)]] = id[find(p)];
    }
    int64_t off = 0;
    for (int32_t c = 0; c < nc; ++c) {
        M.families.push_back({id[find(c)], c, vars[c], off});
        off += M.orig_size[c];
    }
    M.total = off;
    return JT_OK;
}

void evidence_tables(const Plan &P, const std::vector<int32_t> &vars, const std::vector<int32_t> &states,
                     int32_t *idx, JtEv *ent) {
    const int32_t nc = P.n_cliques;
    std::vector<std::vector<JtEv>> per(nc);
    std::vector<int32_t> seen(P.n_vars, 0);
    for (size_t a = 0; a < vars.size(); ++a) {
        const int32_t v = vars[a], s = states[a];
        if (seen[v]) continue;   // repeats carry the same state (checked by the caller)
        seen[v] = 1;
        const int32_t c = P.home[v];
        if (c < 0) continue;
        for (const VDigit &d : P.cl[c].digits) {
            if (d.var != v || d.card == 1) continue;
            JtEv e;
            e.outer = d.outer ? 1 : 0;
            e.stride = (int32_t)(d.outer ? d.ostride : d.stride);
            e.card = d.card;
            e.digit = (int32_t)((s / d.w) % d.card);
            per[c].push_back(e);
        }
    }
    int32_t k = 0;
    for (int32_t c = 0; c < nc; ++c) {
        idx[c] = k;
        for (const JtEv &e : per[c]) ent[k++] = e;
    }
    idx[nc] = k;
}

void expand_map(const Plan &P, int32_t view, int32_t *out) {
    const JtView &V = P.views[view];
    const CliqueInfo &C = P.cl[V.clique];
    const int32_t *jin = P.meta.data() + V.jin_off;
    const int32_t *jout = P.meta.data() + V.jout_off;
    for (int64_t o = 0; o < C.n_tiles; ++o)
        for (int64_t i = 0; i < C.T; ++i) out[o * C.T + i] = jin[i] + jout[o];
}

}  // namespace jt
