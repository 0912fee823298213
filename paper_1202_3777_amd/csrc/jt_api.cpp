// jt_api.cpp -- the C ABI of include/jt.h: handles, binding of caller-owned
// device memory, evidence upload, the propagation schedules (level-fused,
// captured graph, one message at a time) and read-out.
#include <hip/hip_runtime_api.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "jt.h"
#include "jt_api_internal.h"
#include "jt_plan.h"

hipError_t jt_launch_pass(const JtDev &d, int task_begin, int n_tasks, int n_slots, int lds_floats, int flags,
                          int64_t work_off, int work_idx, int grid, hipStream_t s);
hipError_t jt_launch_pass_multi(const JtDev &d, int task_begin, int lds_floats, int64_t work_off, int work_idx,
                                int grid, hipStream_t s);
hipError_t jt_launch_plain_init(const JtDev &d, int n_slots, hipStream_t s);
hipError_t jt_launch_paper_slot(const JtDev &d, const JtPaperMsg *host_msgs, int n_msgs, const JtPaperBlk *dev_blocks,
                                int n_blocks, const int32_t *dev_mu, int32_t layout, int32_t tpb, int32_t root,
                                int slot, hipStream_t s);
hipError_t jt_launch_bn_init(const JtDev &d, const JtFamily *fam, const int32_t *fam_rng, const JtCliqueShape *shape,
                             int n_cliques, int64_t max_tiles, const float *cpts, hipStream_t s);
hipError_t jt_launch_family_marginal(const JtDev &d, const JtFamily *fam, int fam0, int n_fam, int64_t max_fsize,
                                     const int32_t *mu, const JtCliqueShape *shape, int s0, int n_slots, float *dst,
                                     int64_t dst_base, hipStream_t s);
hipError_t jt_launch_bn_mstep(const JtFamily *fam, int n_fam, int64_t max_rows, const int32_t *card,
                              const float *counts, float alpha, float *cpts, hipStream_t s);
hipError_t jt_launch_read_out(const JtDev &d, int slot0, int n_slots, int64_t packed_total, float *dst,
                              double *log_z, hipStream_t s);

namespace jt_detail {

thread_local std::string g_err;

jt_status set_err(jt_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

jt_status hip_err(hipError_t e, const char *what) {
    return set_err(JT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace jt_detail

using namespace jt_detail;

namespace {

// The persistent dataflow schedule is switched off: its first run on the GPU
// did not complete and no cause was shown, so its kernel was taken out and
// the mode is refused.
jt_status dataflow_disabled() {
    return set_err(JT_E_ARG, "the dataflow schedule is disabled (its launch did not complete on the GPU; "
                             "cause not found)");
}

}  // namespace

namespace jt_detail {

jt_status check_tree(jt_tree t) {
    if (!t) return set_err(JT_E_ARG, "tree handle is NULL");
    return JT_OK;
}

// ---- staging ---------------------------------------------------------------

hipError_t stage_begin(Staging &S) {
    S.k ^= 1;
    S.used = 0;
    if (S.pending[S.k]) {
        hipError_t e = hipEventSynchronize(S.done[S.k]);
        if (e != hipSuccess) return e;
        S.pending[S.k] = false;
    }
    return hipSuccess;
}

hipError_t stage_put(Staging &S, void *dev, const void *src, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (S.used + n > S.cap) return hipErrorInvalidValue;
    char *h = S.host[S.k] + S.used;
    std::memcpy(h, src, n);
    S.used += (n + 255) / 256 * 256;
    return hipMemcpyAsync(dev, h, n, hipMemcpyHostToDevice, s);
}

hipError_t stage_end(Staging &S, hipStream_t s) {
    hipError_t e = hipEventRecord(S.done[S.k], s);
    if (e == hipSuccess) S.pending[S.k] = true;
    return e;
}

void drop_staging(Staging &S) {
    for (int k = 0; k < 2; ++k) {
        if (S.pending[k] && S.done[k]) (void)hipEventSynchronize(S.done[k]);
        if (S.done[k]) (void)hipEventDestroy(S.done[k]);
        if (S.host[k]) (void)hipHostFree(S.host[k]);
        S.host[k] = nullptr;
        S.done[k] = nullptr;
        S.pending[k] = false;
    }
    S.cap = S.used = 0;
}

// Device views of a workspace laid out by the plan.
void fill_dev(const jt::Plan &P, char *base, JtDev &d) {
    std::memset(&d, 0, sizeof(d));
    d.meta = reinterpret_cast<const int32_t *>(base + P.off_meta);
    d.views = reinterpret_cast<const JtView *>(base + P.off_views);
    d.gathers = reinterpret_cast<const JtGather *>(base + P.off_gathers);
    d.items = reinterpret_cast<const JtItem *>(base + P.off_items);
    d.tasks = reinterpret_cast<const JtTask *>(base + P.off_tasks);
    d.blocks = reinterpret_cast<const JtBlock *>(base + P.off_blocks);
    d.msgs = reinterpret_cast<const JtMsg *>(base + P.off_msgs);
    d.child_edges = reinterpret_cast<const int32_t *>(base + P.off_child);
    d.icnt = reinterpret_cast<int32_t *>(base + P.off_icnt);
    d.init = reinterpret_cast<const float *>(base + P.off_init);
    d.coll = reinterpret_cast<float *>(base + P.off_coll);
    d.out = reinterpret_cast<float *>(base + P.off_out);
    d.sep = reinterpret_cast<float *>(base + P.off_sep);
    d.partial = reinterpret_cast<float *>(base + P.off_partial);
    d.lam = reinterpret_cast<double *>(base + P.off_lam);
    d.scale = reinterpret_cast<float *>(base + P.off_scale);
    d.flag = reinterpret_cast<int32_t *>(base + P.off_flag);
    d.ev_idx = reinterpret_cast<const int32_t *>(base + P.off_ev_idx);
    d.ev_ent = reinterpret_cast<const JtEv *>(base + P.off_ev_ent);
    d.csrc = reinterpret_cast<const int32_t *>(base + P.off_csrc);
    d.work = reinterpret_cast<const JtWork *>(base + P.off_work);
    d.work_count = reinterpret_cast<const int32_t *>(base + P.off_work_count);
    d.chunks = reinterpret_cast<const JtChunk *>(base + P.off_chunks);
    d.cltab = reinterpret_cast<const int64_t *>(base + P.off_cltab);
    d.coll_stride = P.coll_stride;
    d.out_stride = P.out_stride;
    d.sep_stride = P.sep_stride;
    d.partial_stride = P.partial_stride;
    d.lam_stride = P.lam_stride;
    d.scale_stride = P.scale_stride;
    d.ev_idx_stride = P.ev_idx_stride;
    d.ev_ent_stride = P.ev_ent_stride;
    d.icnt_stride = P.icnt_stride;
    d.csrc_stride = P.csrc_stride;
    d.n_cliques = P.n_cliques;
    d.n_msgs = (int32_t)P.msgs.size();
}

// Enqueue the plan's read-only metadata, the initial tables (aligned layout,
// one copy per clique) and zeroed arrival counters into a workspace.
hipError_t upload_static(const jt::Plan &P, char *base, const float *init_potentials, hipStream_t s) {
    auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(base + off, src, n, hipMemcpyHostToDevice, s);
    };
    hipError_t e = up(P.off_meta, P.meta.data(), P.meta.size() * sizeof(int32_t));
    if (e == hipSuccess) e = up(P.off_views, P.views.data(), P.views.size() * sizeof(JtView));
    if (e == hipSuccess) e = up(P.off_gathers, P.gathers.data(), P.gathers.size() * sizeof(JtGather));
    if (e == hipSuccess) e = up(P.off_items, P.items.data(), P.items.size() * sizeof(JtItem));
    if (e == hipSuccess) e = up(P.off_tasks, P.tasks.data(), P.tasks.size() * sizeof(JtTask));
    if (e == hipSuccess) e = up(P.off_blocks, P.blocks.data(), P.blocks.size() * sizeof(JtBlock));
    if (e == hipSuccess) e = up(P.off_msgs, P.msgs.data(), P.msgs.size() * sizeof(JtMsg));
    if (e == hipSuccess) e = up(P.off_child, P.child_edges.data(), P.child_edges.size() * sizeof(int32_t));
    if (e == hipSuccess) e = up(P.off_cltab, P.cltab.data(), P.cltab.size() * sizeof(int64_t));
    // pass arrival counters start at zero; the block that finalizes a message
    // resets its counter, so no clearing is needed between propagations
    if (e == hipSuccess)
        e = hipMemsetAsync(base + P.off_icnt, 0, (size_t)P.n_regions * P.icnt_stride * sizeof(int32_t), s);
    // network trees: family records, their ranges and the clique shapes (the
    // initial tables are then computed from the conditional tables)
    if (e == hipSuccess && !P.fam.empty()) {
        e = up(P.off_fam, P.fam.data(), P.fam.size() * sizeof(JtFamily));
        if (e == hipSuccess) e = up(P.off_fam_rng, P.fam_rng.data(), P.fam_rng.size() * sizeof(int32_t));
        if (e == hipSuccess) e = up(P.off_cshape, P.cshape.data(), P.cshape.size() * sizeof(JtCliqueShape));
        if (e == hipSuccess) e = up(P.off_card, P.card.data(), P.card.size() * sizeof(int32_t));
    }
    int64_t src_off = 0;
    for (int32_t c = 0; c < P.n_cliques && e == hipSuccess && init_potentials; ++c) {
        const jt::CliqueInfo &C = P.cl[c];
        e = hipMemcpyAsync(base + P.off_init + C.init_off * sizeof(float), init_potentials + src_off,
                           (size_t)C.size * sizeof(float), hipMemcpyDefault, s);
        src_off += C.size;
    }
    return e;
}

// Before a propagation over slots [0, n_active): upload the evidence of the
// slots whose evidence changed and, for a batched tree, the dynamic schedule
// (collect sources and work lists) when the evidence or n_active changed.
jt_status prepare(jt_tree t, int n_active, bool fused) {
    const jt::Plan &P = t->plan;
    const int R = P.n_regions;
    int lo = R, hi = -1;
    for (int r = 0; r < R; ++r)
        if (t->ev_dirty[r]) {
            jt::evidence_tables(P, t->ev_vars[r], t->ev_states[r], &t->ev_idx_host[(size_t)r * P.ev_idx_stride],
                                &t->ev_ent_host[(size_t)r * P.ev_ent_stride]);
            t->ev_dirty[r] = 0;
            lo = std::min(lo, r);
            hi = std::max(hi, r);
        }
    const bool dyn = P.share && fused && (t->dyn_version != t->ev_version || t->dyn_n_active != n_active);
    if (hi < 0 && !dyn) return JT_OK;
    hipError_t e = stage_begin(t->stage);
    if (e != hipSuccess) return hip_err(e, "staging");
    if (hi >= 0) {
        const size_t n = (size_t)(hi - lo + 1);
        e = stage_put(t->stage, t->ws + P.off_ev_idx + (size_t)lo * P.ev_idx_stride * sizeof(int32_t),
                      &t->ev_idx_host[(size_t)lo * P.ev_idx_stride], n * P.ev_idx_stride * sizeof(int32_t), t->stream);
        if (e == hipSuccess)
            e = stage_put(t->stage, t->ws + P.off_ev_ent + (size_t)lo * P.ev_ent_stride * sizeof(JtEv),
                          &t->ev_ent_host[(size_t)lo * P.ev_ent_stride], n * P.ev_ent_stride * sizeof(JtEv),
                          t->stream);
    }
    if (e == hipSuccess && dyn) {
        try {
            jt::build_dynamic(P, t->ev_vars, n_active, t->dyn);
        } catch (const std::bad_alloc &) {
            return set_err(JT_E_NO_MEM, "host allocation failed");
        } catch (const std::exception &x) {
            return set_err(JT_E_ARG, std::string("schedule: ") + x.what());
        }
        t->dyn_version = t->ev_version;
        t->dyn_n_active = n_active;
        e = stage_put(t->stage, t->ws + P.off_csrc, t->dyn.csrc.data(), t->dyn.csrc.size() * sizeof(int32_t),
                      t->stream);
        if (e == hipSuccess)
            e = stage_put(t->stage, t->ws + P.off_work_count, t->dyn.count.data(),
                          t->dyn.count.size() * sizeof(int32_t), t->stream);
        if (e == hipSuccess)
            e = stage_put(t->stage, t->ws + P.off_work, t->dyn.work.data(), t->dyn.work.size() * sizeof(JtWork),
                          t->stream);
        if (e == hipSuccess && P.chunk_total > 0)
            e = stage_put(t->stage, t->ws + P.off_chunks, t->dyn.chunks.data(),
                          t->dyn.chunks.size() * sizeof(JtChunk), t->stream);
    }
    hipError_t e2 = stage_end(t->stage, t->stream);
    if (e != hipSuccess) return hip_err(e, "evidence upload");
    if (e2 != hipSuccess) return hip_err(e2, "evidence upload");
    return JT_OK;
}

// Launch flags: batched fused launches read collect data through the collect
// sources.
int launch_flags(const jt::Plan &P, bool fused) { return (P.share && fused) ? JT_PF_SHARE : 0; }

// Launch list L on the bound stream and, for launches of a lane, on that
// lane's stream: the lanes first wait for the bound stream (fork), a launch
// marked join_before first makes the bound stream wait for every lane, one
// marked fork_after lets the lanes continue after it, and the bound stream
// waits for every lane at the end.  Under stream capture this records a
// graph whose lane branches run side by side.
jt_status enqueue(jt_tree t, const JtDev &d, const std::vector<jt::Launch> &L, int S, bool fused, hipStream_t stream,
                  const std::vector<int32_t> *grids) {
    bool lanes = false;
    for (const jt::Launch &l : L) lanes = lanes || l.lane >= 0;
    if (lanes && (t->lane_stream.empty() || stream != t->stream)) return set_err(JT_E_STATE, "lane streams missing");
    auto fork = [&]() -> hipError_t {
        hipError_t e = hipEventRecord(t->fork_ev, stream);
        for (hipStream_t ls : t->lane_stream)
            if (e == hipSuccess) e = hipStreamWaitEvent(ls, t->fork_ev, 0);
        return e;
    };
    auto join = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (size_t k = 0; k < t->lane_stream.size() && e == hipSuccess; ++k) {
            e = hipEventRecord(t->lane_done[k], t->lane_stream[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(stream, t->lane_done[k], 0);
        }
        return e;
    };
    hipError_t e = lanes ? fork() : hipSuccess;
    if (e != hipSuccess) return hip_err(e, "lane fork");
    // A level's multi-slot and one-slot distribute launches touch disjoint
    // (task, slot) pairs and read the same finished messages, so the
    // multi-slot one runs on the side stream (forked from the bound stream
    // by an event, i.e. after every earlier one-slot launch) while the
    // one-slot one runs on the bound stream.  A one-slot pair has evidence
    // below its clique, so its parent pass ran one-slot as well: the bound
    // stream goes on to the next level without waiting for the side stream,
    // except before a launch marked after_multi and at the end of the list
    // (join event).  Inside a captured graph these are parallel branches;
    // the one-slot launch is enqueued first, so that in the graph it is the
    // first child of the previous level's one-slot node (the runtime keeps a
    // node's first child on that node's stream) and the multi-slot nodes
    // form the branch.
    bool pending_join = false;
    // host-side trace ranges (roctx) around the enqueue of each sweep of the
    // fused schedule, "jt collect sweep" then "jt distribute sweep"; the open
    // one is closed on every way out
    struct SweepRange {
        int open = -1;   // -1 none, 0 collect, 1 distribute
        void to(int next) {
            if (next == open) return;
            if (open >= 0) roctxRangePop();
            if (next >= 0) roctxRangePushA(next == 0 ? "jt collect sweep" : "jt distribute sweep");
            open = next;
        }
        ~SweepRange() { to(-1); }
    } sweep;
    const jt::Launch *deferred = nullptr;   // multi-slot launch waiting for its level's one-slot launch
    int deferred_grid = 0;
    auto launch_deferred = [&]() -> hipError_t {
        const jt::Launch &m = *deferred;
        deferred = nullptr;
        hipError_t r = jt_launch_pass_multi(d, m.begin, m.lds_floats, m.work_off, m.work_idx, deferred_grid, t->side);
        if (r == hipSuccess) r = hipEventRecord(t->side_join, t->side);
        pending_join = r == hipSuccess;
        return r;
    };
    for (const jt::Launch &l : L) {
        if (l.join_before && lanes) {
            e = join();
            if (e != hipSuccess) return hip_err(e, "lane join");
        }
        if (pending_join && !l.multi && (l.after_multi || l.collect || l.is_pass != 1)) {
            e = hipStreamWaitEvent(stream, t->side_join, 0);
            pending_join = false;
            if (e != hipSuccess) return hip_err(e, "side stream join");
        }
        hipStream_t s = l.lane >= 0 ? t->lane_stream[l.lane] : stream;
        if (fused && l.is_pass == 1) sweep.to(l.collect ? 0 : 1);
        if (l.is_pass == 2) {
            e = jt_launch_plain_init(d, S, s);
        } else if (l.count > 0) {
            if ((int64_t)l.count * S > 0x7fffffffLL) return set_err(JT_E_TOO_LARGE, "grid too large");
            int grid = 0;
            if (l.listed) {
                if (!grids || l.work_idx >= (int32_t)grids->size()) return set_err(JT_E_STATE, "work lists missing");
                grid = (*grids)[l.work_idx];
                if (grid < 1 || grid > l.work_cap) return set_err(JT_E_STATE, "listed grid out of range");
            }
            if (l.multi && t->side && s == stream) {
                // forked here (after every earlier one-slot launch), launched
                // after the level's one-slot launch has been enqueued
                if (deferred) e = launch_deferred();
                if (e == hipSuccess) e = hipEventRecord(t->side_fork, stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(t->side, t->side_fork, 0);
                deferred = &l;
                deferred_grid = grid;
            } else if (l.multi)
                e = jt_launch_pass_multi(d, l.begin, l.lds_floats, l.work_off, l.work_idx, grid, s);
            else
                e = jt_launch_pass(d, l.begin, l.count, S, l.lds_floats, launch_flags(t->plan, fused),
                                   l.listed ? l.work_off : -1, l.work_idx, grid, s);
        }
        if (e == hipSuccess && deferred && !l.multi) e = launch_deferred();
        if (e != hipSuccess) return hip_err(e, "kernel launch");
        if (l.fork_after && lanes) {
            e = fork();
            if (e != hipSuccess) return hip_err(e, "lane fork");
        }
    }
    if (deferred) {
        e = launch_deferred();
        if (e != hipSuccess) return hip_err(e, "kernel launch");
    }
    sweep.to(-1);
    if (pending_join) {
        e = hipStreamWaitEvent(stream, t->side_join, 0);
        if (e != hipSuccess) return hip_err(e, "side stream join");
    }
    if (lanes) {
        e = join();
        if (e != hipSuccess) return hip_err(e, "lane join");
    }
    return JT_OK;
}

}  // namespace jt_detail

namespace {

// The paper-faithful schedule for slots [0, S): separators := 1 and
// log-scales := 0 for all, then each slot's messages one after the other.
jt_status enqueue_paper(jt_tree t, int S, hipStream_t stream) {
    const jt::PaperPlan &pp = t->paper;
    hipError_t e = jt_launch_plain_init(t->dev, S, stream);
    for (int s = 0; s < S && e == hipSuccess; ++s)
        e = jt_launch_paper_slot(t->dev, pp.msgs.data(), (int)pp.msgs.size(),
                                 reinterpret_cast<const JtPaperBlk *>(t->paper_ws + pp.off_blocks),
                                 (int)pp.blocks.size(), reinterpret_cast<const int32_t *>(t->paper_ws + pp.off_mu),
                                 t->paper_layout, t->paper_tpb, t->plan.user_root, s, stream);
    if (e != hipSuccess) return hip_err(e, "paper schedule launch");
    return JT_OK;
}

void drop_lanes(jt_tree t) {
    for (hipStream_t s : t->lane_stream)
        if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t e : t->lane_done)
        if (e) (void)hipEventDestroy(e);
    if (t->fork_ev) (void)hipEventDestroy(t->fork_ev);
    if (t->side) (void)hipStreamDestroy(t->side);
    if (t->side_fork) (void)hipEventDestroy(t->side_fork);
    if (t->side_join) (void)hipEventDestroy(t->side_join);
    t->side = nullptr;
    t->side_fork = t->side_join = nullptr;
    t->lane_stream.clear();
    t->lane_done.clear();
    t->fork_ev = nullptr;
}

constexpr size_t kMaxGraphs = 64;

void drop_graph(jt_tree t) {
    for (auto &kv : t->graphs) {
        if (kv.second.second) (void)hipGraphExecDestroy(kv.second.second);
        if (kv.second.first) (void)hipGraphDestroy(kv.second.first);
    }
    t->graphs.clear();
}

// Capture the launches of one propagation once per number of active slots
// (and, for a batched tree, per set of listed grid sizes), then replay the
// graph.
jt_status run_graph(jt_tree t, int S, bool paper = false) {
    std::vector<int32_t> key{paper ? -S : S};
    if (t->plan.share && !paper) key.insert(key.end(), t->dyn.grid.begin(), t->dyn.grid.end());
    if (paper) {
        key.push_back(t->paper_layout);
        key.push_back(t->paper_tpb);
    }
    auto f = t->graphs.find(key);
    if (f == t->graphs.end()) {
        if (t->graphs.size() >= kMaxGraphs) {
            // bounded cache: let queued replays finish, then start over
            hipError_t e = hipStreamSynchronize(t->stream);
            if (e != hipSuccess) return hip_err(e, "stream synchronize");
            drop_graph(t);
        }
        hipError_t e = hipStreamBeginCapture(t->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_err(e, "begin capture");
        jt_status rc = paper ? enqueue_paper(t, S, t->stream)
                             : enqueue(t, t->dev, t->plan.fused, S, true, t->stream, &t->dyn.grid);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(t->stream, &g);
        if (rc != JT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_err(e, "end capture");
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_err(e, "graph instantiate");
        }
        f = t->graphs.emplace(key, std::make_pair(g, x)).first;
    }
    hipError_t e = hipGraphLaunch(f->second.second, t->stream);
    if (e != hipSuccess) return hip_err(e, "graph launch");
    return JT_OK;
}

// Record what the propagation just enqueued moves (FP32 table bytes).
void note_last(jt_tree t, int mode, int n_active) {
    const jt::Plan &P = t->plan;
    t->last_launch_bytes.clear();
    if (mode == JT_MODE_FUSED || mode == JT_MODE_GRAPH)
        for (size_t k = 0; k < P.fused.size(); ++k)
            if (P.fused[k].count > 0)
                t->last_launch_bytes.push_back(P.share ? t->dyn.launch_bytes[k] : P.fused[k].bytes);
    if (mode == JT_MODE_PAPER || mode == JT_MODE_PAPER_GRAPH) {
        // tables: reset (init read, table written), each message reads the
        // sender and reads and writes the receiver, read-out reads and
        // writes every table; mapping lists are not counted
        int64_t b = 0;
        for (const JtPaperMsg &m : t->paper.msgs) b += 4 * (m.m_from + 2 * (int64_t)m.m_to) * m.ssize;
        t->last_bytes = (b + 4 * 4 * P.total_entries) * n_active;
        t->last_shared = 0;
        t->last_collect_pairs = 0;
    } else if (mode == JT_MODE_PLAIN) {
        t->last_bytes = P.bytes_plain;
        t->last_shared = 0;
        t->last_collect_pairs = 0;
    } else if (P.share) {
        t->last_bytes = t->dyn.bytes;
        t->last_shared = t->dyn.shared;
        t->last_collect_pairs = t->dyn.collect_pairs;
    } else {
        t->last_bytes = P.bytes_fused;
        t->last_shared = 0;
        t->last_collect_pairs = (int64_t)P.n_cliques * n_active;
    }
}

jt_status read_slot(jt_tree t, int32_t slot, double *log_z, bool *zero) {
    const jt::Plan &P = t->plan;
    int32_t flag = 0;
    double lz = 0.0;
    hipError_t e = hipStreamSynchronize(t->stream);
    if (e != hipSuccess) return hip_err(e, "stream synchronize");
    e = hipMemcpy(&flag, t->ws + P.off_flag + (size_t)slot * sizeof(int32_t), sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(e, "read flag");
    e = hipMemcpy(&lz, t->ws + P.off_lam + ((size_t)slot * P.lam_stride + JT_LAM_LOGZ(P.n_cliques)) * sizeof(double),
                  sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_err(e, "read log Z");
    *zero = flag != 0;
    if (log_z) *log_z = *zero ? -INFINITY : lz;
    return JT_OK;
}

}  // namespace

extern "C" {

const char *jt_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

jt_status new_handle(const jt_tree_desc *desc, jt_tree *out, size_t *device_bytes, const jt::BnTree *bn,
                     const jt::MergedTree *merged = nullptr) {
    try {
        if (!out || !device_bytes) return set_err(JT_E_ARG, "out or device_bytes is NULL");
        *out = nullptr;
        jt_tree t = new jt_tree_s();
        std::string err;
        const std::vector<jt::FamilyReq> *fam = bn ? &bn->families : merged ? &merged->families : nullptr;
        const int64_t ftot = bn ? bn->cpt_total : merged ? merged->total : 0;
        const jt_status rc = jt::compile_plan(desc, t->plan, err, fam, ftot);
        if (rc != JT_OK) {
            delete t;
            return set_err(rc, err);
        }
        if (bn) {
            t->is_bn = true;
            t->bn = *bn;
        }
        if (merged) {
            t->is_merged = true;
            t->merged = *merged;
        }
        const jt::Plan &P = t->plan;
        t->ev_vars.assign(P.n_regions, {});
        t->ev_states.assign(P.n_regions, {});
        t->ev_dirty.assign(P.n_regions, 1);
        t->ev_idx_host.assign((size_t)P.n_regions * P.ev_idx_stride, 0);
        t->ev_ent_host.assign((size_t)P.n_regions * P.ev_ent_stride, JtEv{0, 1, 1, 0});
        *device_bytes = P.total_bytes;
        *out = t;
        g_err.clear();
        return JT_OK;
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    } catch (...) {
        return set_err(JT_E_ARG, "unexpected failure in compiling the tree");
    }
}

}  // namespace

extern "C" {

jt_status jt_compile_index_maps(const jt_tree_desc *desc, jt_tree *out, size_t *device_bytes) {
    return new_handle(desc, out, device_bytes, nullptr);
}

jt_status jt_compile_bn(const jt_bn_desc *bn, jt_tree *out, size_t *device_bytes, int32_t *n_cliques) {
    try {
        if (!out || !device_bytes || !n_cliques) return set_err(JT_E_ARG, "NULL output");
        *out = nullptr;
        jt::BnTree T;
        std::string err;
        const jt_status rc = jt::compile_bn(bn, T, err);
        if (rc != JT_OK) return set_err(rc, err);
        const int32_t nc = (int32_t)T.cliques.size();
        std::vector<int64_t> off(nc + 1, 0);
        std::vector<int32_t> vars;
        for (int32_t c = 0; c < nc; ++c) {
            vars.insert(vars.end(), T.cliques[c].begin(), T.cliques[c].end());
            off[c + 1] = (int64_t)vars.size();
        }
        jt_tree_desc d{bn->n_vars, T.card.data(), nc, off.data(), vars.data(), T.parent.data(), bn->n_slots, bn->tuning};
        const jt_status rc2 = new_handle(&d, out, device_bytes, &T);
        if (rc2 == JT_OK) *n_cliques = nc;
        return rc2;
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    }
}

jt_status jt_compile_merged(const jt_tree_desc *desc, int32_t max_sep, int64_t max_entries, jt_tree *out,
                            size_t *device_bytes, int32_t *n_compiled) {
    try {
        if (!desc || !out || !device_bytes || !n_compiled) return set_err(JT_E_ARG, "NULL argument");
        *out = nullptr;
        jt::MergedTree M;
        std::string err;
        const jt_status rc = jt::merge_tree(desc, max_sep, max_entries, M, err);
        if (rc != JT_OK) return set_err(rc, err);
        const int32_t nm = (int32_t)M.cliques.size();
        std::vector<int64_t> off(nm + 1, 0);
        std::vector<int32_t> vars;
        for (int32_t c = 0; c < nm; ++c) {
            vars.insert(vars.end(), M.cliques[c].begin(), M.cliques[c].end());
            off[c + 1] = (int64_t)vars.size();
        }
        jt_tree_desc d{desc->n_vars, M.card.data(), nm, off.data(), vars.data(), M.parent.data(), desc->n_slots,
                       desc->tuning};
        const jt_status rc2 = new_handle(&d, out, device_bytes, nullptr, &M);
        if (rc2 == JT_OK) *n_compiled = nm;
        return rc2;
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    }
}

jt_status jt_bn_structure(jt_tree t, int64_t *clique_off, int32_t *clique_vars, int32_t *parent,
                          int32_t *family_clique) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->is_bn) return set_err(JT_E_STATE, "not a network tree");
    if (!clique_off || !clique_vars || !parent || !family_clique) return set_err(JT_E_ARG, "NULL output");
    const jt::BnTree &B = t->bn;
    int64_t k = 0;
    clique_off[0] = 0;
    for (size_t c = 0; c < B.cliques.size(); ++c) {
        for (int32_t v : B.cliques[c]) clique_vars[k++] = v;
        clique_off[c + 1] = k;
        parent[c] = B.parent[c];
    }
    for (const jt::FamilyReq &f : B.families) family_clique[f.var] = f.clique;
    return JT_OK;
}

}  // extern "C"

namespace {

jt_status bind_common(jt_tree t, void *workspace, size_t bytes, const float *init_potentials, void *hip_stream) {
    const jt::Plan &P = t->plan;
    if (!workspace) return set_err(JT_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return set_err(JT_E_ARG, "workspace not 256-byte aligned");
    if (bytes < P.total_bytes)
        return set_err(JT_E_NO_MEM, "workspace of " + std::to_string(bytes) + " bytes, need " + std::to_string(P.total_bytes));
    // work still queued on the previous binding finishes before its objects go
    if (t->bound && t->stream) (void)hipStreamSynchronize(t->stream);
    drop_graph(t);
    drop_lanes(t);
    drop_staging(t->stage);
    if (P.share) {
        // default priority, like every stream here
        hipError_t se = hipStreamCreateWithFlags(&t->side, hipStreamNonBlocking);
        if (se == hipSuccess) se = hipEventCreateWithFlags(&t->side_fork, hipEventDisableTiming);
        if (se == hipSuccess) se = hipEventCreateWithFlags(&t->side_join, hipEventDisableTiming);
        if (se != hipSuccess) {
            drop_lanes(t);
            return hip_err(se, "side stream");
        }
    }
    if (P.n_lanes > 0) {
        hipError_t le = hipEventCreateWithFlags(&t->fork_ev, hipEventDisableTiming);
        for (int32_t k = 0; k < P.n_lanes && le == hipSuccess; ++k) {
            hipStream_t ls = nullptr;
            hipEvent_t de = nullptr;
            le = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking);
            if (le == hipSuccess) t->lane_stream.push_back(ls);
            if (le == hipSuccess) le = hipEventCreateWithFlags(&de, hipEventDisableTiming);
            if (le == hipSuccess) t->lane_done.push_back(de);
        }
        if (le != hipSuccess) {
            drop_lanes(t);
            return hip_err(le, "lane streams");
        }
    }
    {
        Staging &S = t->stage;
        S.cap = P.dyn_bytes + 4096;
        hipError_t se = hipSuccess;
        for (int k = 0; k < 2 && se == hipSuccess; ++k) {
            se = hipHostMalloc(reinterpret_cast<void **>(&S.host[k]), S.cap, hipHostMallocDefault);
            if (se == hipSuccess) se = hipEventCreateWithFlags(&S.done[k], hipEventDisableTiming);
        }
        if (se != hipSuccess) {
            drop_staging(S);
            return hip_err(se, "pinned staging buffers");
        }
    }
    t->ws = static_cast<char *>(workspace);
    t->ws_bytes = bytes;
    t->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = upload_static(P, t->ws, init_potentials, t->stream);
    if (e != hipSuccess) return hip_err(e, "jt_bind upload");
    fill_dev(P, t->ws, t->dev);
    std::fill(t->ev_dirty.begin(), t->ev_dirty.end(), 1);
    t->dyn_version = 0;
    t->dyn_n_active = -1;
    t->bound = true;
    t->propagated = false;
    g_err.clear();
    return JT_OK;
}

}  // namespace

extern "C" {

jt_status bind_families(jt_tree t, void *workspace, size_t bytes, const float *cpts, void *hip_stream);

jt_status jt_bind(jt_tree t, void *workspace, size_t bytes, const float *init_potentials, void *hip_stream) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!init_potentials) return set_err(JT_E_ARG, "init_potentials is NULL");
    if (t->is_bn) return set_err(JT_E_STATE, "a network tree is bound with jt_bind_bn");
    // a merged tree's tables are the products of the caller's tables
    if (t->is_merged) return bind_families(t, workspace, bytes, init_potentials, hip_stream);
    return bind_common(t, workspace, bytes, init_potentials, hip_stream);
}

jt_status jt_bind_bn(jt_tree t, void *workspace, size_t bytes, const float *cpts, void *hip_stream) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->is_bn) return set_err(JT_E_STATE, "not a network tree");
    if (!cpts) return set_err(JT_E_ARG, "cpts is NULL");
    return bind_families(t, workspace, bytes, cpts, hip_stream);
}

// Bind, then compute every clique's table as the product of its families'
// tables (the conditional tables of a network, or a merged tree's original
// clique tables), and upload the families' mapping lists.
jt_status bind_families(jt_tree t, void *workspace, size_t bytes, const float *cpts, void *hip_stream) {
    if (jt_status rc = bind_common(t, workspace, bytes, nullptr, hip_stream)) return rc;
    const jt::Plan &P = t->plan;
    hipError_t e = hipSuccess;
    try {
        std::vector<int32_t> mu((size_t)std::max<int64_t>(1, P.fam_mu_total));
        jt::family_mu_lists(P, mu.data());
        e = hipMemcpyAsync(t->ws + P.off_fam_mu, mu.data(), (size_t)P.fam_mu_total * sizeof(int32_t),
                           hipMemcpyHostToDevice, t->stream);
        if (e == hipSuccess)
            e = jt_launch_bn_init(t->dev, reinterpret_cast<const JtFamily *>(t->ws + P.off_fam),
                                  reinterpret_cast<const int32_t *>(t->ws + P.off_fam_rng),
                                  reinterpret_cast<const JtCliqueShape *>(t->ws + P.off_cshape), P.n_cliques,
                                  P.max_tiles, cpts, t->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(t->stream);   // `mu` and `cpts` are read by now
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    }
    if (e != hipSuccess) {
        t->bound = false;
        return hip_err(e, "network initialization");
    }
    return JT_OK;
}

jt_status jt_bn_set_cpts(jt_tree t, const float *cpts) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->is_bn) return set_err(JT_E_STATE, "not a network tree");
    if (!t->bound) return set_err(JT_E_STATE, "jt_bn_set_cpts before jt_bind_bn");
    if (!cpts) return set_err(JT_E_ARG, "cpts is NULL");
    const jt::Plan &P = t->plan;
    hipError_t e = jt_launch_bn_init(t->dev, reinterpret_cast<const JtFamily *>(t->ws + P.off_fam),
                                     reinterpret_cast<const int32_t *>(t->ws + P.off_fam_rng),
                                     reinterpret_cast<const JtCliqueShape *>(t->ws + P.off_cshape), P.n_cliques,
                                     P.max_tiles, cpts, t->stream);
    if (e != hipSuccess) return hip_err(e, "network initialization");
    t->propagated = false;
    return JT_OK;
}

jt_status jt_bn_m_step(jt_tree t, const float *counts, float alpha, float *cpts) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->is_bn) return set_err(JT_E_STATE, "not a network tree");
    if (!t->bound) return set_err(JT_E_STATE, "jt_bn_m_step before jt_bind_bn");
    if (!counts || !cpts || !(alpha >= 0.f)) return set_err(JT_E_ARG, "NULL pointer or negative alpha");
    const jt::Plan &P = t->plan;
    int64_t rows = 1;
    for (const JtFamily &F : P.fam) rows = std::max<int64_t>(rows, F.fsize / P.card[F.var]);
    hipError_t e = jt_launch_bn_mstep(reinterpret_cast<const JtFamily *>(t->ws + P.off_fam), (int)P.fam.size(), rows,
                                      reinterpret_cast<const int32_t *>(t->ws + P.off_card), counts, alpha, cpts,
                                      t->stream);
    if (e != hipSuccess) return hip_err(e, "M-step launch");
    return JT_OK;
}

jt_status jt_bn_expected_counts(jt_tree t, int32_t n_active, float *counts) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->is_bn) return set_err(JT_E_STATE, "not a network tree");
    if (!counts) return set_err(JT_E_ARG, "counts is NULL");
    if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
    if (n_active < 1 || n_active > t->last_n_active) return set_err(JT_E_STATE, "slots not active in the last propagation");
    const jt::Plan &P = t->plan;
    hipError_t e = jt_launch_family_marginal(t->dev, reinterpret_cast<const JtFamily *>(t->ws + P.off_fam), 0,
                                             (int)P.fam.size(), P.max_fsize,
                                             reinterpret_cast<const int32_t *>(t->ws + P.off_fam_mu),
                                             reinterpret_cast<const JtCliqueShape *>(t->ws + P.off_cshape), 0, n_active,
                                             counts, 0, t->stream);
    if (e != hipSuccess) return hip_err(e, "expected counts launch");
    return JT_OK;
}

jt_status jt_set_evidence(jt_tree t, int32_t slot, int32_t n_obs, const int32_t *vars, const int32_t *states) {
    if (jt_status rc = check_tree(t)) return rc;
    const jt::Plan &P = t->plan;
    if (slot < 0 || slot >= P.n_slots) return set_err(JT_E_ARG, "slot out of range");
    if (n_obs < 0 || (n_obs > 0 && (!vars || !states))) return set_err(JT_E_ARG, "bad evidence arrays");
    std::vector<int32_t> seen(P.n_vars, -1);
    for (int32_t a = 0; a < n_obs; ++a) {
        const int32_t v = vars[a], s = states[a];
        if (v < 0 || v >= P.n_vars) return set_err(JT_E_ARG, "evidence variable out of range");
        if (s < 0 || s >= P.card[v]) return set_err(JT_E_ARG, "evidence state out of range");
        if (seen[v] >= 0 && seen[v] != s) return set_err(JT_E_ARG, "conflicting evidence for one variable");
        seen[v] = s;
    }
    t->ev_vars[slot].assign(vars, vars + n_obs);
    t->ev_states[slot].assign(states, states + n_obs);
    t->ev_dirty[slot] = 1;
    ++t->ev_version;
    return JT_OK;
}

jt_status jt_propagate_n(jt_tree t, int32_t mode, int32_t n_active) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->bound) return set_err(JT_E_STATE, "jt_propagate before jt_bind");
    if (mode != JT_MODE_FUSED && mode != JT_MODE_GRAPH && mode != JT_MODE_PLAIN && mode != JT_MODE_DATAFLOW &&
        mode != JT_MODE_PAPER && mode != JT_MODE_PAPER_GRAPH)
        return set_err(JT_E_ARG, "unknown mode");
    if (n_active < 1 || n_active > t->plan.n_slots) return set_err(JT_E_ARG, "n_active out of range");
    if (mode == JT_MODE_DATAFLOW) return dataflow_disabled();
    const bool paper = mode == JT_MODE_PAPER || mode == JT_MODE_PAPER_GRAPH;
    if (paper && !t->paper_ws) return set_err(JT_E_STATE, "paper schedule before jt_paper_bind");
    if (jt_status rc = prepare(t, n_active, mode == JT_MODE_FUSED || mode == JT_MODE_GRAPH)) return rc;
    // host-side trace range (roctx) around one propagation's enqueue or graph launch
    roctxRangePushA("jt_propagate");
    jt_status rc = JT_OK;
    if (mode == JT_MODE_PAPER)
        rc = enqueue_paper(t, n_active, t->stream);
    else if (mode == JT_MODE_PAPER_GRAPH)
        rc = run_graph(t, n_active, true);
    else if (mode == JT_MODE_FUSED)
        rc = enqueue(t, t->dev, t->plan.fused, n_active, true, t->stream, &t->dyn.grid);
    else if (mode == JT_MODE_PLAIN)
        rc = enqueue(t, t->dev, t->plan.plain, n_active, false, t->stream, nullptr);
    else
        rc = run_graph(t, n_active);
    roctxRangePop();
    if (rc == JT_OK) {
        t->propagated = true;
        t->last_mode = mode;
        t->last_n_active = n_active;
        note_last(t, mode, n_active);
    }
    return rc;
}

jt_status jt_propagate(jt_tree t, int32_t mode) {
    if (jt_status rc = check_tree(t)) return rc;
    return jt_propagate_n(t, mode, t->plan.n_slots);
}

}  // extern "C"

namespace {

// Merged trees: the posteriors of original cliques [c0, c0 + n) of one slot,
// marginalized from their merged cliques into the staging region, then
// copied to `out` (host or device).
jt_status merged_read(jt_tree t, int32_t slot, int32_t c0, int32_t n, float *out) {
    const jt::Plan &P = t->plan;
    const JtFamily *fam = reinterpret_cast<const JtFamily *>(t->ws + P.off_fam);
    float *stage = reinterpret_cast<float *>(t->ws + P.off_stage);
    // families are sorted by merged clique: find the records of c0 .. c0+n-1
    hipError_t e = hipSuccess;
    int64_t lo = -1, hi = -1;
    for (size_t k = 0; k < P.fam.size() && e == hipSuccess; ++k) {
        const int32_t oc = P.fam[k].var;
        if (oc < c0 || oc >= c0 + n) continue;
        e = jt_launch_family_marginal(t->dev, fam, (int)k, 1, P.fam[k].fsize,
                                      reinterpret_cast<const int32_t *>(t->ws + P.off_fam_mu),
                                      reinterpret_cast<const JtCliqueShape *>(t->ws + P.off_cshape), slot, 1, stage, 0,
                                      t->stream);
        lo = lo < 0 ? P.fam[k].cpt_off : std::min<int64_t>(lo, P.fam[k].cpt_off);
        hi = std::max<int64_t>(hi, P.fam[k].cpt_off + P.fam[k].fsize);
    }
    if (e == hipSuccess && lo >= 0)
        e = hipMemcpyAsync(out, stage + lo, (size_t)(hi - lo) * sizeof(float), hipMemcpyDefault, t->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(t->stream);
    if (e != hipSuccess) return hip_err(e, "merged read-out");
    return JT_OK;
}

}  // namespace

extern "C" {

jt_status jt_marginal(jt_tree t, int32_t slot, int32_t clique, float *out, double *log_z) {
    if (jt_status rc = check_tree(t)) return rc;
    const jt::Plan &P = t->plan;
    if (slot < 0 || slot >= P.n_slots) return set_err(JT_E_ARG, "slot out of range");
    const int32_t n_user = t->is_merged ? (int32_t)t->merged.orig_size.size() : P.n_cliques;
    if (clique < 0 || clique >= n_user) return set_err(JT_E_ARG, "clique out of range");
    if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
    if (slot >= t->last_n_active) return set_err(JT_E_STATE, "slot was not active in the last propagation");
    bool zero = false;
    if (jt_status rc = read_slot(t, slot, log_z, &zero)) return rc;
    if (zero) return set_err(JT_E_ZERO_EVIDENCE, "evidence has probability zero");
    if (out && t->is_merged) return merged_read(t, slot, clique, 1, out);
    if (out) {
        const jt::CliqueInfo &C = P.cl[clique];
        hipError_t e = hipMemcpy(out, t->ws + P.off_out + ((size_t)slot * P.out_stride + C.out_off) * sizeof(float),
                                 (size_t)C.size * sizeof(float), hipMemcpyDefault);
        if (e != hipSuccess) return hip_err(e, "copy marginal");
    }
    return JT_OK;
}

jt_status jt_marginals_all(jt_tree t, int32_t slot, float *out, double *log_z) {
    if (jt_status rc = check_tree(t)) return rc;
    const jt::Plan &P = t->plan;
    if (slot < 0 || slot >= P.n_slots) return set_err(JT_E_ARG, "slot out of range");
    if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
    if (slot >= t->last_n_active) return set_err(JT_E_STATE, "slot was not active in the last propagation");
    bool zero = false;
    if (jt_status rc = read_slot(t, slot, log_z, &zero)) return rc;
    if (zero) return set_err(JT_E_ZERO_EVIDENCE, "evidence has probability zero");
    if (out && t->is_merged) return merged_read(t, slot, 0, (int32_t)t->merged.orig_size.size(), out);
    if (out) {
        int64_t dst = 0;
        for (int32_t c = 0; c < P.n_cliques; ++c) {
            const jt::CliqueInfo &C = P.cl[c];
            hipError_t e = hipMemcpyAsync(out + dst,
                                          t->ws + P.off_out + ((size_t)slot * P.out_stride + C.out_off) * sizeof(float),
                                          (size_t)C.size * sizeof(float), hipMemcpyDefault, t->stream);
            if (e != hipSuccess) return hip_err(e, "copy marginals");
            dst += C.size;
        }
        hipError_t e = hipStreamSynchronize(t->stream);
        if (e != hipSuccess) return hip_err(e, "stream synchronize");
    }
    return JT_OK;
}

jt_status jt_read_out(jt_tree t, int32_t slot0, int32_t n, float *posteriors, double *log_z) {
    if (jt_status rc = check_tree(t)) return rc;
    const jt::Plan &P = t->plan;
    if (!posteriors || !log_z) return set_err(JT_E_ARG, "NULL output pointer");
    if (slot0 < 0 || n < 1 || (int64_t)slot0 + n > P.n_slots) return set_err(JT_E_ARG, "slot range out of range");
    if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
    if (slot0 + n > t->last_n_active) return set_err(JT_E_STATE, "slot was not active in the last propagation");
    hipError_t e = jt_launch_read_out(t->dev, slot0, n, P.total_entries, posteriors, log_z, t->stream);
    if (e != hipSuccess) return hip_err(e, "read-out launch");
    return JT_OK;
}

jt_status jt_paper_bytes(jt_tree t, size_t *bytes) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!bytes) return set_err(JT_E_ARG, "bytes is NULL");
    try {
        if (!t->paper_planned) {
            jt::build_paper_plan(t->plan, t->paper);
            t->paper_planned = true;
        }
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    }
    *bytes = t->paper.bytes;
    return JT_OK;
}

jt_status jt_paper_bind(jt_tree t, void *workspace, size_t bytes, int32_t layout, int32_t threads_per_block) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->bound) return set_err(JT_E_STATE, "jt_paper_bind before jt_bind");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return set_err(JT_E_ARG, "paper workspace NULL or not 256-byte aligned");
    if (layout != JT_LAYOUT_NAIVE && layout != JT_LAYOUT_INTERLEAVED) return set_err(JT_E_ARG, "unknown layout");
    if (threads_per_block < 1 || threads_per_block > 1024) return set_err(JT_E_ARG, "threads per block out of range");
    size_t need = 0;
    if (jt_status rc = jt_paper_bytes(t, &need)) return rc;
    if (bytes < need) return set_err(JT_E_NO_MEM, "paper workspace of " + std::to_string(bytes) + " bytes, need " +
                                                      std::to_string(need));
    const jt::PaperPlan &pp = t->paper;
    hipError_t e = hipStreamSynchronize(t->stream);   // nothing queued still reads the old lists
    if (e != hipSuccess) return hip_err(e, "stream synchronize");
    try {
        std::vector<int32_t> mu((size_t)std::max<int64_t>(1, pp.mu_total));
        jt::paper_mu_lists(t->plan, pp, layout, mu.data());
        char *ws = static_cast<char *>(workspace);
        e = hipMemcpyAsync(ws + pp.off_msgs, pp.msgs.data(), pp.msgs.size() * sizeof(JtPaperMsg),
                           hipMemcpyHostToDevice, t->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + pp.off_blocks, pp.blocks.data(), pp.blocks.size() * sizeof(JtPaperBlk),
                               hipMemcpyHostToDevice, t->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws + pp.off_mu, mu.data(), (size_t)pp.mu_total * sizeof(int32_t), hipMemcpyHostToDevice,
                               t->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(t->stream);   // `mu` is freed on return
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    }
    if (e != hipSuccess) return hip_err(e, "paper workspace upload");
    // graphs of the paper schedule captured for another layout or block size stay valid (keyed by both)
    t->paper_ws = static_cast<char *>(workspace);
    t->paper_layout = layout;
    t->paper_tpb = threads_per_block;
    return JT_OK;
}

jt_status jt_get_index_map(jt_tree t, int32_t child, int32_t side, int32_t *host_out) {
    if (jt_status rc = check_tree(t)) return rc;
    const jt::Plan &P = t->plan;
    if (child < 0 || child >= P.n_cliques || P.parent[child] < 0) return set_err(JT_E_ARG, "not a child clique");
    if ((side != 0 && side != 1) || !host_out) return set_err(JT_E_ARG, "bad side or NULL output");
    jt::expand_map(P, side == 0 ? P.edge[child].view_child : P.edge[child].view_parent, host_out);
    return JT_OK;
}

jt_status jt_get_mu_lists(jt_tree t, int32_t child, int32_t side, int32_t *host_out) {
    if (jt_status rc = check_tree(t)) return rc;
    const jt::Plan &P = t->plan;
    if (child < 0 || child >= P.n_cliques || P.parent[child] < 0) return set_err(JT_E_ARG, "not a child clique");
    if ((side != 0 && side != 1) || !host_out) return set_err(JT_E_ARG, "bad side or NULL output");
    try {
        const int32_t c = side == 0 ? child : P.parent[child];
        const int64_t n = P.cl[c].size, ss = P.edge[child].ssize, m = n / ss;
        std::vector<int32_t> map(n);
        jt::expand_map(P, side == 0 ? P.edge[child].view_child : P.edge[child].view_parent, map.data());
        std::vector<int64_t> fill(ss, 0);
        for (int64_t r = 0; r < n; ++r) host_out[map[r] * m + fill[map[r]]++] = (int32_t)r;
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    }
    return JT_OK;
}

jt_status jt_query(jt_tree t, int32_t what, int64_t arg, int64_t *out) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!out) return set_err(JT_E_ARG, "out is NULL");
    const jt::Plan &P = t->plan;
    auto nlaunch = [](const std::vector<jt::Launch> &L) {
        int64_t n = 0;
        for (const jt::Launch &l : L) n += (l.is_pass == 2 || l.count > 0) ? 1 : 0;
        return n;
    };
    switch (what) {
        case JT_Q_N_SLOTS: *out = P.n_slots; break;
        case JT_Q_TOTAL_ENTRIES: *out = t->is_merged ? t->merged.total : P.total_entries; break;
        case JT_Q_TABLE_SIZE:
            if (t->is_merged) {
                if (arg < 0 || arg >= (int64_t)t->merged.orig_size.size()) return set_err(JT_E_ARG, "clique out of range");
                *out = t->merged.orig_size[arg];
                break;
            }
            if (arg < 0 || arg >= P.n_cliques) return set_err(JT_E_ARG, "clique out of range");
            *out = P.cl[arg].size;
            break;
        case JT_Q_N_COMPILED_CLIQUES: *out = P.n_cliques; break;
        case JT_Q_COMPILED_TABLE_SIZE:
            if (arg < 0 || arg >= P.n_cliques) return set_err(JT_E_ARG, "clique out of range");
            *out = P.cl[arg].size;
            break;
        case JT_Q_SEP_SIZE:
            if (arg < 0 || arg >= P.n_cliques || P.parent[arg] < 0) return set_err(JT_E_ARG, "not a child clique");
            *out = P.edge[arg].ssize;
            break;
        case JT_Q_ENTRIES_PER_SWEEP: *out = P.entries_per_sweep; break;
        case JT_Q_BYTES_FUSED: *out = P.bytes_fused; break;
        case JT_Q_BYTES_PLAIN: *out = P.bytes_plain; break;
        case JT_Q_N_LAUNCHES_FUSED: *out = nlaunch(P.fused); break;
        case JT_Q_N_LAUNCHES_PLAIN: *out = nlaunch(P.plain); break;
        case JT_Q_HEIGHT: *out = P.height + 1; break;
        case JT_Q_DEPTH: *out = P.depth + 1; break;
        case JT_Q_SLOT_BYTES: *out = (int64_t)P.slot_bytes; break;
        case JT_Q_SHARED_BYTES: *out = (int64_t)P.total_bytes - (int64_t)P.slot_bytes * P.n_slots; break;
        case JT_Q_ROOT: *out = P.root; break;
        case JT_Q_ALG_BYTES: {
            // FP32 bytes a fused propagation must move per slot, per clique
            // and entry: a leaf reads its table twice and writes its
            // posterior (12 B), an inner clique also writes its absorbed
            // table (16 B), the root reads once and writes once (8 B)
            if (arg < 0 || arg > P.n_slots) return set_err(JT_E_ARG, "slot count out of range");
            int64_t b = 0;
            for (int32_t c = 0; c < P.n_cliques; ++c)
                b += P.cl[c].size * (c == P.root ? 8 : P.cl[c].children.empty() ? 12 : 16);
            *out = b * (arg > 0 ? arg : P.n_slots);
            break;
        }
        case JT_Q_TOTAL_CLIQUE_VARS: {
            int64_t k = 0;
            for (const jt::CliqueInfo &C : P.cl) k += (int64_t)C.vars.size();
            *out = k;
            break;
        }
        case JT_Q_CPT_TOTAL: *out = P.cpt_total; break;
        case JT_Q_N_LANES: *out = P.n_lanes; break;
        case JT_Q_CLIQUE_LANE:
            if (arg < 0 || arg >= P.n_cliques) return set_err(JT_E_ARG, "clique out of range");
            *out = P.lane[arg];
            break;
        case JT_Q_FUSED_LAUNCH_KIND:
        case JT_Q_FUSED_LAUNCH_LANE:
        case JT_Q_FUSED_LAUNCH_MULTI:
        case JT_Q_FUSED_LAUNCH_BLOCKS:
        case JT_Q_FUSED_LAUNCH_BYTES: {
            std::vector<const jt::Launch *> live;
            for (const jt::Launch &l : P.fused)
                if (l.count > 0) live.push_back(&l);
            if (arg < 0 || arg >= (int64_t)live.size()) return set_err(JT_E_ARG, "launch index out of range");
            *out = what == JT_Q_FUSED_LAUNCH_KIND    ? live[arg]->is_pass
                   : what == JT_Q_FUSED_LAUNCH_LANE  ? live[arg]->lane
                   : what == JT_Q_FUSED_LAUNCH_MULTI ? live[arg]->multi
                   : what == JT_Q_FUSED_LAUNCH_BLOCKS ? live[arg]->count
                                                      : live[arg]->bytes;
            break;
        }
        case JT_Q_BYTES_LAST:
            if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
            *out = t->last_bytes;
            break;
        case JT_Q_LAST_SHARED:
            if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
            *out = t->last_shared;
            break;
        case JT_Q_LAST_COLLECT_PASSES:
            if (!t->propagated) return set_err(JT_E_STATE, "nothing propagated yet");
            *out = t->last_collect_pairs;
            break;
        case JT_Q_LAST_LAUNCH_BYTES:
            if (!t->propagated || t->last_launch_bytes.empty())
                return set_err(JT_E_STATE, "no fused propagation yet");
            if (arg < 0 || arg >= (int64_t)t->last_launch_bytes.size())
                return set_err(JT_E_ARG, "launch index out of range");
            *out = t->last_launch_bytes[arg];
            break;
        default: return set_err(JT_E_ARG, "unknown query");
    }
    return JT_OK;
}

jt_status jt_profile(jt_tree t, int32_t mode, double *pass_ms, double *finalize_ms, int32_t *n_pass,
                     int32_t *n_finalize) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!t->bound) return set_err(JT_E_STATE, "jt_profile before jt_bind");
    if (mode != JT_MODE_FUSED && mode != JT_MODE_PLAIN && mode != JT_MODE_DATAFLOW)
        return set_err(JT_E_ARG, "profile mode must be fused, plain or dataflow");
    if (mode == JT_MODE_DATAFLOW) return dataflow_disabled();
    const int S = t->plan.n_slots;
    const bool fused = mode == JT_MODE_FUSED;
    if (jt_status rc = prepare(t, S, fused)) return rc;
    const std::vector<jt::Launch> &L = fused ? t->plan.fused : t->plan.plain;
    t->last_n_active = S;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    jt_status rc = JT_OK;
    hipError_t e = hipSuccess;
    for (const jt::Launch &l : L) {
        if (l.is_pass != 2 && l.count == 0) continue;
        hipEvent_t a = nullptr, b = nullptr;
        e = hipEventCreate(&a);
        if (e == hipSuccess) e = hipEventCreate(&b);
        if (e != hipSuccess) {
            if (a) (void)hipEventDestroy(a);
            rc = hip_err(e, "event create");
            break;
        }
        ev.push_back(a);
        ev.push_back(b);
        kind.push_back(l.is_pass);
        e = hipEventRecord(a, t->stream);
        if (e == hipSuccess) {
            if (l.is_pass == 2)
                e = jt_launch_plain_init(t->dev, S, t->stream);
            else if (l.listed && (size_t)l.work_idx >= t->dyn.grid.size())
                e = hipErrorInvalidValue;
            else if (l.multi)
                e = jt_launch_pass_multi(t->dev, l.begin, l.lds_floats, l.work_off, l.work_idx,
                                         t->dyn.grid[l.work_idx], t->stream);
            else
                e = jt_launch_pass(t->dev, l.begin, l.count, S, l.lds_floats, launch_flags(t->plan, fused),
                                   l.listed ? l.work_off : -1, l.work_idx, l.listed ? t->dyn.grid[l.work_idx] : 0,
                                   t->stream);
        }
        if (e == hipSuccess) e = hipEventRecord(b, t->stream);
        if (e != hipSuccess) {
            rc = hip_err(e, "profiled launch");
            break;
        }
    }
    double tp = 0.0, tf = 0.0;
    int np = 0, nf = 0;
    if (rc == JT_OK) {
        e = hipStreamSynchronize(t->stream);
        if (e != hipSuccess) rc = hip_err(e, "stream synchronize");
    }
    for (size_t i = 0; rc == JT_OK && i < kind.size(); ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
        if (e != hipSuccess) {
            rc = hip_err(e, "event elapsed");
            break;
        }
        if (kind[i] == 1) {
            tp += ms;
            ++np;
        } else {
            tf += ms;
            ++nf;
        }
    }
    for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    if (rc != JT_OK) return rc;
    t->propagated = true;
    t->last_mode = mode;
    note_last(t, mode, S);
    if (pass_ms) *pass_ms = tp;
    if (finalize_ms) *finalize_ms = tf;
    if (n_pass) *n_pass = np;
    if (n_finalize) *n_finalize = nf;
    return JT_OK;
}

void jt_free(jt_tree t) {
    if (!t) return;
    // let queued work on the bound stream finish before its graphs, lane
    // streams and staging buffers go (and before the caller may release the
    // workspace)
    if (t->bound && t->stream) (void)hipStreamSynchronize(t->stream);
    drop_graph(t);
    drop_lanes(t);
    drop_staging(t->stage);
    delete t;
}

}  // extern "C"
