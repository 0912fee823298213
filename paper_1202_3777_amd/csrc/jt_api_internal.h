// jt_api_internal.h -- host-side state of a tree handle and the helpers the
// C ABI's source files share (not part of the public interface).
#pragma once
#include <hip/hip_runtime_api.h>

#include <map>
#include <string>
#include <vector>

#include "jt.h"
#include "jt_plan.h"

// Pinned host staging for the per-propagation uploads (evidence tables,
// collect sources, work lists): two buffers used in turn, each reused only
// after the copies out of it have completed (its event), so a later upload
// never rewrites bytes a queued copy still reads.
struct Staging {
    char *host[2] = {nullptr, nullptr};
    hipEvent_t done[2] = {nullptr, nullptr};
    bool pending[2] = {false, false};
    size_t cap = 0, used = 0;
    int k = 0;
};

struct jt_tree_s {
    jt::Plan plan;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool propagated = false;
    JtDev dev;
    std::vector<std::vector<int32_t>> ev_vars, ev_states;   // per slot region (the last: evidence-free)
    std::vector<char> ev_dirty;
    uint64_t ev_version = 1;            // bumped by every evidence change
    std::vector<int32_t> ev_idx_host;   // [n_regions][ev_idx_stride]
    std::vector<JtEv> ev_ent_host;      // [n_regions][ev_ent_stride]
    Staging stage;
    // dynamic schedule of the fused propagation (batched trees), and what it
    // was built for
    jt::Dynamic dyn;
    uint64_t dyn_version = 0;
    int dyn_n_active = -1;
    int64_t last_bytes = 0;
    int last_shared = 0;
    int64_t last_collect_pairs = 0;
    std::vector<int64_t> last_launch_bytes;   // per live fused launch (fused and graph modes)
    // host copies the scratch entry point uploads from (kept until its next call)
    std::vector<int32_t> sx_ev_idx;
    std::vector<JtEv> sx_ev_ent;
    jt::Dynamic sx_dyn;
    // captured graphs of the level launches, keyed by the number of active
    // slots followed by the grids of the listed launches
    std::map<std::vector<int32_t>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
    // lane streams of the fused schedule (default priority, created at bind)
    std::vector<hipStream_t> lane_stream;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t fork_ev = nullptr;
    // batched trees: a level's multi-slot launch runs on `side`, beside the
    // level's one-slot launch on the bound stream (fork and join by events)
    hipStream_t side = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    int last_mode = -1;
    int last_n_active = 0;
    // Bayesian-network trees: the compiled network (cliques, families)
    bool is_bn = false;
    jt::BnTree bn;
    // merged trees: the caller's cliques are families of the compiled ones
    bool is_merged = false;
    jt::MergedTree merged;
    // paper-faithful schedule: its plan, its workspace (mapping lists,
    // message and block records), layout and threads per block
    jt::PaperPlan paper;
    bool paper_planned = false;
    char *paper_ws = nullptr;
    int32_t paper_layout = 0, paper_tpb = 0;
};

namespace jt_detail {

jt_status set_err(jt_status code, const std::string &msg);
jt_status hip_err(hipError_t e, const char *what);
jt_status check_tree(jt_tree t);
// Device views of a workspace laid out by the plan.
void fill_dev(const jt::Plan &P, char *base, JtDev &d);
// Enqueue the plan's read-only metadata, the initial tables and zeroed
// arrival counters into a workspace.
hipError_t upload_static(const jt::Plan &P, char *base, const float *init_potentials, hipStream_t s);
// Enqueue launch list L for slots [0, S) on `stream` with device views d.
// `grids`: blocks of each listed launch (the dynamic schedule's), required
// when L has listed launches.
jt_status enqueue(jt_tree t, const JtDev &d, const std::vector<jt::Launch> &L, int S, bool fused, hipStream_t stream,
                  const std::vector<int32_t> *grids);

}  // namespace jt_detail
