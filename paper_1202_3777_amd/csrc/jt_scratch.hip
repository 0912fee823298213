// jt_scratch.hip -- the allocation-free entry point jt_propagate_scratch:
// one propagation of a compiled tree in a static device array owned by the
// library, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>
#include <math.h>

#include <mutex>
#include <string>

#include "jt.h"
#include "jt_api_internal.h"
#include "jt_internal.h"
#include "jt_plan.h"

#define JT_SCRATCH_BYTES (128ull << 20)   // per GPU
#define JT_MAX_DEVICES 64

using namespace jt_detail;

hipError_t jt_launch_read_out(const JtDev &d, int slot0, int n_slots, int64_t packed_total, float *dst,
                              double *log_z, hipStream_t s);

// The library-owned scratch.  Each GPU the library runs on holds one copy
// until the process ends.  Host code never uses the array's name as an
// address: scratch_region looks up its device address once per device, with
// that device current, and every use goes through that pointer.
static __device__ __align__(256) unsigned char scratch[JT_SCRATCH_BYTES];

namespace {

hipError_t scratch_region(void **ptr, size_t *bytes) {
    static std::mutex mu;
    static void *addr[JT_MAX_DEVICES] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= JT_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    *bytes = JT_SCRATCH_BYTES;
    return hipSuccess;
}

}  // namespace

extern "C" {

jt_status jt_propagate_scratch(jt_tree t, const float *init_potentials, float *posteriors, double *log_z,
                               int32_t mode, void *hip_stream) {
    if (jt_status rc = check_tree(t)) return rc;
    if (!init_potentials || !posteriors || !log_z) return set_err(JT_E_ARG, "NULL input or output pointer");
    if (mode != JT_MODE_FUSED && mode != JT_MODE_PLAIN) return set_err(JT_E_ARG, "mode must be fused or plain");
    const jt::Plan &P = t->plan;
    if (P.n_lanes > 0) return set_err(JT_E_ARG, "lanes are not available with the static scratch");
    void *base = nullptr;
    size_t cap = 0;
    hipError_t e = scratch_region(&base, &cap);
    if (e != hipSuccess) return hip_err(e, "static scratch address");
    if (P.total_bytes > cap)
        return set_err(JT_E_NO_MEM, "tree needs " + std::to_string(P.total_bytes) + " bytes of device memory; the static "
                                    "scratch holds " + std::to_string(cap));
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    char *ws = static_cast<char *>(base);
    JtDev d;
    fill_dev(P, ws, d);
    e = upload_static(P, ws, init_potentials, s);
    if (e != hipSuccess) return hip_err(e, "scratch upload");
    const bool fused = mode == JT_MODE_FUSED;
    try {
        // every region's evidence (the evidence-free one last), and for a
        // batched tree the dynamic schedule, from host copies kept in the
        // handle until its next call
        t->sx_ev_idx.assign((size_t)P.n_regions * P.ev_idx_stride, 0);
        t->sx_ev_ent.assign((size_t)P.n_regions * P.ev_ent_stride, JtEv{0, 1, 1, 0});
        for (int32_t r = 0; r < P.n_regions; ++r)
            jt::evidence_tables(P, t->ev_vars[r], t->ev_states[r], &t->sx_ev_idx[(size_t)r * P.ev_idx_stride],
                                &t->sx_ev_ent[(size_t)r * P.ev_ent_stride]);
        if (P.share && fused) jt::build_dynamic(P, t->ev_vars, P.n_slots, t->sx_dyn);
    } catch (const std::bad_alloc &) {
        return set_err(JT_E_NO_MEM, "host allocation failed");
    } catch (const std::exception &x) {
        return set_err(JT_E_ARG, std::string("schedule: ") + x.what());
    }
    auto up = [&](size_t off, const void *src, size_t n) -> hipError_t {
        if (n == 0) return hipSuccess;
        return hipMemcpyAsync(ws + off, src, n, hipMemcpyHostToDevice, s);
    };
    e = up(P.off_ev_idx, t->sx_ev_idx.data(), t->sx_ev_idx.size() * sizeof(int32_t));
    if (e == hipSuccess) e = up(P.off_ev_ent, t->sx_ev_ent.data(), t->sx_ev_ent.size() * sizeof(JtEv));
    if (e == hipSuccess && P.share && fused) {
        e = up(P.off_csrc, t->sx_dyn.csrc.data(), t->sx_dyn.csrc.size() * sizeof(int32_t));
        if (e == hipSuccess) e = up(P.off_work_count, t->sx_dyn.count.data(), t->sx_dyn.count.size() * sizeof(int32_t));
        if (e == hipSuccess) e = up(P.off_work, t->sx_dyn.work.data(), t->sx_dyn.work.size() * sizeof(JtWork));
        if (e == hipSuccess && P.chunk_total > 0)
            e = up(P.off_chunks, t->sx_dyn.chunks.data(), t->sx_dyn.chunks.size() * sizeof(JtChunk));
    }
    if (e != hipSuccess) return hip_err(e, "scratch evidence upload");
    if (jt_status rc = enqueue(t, d, fused ? P.fused : P.plain, P.n_slots, fused, s, &t->sx_dyn.grid)) return rc;
    e = jt_launch_read_out(d, 0, P.n_slots, (int64_t)P.total_entries, posteriors, log_z, s);
    if (e != hipSuccess) return hip_err(e, "read-out launch");
    return JT_OK;
}

}  // extern "C"
