// jt_kernels.hip -- gfx950 kernels of the junction-tree message engine.
//
// A message i -> k (eq. (1)-(3)) is split into streaming "passes" over clique
// tables and a small per-message "finalize":
//
//   pass      v(r) = src[r] * [evidence] * prod_g ratio_g[j_g(r)] * scale
//             optionally dst[r] = v(r) (the scatter-multiply of eq. (3), fused
//             with everything absorbed so far) and/or a segmented sum of v
//             into the entries of one separator (the marginalization of
//             eq. (2)).
//   finalize  sum the pass's split partials into the new separator table,
//             rescale it to mean one, form new/old with 0/0 := 0 (the rule
//             stated after eq. (3)), update the FP64 log-scales.
//
// The separator index of an entry is j(r) = Jin[r % T] + Jout[r / T]
// (factored cluster-separator mapping, Sec. 3.2).  A wave owns whole tiles
// of T <= 256 entries; each lane holds the same 4 in-tile positions for
// every tile, so its Jin values sit in registers and Jout is one scalar load
// per tile.  The segmented reduction is atomics-free and has a fixed order:
// a wave sums its tiles position by position in registers, then folds the
// positions of one class (the separator configurations inside a tile) in
// LDS and with lane shuffles, and writes one partial per (split, separator
// entry); the finalize adds the splits in order.  Every result is therefore
// bit-identical from run to run.
#include <hip/hip_runtime.h>
#include <math.h>

#include "jt_internal.h"

namespace {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct GatherReg {
    int64_t jout_off;
    int32_t off;      // LDS float offset, or float offset in the slot's separator region
    int32_t in_lds;
};

template <int VEC>
__device__ __forceinline__ void pass_body(const JtDev &d, const JtItem &it, const JtTask &task, int slot,
                                          const float *__restrict__ lds_ratio, float *__restrict__ lds_red) {
    const int lane = threadIdx.x & (JT_WAVE - 1);
    const int wave = threadIdx.x / JT_WAVE;
    const int T = it.T;
    const int32_t *__restrict__ meta = d.meta;

    int pos[4];
    bool valid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        pos[q] = (VEC == 4) ? 4 * lane + q : lane + JT_WAVE * q;
        valid[q] = pos[q] < T;
    }

    // gathers: per-lane Jin in registers, Jout offset and table location
    const int ng = it.n_gather;
    const int ngr = ng < JT_NG_REG ? ng : JT_NG_REG;
    GatherReg gr[JT_NG_REG];
    int jin[JT_NG_REG][4];
    const float *__restrict__ sep_slot = d.sep + (int64_t)slot * d.sep_stride;
#pragma unroll
    for (int g = 0; g < JT_NG_REG; ++g) {
        if (g < ngr) {
            const JtGather G = d.gathers[it.gather_base + g];
            const JtView V = d.views[G.view];
            gr[g].jout_off = V.jout_off;
            gr[g].in_lds = G.lds_off >= 0;
            gr[g].off = G.lds_off >= 0 ? G.lds_off : G.sep_off;
#pragma unroll
            for (int q = 0; q < 4; ++q) jin[g][q] = valid[q] ? meta[V.jin_off + pos[q]] : 0;
        } else {
            gr[g].jout_off = 0;
            gr[g].in_lds = 0;
            gr[g].off = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) jin[g][q] = 0;
        }
    }

    // evidence: inner digits give a per-lane mask, outer digits zero whole tiles
    bool keep[4] = {true, true, true, true};
    int ev0 = 0, ev1 = 0;
    const JtEv *__restrict__ evs = d.ev_ent + (int64_t)slot * d.ev_ent_stride;
    if (it.ev) {
        const int32_t *ei = d.ev_idx + (int64_t)slot * d.ev_idx_stride;
        ev0 = ei[it.clique];
        ev1 = ei[it.clique + 1];
        for (int e = ev0; e < ev1; ++e) {
            const JtEv E = evs[e];
            if (!E.outer) {
#pragma unroll
                for (int q = 0; q < 4; ++q) keep[q] = keep[q] && ((pos[q] / E.stride) % E.card) == E.digit;
            }
        }
    }

    const float scale = it.scale_clique >= 0 ? d.scale[(int64_t)slot * d.scale_stride + it.scale_clique] : 1.0f;
    const float *__restrict__ src =
        (it.src_kind == JT_SRC_INIT ? d.init
                                    : (it.src_kind == JT_SRC_COLL ? d.coll + (int64_t)slot * d.coll_stride
                                                                  : d.out + (int64_t)slot * d.out_stride)) +
        it.src_off;
    float *__restrict__ dst = nullptr;
    if (it.dst_kind == JT_DST_COLL) dst = d.coll + (int64_t)slot * d.coll_stride + it.dst_off;
    if (it.dst_kind == JT_DST_OUT) dst = d.out + (int64_t)slot * d.out_stride + it.dst_off;

    const bool has_out = it.out_view >= 0;
    JtView OV;
    if (has_out) OV = d.views[it.out_view];
    float *__restrict__ part = d.partial + (int64_t)slot * d.partial_stride + it.partial_off;

    for (int g = task.g0 + wave; g < task.g1; g += JT_WAVES_PER_BLOCK) {
        int k = 0, sp = 0, q0, q1, tile_k = 0;
        if (has_out) {
            k = g / it.nsplit;
            sp = g - k * it.nsplit;
            q0 = sp * it.tpg;
            q1 = min(q0 + it.tpg, OV.n_rout);
            tile_k = meta[OV.kout_tile_off + k];
        } else {
            q0 = g * it.tpg;
            q1 = min(q0 + it.tpg, it.n_tiles);
        }
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int qq = q0; qq < q1; qq += JT_UNROLL) {
            int o[JT_UNROLL];
            float x[JT_UNROLL][4];
#pragma unroll
            for (int u = 0; u < JT_UNROLL; ++u) {
                const int t = qq + u;
                o[u] = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) x[u][q] = 0.f;
                if (t < q1) {
                    o[u] = has_out ? tile_k + meta[OV.rout_tile_off + t] : t;
                    bool zero = false;
                    for (int e = ev0; e < ev1; ++e) {
                        const JtEv E = evs[e];
                        if (E.outer && ((o[u] / E.stride) % E.card) != E.digit) zero = true;
                    }
                    if (!zero) {
                        const float *base = src + (int64_t)o[u] * T;
                        if (VEC == 4) {
                            if (valid[0]) {
                                const float4 v4 = *reinterpret_cast<const float4 *>(base + pos[0]);
                                x[u][0] = v4.x;
                                x[u][1] = v4.y;
                                x[u][2] = v4.z;
                                x[u][3] = v4.w;
                            }
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                if (valid[q]) x[u][q] = base[pos[q]];
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < JT_UNROLL; ++u) {
                if (qq + u >= q1) break;
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = x[u][q];
#pragma unroll
                for (int gg = 0; gg < JT_NG_REG; ++gg) {
                    if (gg < ngr) {
                        const int jo = meta[gr[gg].jout_off + o[u]];
                        if (gr[gg].in_lds) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) v[q] *= lds_ratio[gr[gg].off + jo + jin[gg][q]];
                        } else {
#pragma unroll
                            for (int q = 0; q < 4; ++q) v[q] *= sep_slot[gr[gg].off + jo + jin[gg][q]];
                        }
                    }
                }
                for (int gg = JT_NG_REG; gg < ng; ++gg) {
                    const JtGather G = d.gathers[it.gather_base + gg];
                    const JtView V = d.views[G.view];
                    const int jo = meta[V.jout_off + o[u]];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int j = jo + (valid[q] ? meta[V.jin_off + pos[q]] : 0);
                        v[q] *= G.lds_off >= 0 ? lds_ratio[G.lds_off + j] : sep_slot[G.sep_off + j];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = keep[q] ? v[q] * scale : 0.f;
                if (dst) {
                    float *b = dst + (int64_t)o[u] * T;
                    if (VEC == 4) {
                        if (valid[0]) *reinterpret_cast<float4 *>(b + pos[0]) = make_float4(v[0], v[1], v[2], v[3]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (valid[q]) b[pos[q]] = v[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] += v[q];
            }
        }
        if (!has_out) continue;

        // fold the in-tile positions of each class, in a fixed order
        wave_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (valid[q]) lds_red[pos[q]] = acc[q];
        wave_sync();
        const int n_cls = OV.n_cls, m_in = OV.m_in;
        const int jk = meta[OV.kout_j_off + k];
        float *pout = part + (int64_t)sp * OV.ssize + jk;
        const int32_t *perm = meta + OV.perm_off;
        const int32_t *clsj = meta + OV.clsj_off;
        if (n_cls >= JT_WAVE) {
            for (int cls = lane; cls < n_cls; cls += JT_WAVE) {
                float s = 0.f;
                for (int n = 0; n < m_in; ++n) s += lds_red[perm[cls * m_in + n]];
                pout[clsj[cls]] = s;
            }
        } else {
            int P = JT_WAVE / n_cls;
            P = 1 << (31 - __clz(P));            // largest power of two <= 64 / n_cls
            const int cls = lane / P, part_i = lane - cls * P;
            float s = 0.f;
            if (cls < n_cls)
                for (int n = part_i; n < m_in; n += P) s += lds_red[perm[cls * m_in + n]];
            for (int off = P >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (cls < n_cls && part_i == 0) pout[clsj[cls]] = s;
        }
    }
}

}  // namespace

// One launch = the passes of one tree level (or one message) for every slot.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_pass_kernel(JtDev d, int task_begin, int n_tasks) {
    __shared__ float lds_ratio[JT_LDS_RATIO_FLOATS];
    __shared__ float lds_red[JT_WAVES_PER_BLOCK][JT_TILE_MAX];
    const int slot = blockIdx.x / n_tasks;
    const JtTask task = d.tasks[task_begin + (blockIdx.x - slot * n_tasks)];
    const JtItem it = d.items[task.item];
    // stage the ratio tables this pass multiplies in
    const float *sep_slot = d.sep + (int64_t)slot * d.sep_stride;
    for (int g = 0; g < it.n_gather_lds; ++g) {
        const JtGather G = d.gathers[it.gather_base + g];
        for (int j = threadIdx.x; j < G.ssize; j += JT_BLOCK) lds_ratio[G.lds_off + j] = sep_slot[G.sep_off + j];
    }
    __syncthreads();
    float *red = lds_red[threadIdx.x / JT_WAVE];
    if (it.vec == 4)
        pass_body<4>(d, it, task, slot, lds_ratio, red);
    else
        pass_body<1>(d, it, task, slot, lds_ratio, red);
}

// One block per (message, slot).
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_finalize_kernel(JtDev d, int msg_begin, int n_msgs) {
    __shared__ float red[JT_BLOCK];
    __shared__ double dred[JT_BLOCK];
    __shared__ float sh_f;
    const int tid = threadIdx.x;
    const int slot = blockIdx.x / n_msgs;
    const JtMsg m = d.msgs[msg_begin + (blockIdx.x - slot * n_msgs)];
    const int nc = d.n_cliques;
    const float *P = d.partial + (int64_t)slot * d.partial_stride + m.partial_off;
    float *sep = d.sep + (int64_t)slot * d.sep_stride;
    double *lam = d.lam + (int64_t)slot * d.lam_stride;
    float *scl = d.scale + (int64_t)slot * d.scale_stride;
    const int ssize = m.ssize, nsplit = m.nsplit;
    float *raw = nullptr;
    if (m.kind == JT_MSG_COLLECT) raw = sep + m.sepc_off;
    if (m.kind == JT_MSG_DIST || m.kind == JT_MSG_PLAIN) raw = sep + m.sepd_off;

    // sum the split partials: column j, rows split over R thread groups
    int sp2 = 1;
    while (sp2 < ssize && sp2 < JT_BLOCK) sp2 <<= 1;
    const int R = JT_BLOCK / sp2;
    const int jj = tid % sp2, r = tid / sp2;
    double local = 0.0;
    for (int j0 = 0; j0 < ssize; j0 += sp2) {
        const int j = j0 + jj;
        float s = 0.f;
        if (j < ssize)
            for (int p = r; p < nsplit; p += R) s += P[(int64_t)p * ssize + j];
        red[tid] = s;
        __syncthreads();
        for (int h = R >> 1; h > 0; h >>= 1) {
            if (r < h) red[tid] += red[tid + h * sp2];
            __syncthreads();
        }
        if (r == 0 && j < ssize) {
            const float v = red[jj];
            if (raw) raw[j] = v;
            local += (double)v;
        }
        __syncthreads();
    }
    dred[tid] = local;
    __syncthreads();
    for (int h = JT_BLOCK >> 1; h > 0; h >>= 1) {
        if (tid < h) dred[tid] += dred[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        const double sigma = dred[0];
        const double ns = (double)ssize;
        double f = 0.0;
        switch (m.kind) {
            case JT_MSG_COLLECT: {
                double lc = 0.0;
                for (int a = 0; a < m.n_children; ++a) lc += lam[JT_LAM_SC(nc) + d.child_edges[m.child_base + a]];
                lam[JT_LAM_COLL(nc) + m.from] = lc;
                if (sigma > 0.0) {
                    f = ns / sigma;
                    lam[JT_LAM_SC(nc) + m.edge] = lc + log(sigma / ns);
                } else {
                    lam[JT_LAM_SC(nc) + m.edge] = 0.0;
                }
                break;
            }
            case JT_MSG_TOTAL: {
                double lc = 0.0;
                for (int a = 0; a < m.n_children; ++a) lc += lam[JT_LAM_SC(nc) + d.child_edges[m.child_base + a]];
                lam[JT_LAM_COLL(nc) + m.from] = lc;
                if (sigma > 0.0) {
                    lam[JT_LAM_LOGZ(nc)] = lc + log(sigma);
                    scl[m.from] = (float)(1.0 / sigma);
                    d.flag[slot] = 0;
                } else {
                    lam[JT_LAM_LOGZ(nc)] = -INFINITY;
                    scl[m.from] = 0.f;
                    d.flag[slot] = 1;
                }
                break;
            }
            case JT_MSG_DIST: {
                const double logz = lam[JT_LAM_LOGZ(nc)];
                double lsd = 0.0;
                if (sigma > 0.0) {
                    f = ns / sigma;
                    lsd = logz + log(sigma / ns);
                }
                lam[JT_LAM_SD(nc) + m.edge] = lsd;
                const double lcal = lam[JT_LAM_COLL(nc) + m.to] + lsd - lam[JT_LAM_SC(nc) + m.edge];
                scl[m.to] = (float)exp(lcal - logz);
                break;
            }
            case JT_MSG_PLAIN: {
                const double lold = lam[JT_LAM_SC(nc) + m.edge];
                double lnew = lold;
                if (sigma > 0.0) {
                    f = ns / sigma;
                    lnew = lam[JT_LAM_COLL(nc) + m.from] + log(sigma / ns);
                }
                lam[JT_LAM_COLL(nc) + m.to] += lnew - lold;
                lam[JT_LAM_SC(nc) + m.edge] = lnew;
                break;
            }
            case JT_MSG_PLAIN_TOTAL: {
                scl[m.from] = sigma > 0.0 ? (float)(1.0 / sigma) : 0.f;
                if (m.to == -2) {
                    lam[JT_LAM_LOGZ(nc)] = sigma > 0.0 ? lam[JT_LAM_COLL(nc) + m.from] + log(sigma) : -INFINITY;
                    d.flag[slot] = sigma > 0.0 ? 0 : 1;
                }
                break;
            }
        }
        sh_f = (float)f;
    }
    __syncthreads();
    const float f = sh_f;
    if (m.kind == JT_MSG_COLLECT) {
        for (int j = tid; j < ssize; j += JT_BLOCK) raw[j] = raw[j] * f;
    } else if (m.kind == JT_MSG_DIST) {
        const float *oldc = sep + m.sepc_off;
        for (int j = tid; j < ssize; j += JT_BLOCK) {
            const float nw = raw[j] * f;
            const float od = oldc[j];
            raw[j] = (od == 0.f) ? 0.f : nw / od;
        }
    } else if (m.kind == JT_MSG_PLAIN) {
        float *oldc = sep + m.sepc_off;
        for (int j = tid; j < ssize; j += JT_BLOCK) {
            const float nw = raw[j] * f;
            const float od = oldc[j];
            raw[j] = (od == 0.f) ? 0.f : nw / od;
            oldc[j] = nw;
        }
    }
}

// One-at-a-time schedule set-up: every separator table := 1, log-scales := 0.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_plain_init_kernel(JtDev d) {
    const int slot = blockIdx.x;
    float *sep = d.sep + (int64_t)slot * d.sep_stride;
    for (int64_t i = threadIdx.x; i < d.sep_stride; i += JT_BLOCK) sep[i] = 1.f;
    double *lam = d.lam + (int64_t)slot * d.lam_stride;
    for (int64_t i = threadIdx.x; i < d.lam_stride; i += JT_BLOCK) lam[i] = 0.0;
}

// ---------------------------------------------------------------------------
// host-side launchers (the C ABI lives in jt_api.cpp)

hipError_t jt_launch_pass(const JtDev &d, int task_begin, int n_tasks, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(jt_pass_kernel, dim3((unsigned)n_tasks * (unsigned)n_slots), dim3(JT_BLOCK), 0, s, d,
                       task_begin, n_tasks);
    return hipGetLastError();
}

hipError_t jt_launch_finalize(const JtDev &d, int msg_begin, int n_msgs, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(jt_finalize_kernel, dim3((unsigned)n_msgs * (unsigned)n_slots), dim3(JT_BLOCK), 0, s, d,
                       msg_begin, n_msgs);
    return hipGetLastError();
}

hipError_t jt_launch_plain_init(const JtDev &d, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(jt_plain_init_kernel, dim3((unsigned)n_slots), dim3(JT_BLOCK), 0, s, d);
    return hipGetLastError();
}
