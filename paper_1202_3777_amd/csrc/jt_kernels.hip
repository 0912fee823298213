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

#include <algorithm>

#include "jt_internal.h"

namespace {

// Wait until this wave's memory operations are acknowledged (vmcnt(0);
// expcnt and lgkmcnt left open).  Partials are written with agent-coherent
// stores, so once acknowledged any block of the chip reads them with
// agent-coherent loads -- no L2 write-back or invalidate is needed.
__device__ __forceinline__ void wait_vm_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct GatherReg {
    int32_t jout_off;  // Jout table of the gather's view (meta offsets stay below 2^30)
    int32_t off;       // LDS float offset, or float offset in the slot's separator region
    int32_t in_lds;
};

// Per-tile context of the tiles a wave has in flight.
template <int VEC>
struct TileBatch {
    int o[JT_UNROLL];
    float x[JT_UNROLL][4];
};

// Strides of the per-slot regions (values only, passed by value).
struct PassStrides {
    int64_t coll, out, sep, partial, scale, ev_idx, ev_ent;
};

template <int VEC>
__device__ __forceinline__ void pass_body(const JtItem &it, const JtTask &task, int slot,
                                          const JtGather *__restrict__ gathers, const int32_t *__restrict__ meta,
                                          const int32_t *__restrict__ ev_idx, const JtEv *__restrict__ ev_ent,
                                          const float *__restrict__ init, float *__restrict__ coll,
                                          float *__restrict__ out, const float *__restrict__ sep,
                                          const float *__restrict__ scale_arr, float *__restrict__ partial,
                                          const PassStrides &st, const float *__restrict__ lds_ratio,
                                          float *__restrict__ lds_red) {
    const int lane = threadIdx.x & (JT_WAVE - 1);
    // wave-uniform by construction; saying so lets the compiler keep the
    // group / tile bookkeeping and the metadata loads on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / JT_WAVE);
    const int T = it.T;

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
    const float *__restrict__ sep_slot = sep + (int64_t)slot * st.sep;
#pragma unroll
    for (int g = 0; g < JT_NG_REG; ++g) {
        gr[g].jout_off = 0;
        gr[g].in_lds = 0;
        gr[g].off = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) jin[g][q] = 0;
        if (g < ngr) {
            const JtGather G = gathers[it.gather_base + g];
            gr[g].jout_off = G.jout_off;
            gr[g].in_lds = G.lds_off >= 0;
            gr[g].off = G.lds_off >= 0 ? G.lds_off : G.sep_off;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (valid[q]) jin[g][q] = meta[G.jin_off + pos[q]];
        }
    }

    // evidence: inner digits give a per-lane mask, outer digits zero whole tiles
    bool keep[4] = {true, true, true, true};
    int ev0 = 0, ev1 = 0;
    const JtEv *__restrict__ evs = ev_ent + (int64_t)slot * st.ev_ent;
    if (it.ev) {
        const int32_t *ei = ev_idx + (int64_t)slot * st.ev_idx;
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

    // written by a finalize earlier in the same dataflow launch: a coherent
    // (vector) load, never the scalar cache
    const float scale = it.scale_clique >= 0 ? __hip_atomic_load(scale_arr + (int64_t)slot * st.scale + it.scale_clique,
                                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                             : 1.0f;
    const float *src =
        (it.src_kind == JT_SRC_INIT ? init
                                    : (it.src_kind == JT_SRC_COLL ? coll + (int64_t)slot * st.coll
                                                                  : out + (int64_t)slot * st.out)) +
        it.src_off;
    float *dst = nullptr;
    if (it.dst_kind == JT_DST_COLL) dst = coll + (int64_t)slot * st.coll + it.dst_off;
    if (it.dst_kind == JT_DST_OUT) dst = out + (int64_t)slot * st.out + it.dst_off;

    const bool has_out = it.out_view >= 0;
    const int32_t rout_off = it.o_rout_tile;
    float *part = partial + (int64_t)slot * st.partial + it.partial_off;

    // Tile metadata of up to 64 tiles is fetched lane-parallel once per chunk
    // (tile offset, each gather's Jout, the outer-evidence verdict) and read
    // back per tile with readlane, so the streaming loads never wait on a
    // dependent scalar lookup.
    // issue the loads of chunk tiles [u0, min(u0 + U, nt))
    auto issue = [&](TileBatch<VEC> &B, int u0, int nt, int my_o, uint64_t zmask) {
#pragma unroll
        for (int u = 0; u < JT_UNROLL; ++u) {
            const int uu = u0 + u;
            B.o[u] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) B.x[u][q] = 0.f;
            if (uu < nt) {
                const int o = __builtin_amdgcn_readlane(my_o, uu);
                B.o[u] = o;
                if (!((zmask >> uu) & 1ull)) {
                    const float *base = src + (int64_t)o * T;
                    if (VEC == 4) {
                        if (valid[0]) {
                            const float4 v4 = *reinterpret_cast<const float4 *>(base + pos[0]);
                            B.x[u][0] = v4.x;
                            B.x[u][1] = v4.y;
                            B.x[u][2] = v4.z;
                            B.x[u][3] = v4.w;
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (valid[q]) B.x[u][q] = base[pos[q]];
                    }
                }
            }
        }
    };
    // multiply in the gathers, mask, scale, store, accumulate
    auto consume = [&](const TileBatch<VEC> &B, int u0, int nt, const int (&my_jo)[JT_NG_REG], float (&acc)[4]) {
#pragma unroll
        for (int u = 0; u < JT_UNROLL; ++u) {
            const int uu = u0 + u;
            if (uu >= nt) break;
            const int o = B.o[u];
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = B.x[u][q];
#pragma unroll
            for (int gg = 0; gg < JT_NG_REG; ++gg) {
                if (gg < ngr) {
                    const int jo = __builtin_amdgcn_readlane(my_jo[gg], uu);
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
                const JtGather G = gathers[it.gather_base + gg];
                const int jo = meta[G.jout_off + o];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = jo + (valid[q] ? meta[G.jin_off + pos[q]] : 0);
                    v[q] *= G.lds_off >= 0 ? lds_ratio[G.lds_off + j] : sep_slot[G.sep_off + j];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = keep[q] ? v[q] * scale : 0.f;
            if (dst) {
                float *b = dst + (int64_t)o * T;
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
    };

    TileBatch<VEC> A, B;
    for (int g = task.g0 + wave; g < task.g1; g += JT_WAVES_PER_BLOCK) {
        int k = 0, sp = 0, q0, q1, tile_k = 0;
        if (has_out) {
            k = g / it.nsplit;
            sp = g - k * it.nsplit;
            q0 = sp * it.tpg;
            q1 = min(q0 + it.tpg, it.o_n_rout);
            tile_k = meta[it.o_kout_tile + k];
        } else {
            q0 = g * it.tpg;
            q1 = min(q0 + it.tpg, it.n_tiles);
        }
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int cb = q0; cb < q1; cb += JT_WAVE) {
            const int nt = min(JT_WAVE, q1 - cb);
            const bool live = lane < nt;
            int my_o = 0;
            if (live) my_o = has_out ? tile_k + meta[rout_off + cb + lane] : cb + lane;
            bool my_zero = false;
            for (int e = ev0; e < ev1; ++e) {
                const JtEv E = evs[e];
                if (E.outer && ((my_o / E.stride) % E.card) != E.digit) my_zero = true;
            }
            const uint64_t zmask = __ballot(live && my_zero);
            int my_jo[JT_NG_REG];
#pragma unroll
            for (int gg = 0; gg < JT_NG_REG; ++gg) my_jo[gg] = (gg < ngr && live) ? meta[gr[gg].jout_off + my_o] : 0;
            // two batches of tiles in flight: load one while the other is consumed
            issue(A, 0, nt, my_o, zmask);
            for (int uq = 0; uq < nt; uq += 2 * JT_UNROLL) {
                if (uq + JT_UNROLL < nt) issue(B, uq + JT_UNROLL, nt, my_o, zmask);
                consume(A, uq, nt, my_jo, acc);
                if (uq + 2 * JT_UNROLL < nt) issue(A, uq + 2 * JT_UNROLL, nt, my_o, zmask);
                if (uq + JT_UNROLL < nt) consume(B, uq + JT_UNROLL, nt, my_jo, acc);
            }
        }
        if (!has_out) continue;

        // fold the in-tile positions of each class, in a fixed order
        wave_sync();
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (valid[q]) lds_red[pos[q]] = acc[q];
        wave_sync();
        const int n_cls = it.o_n_cls, m_in = it.o_m_in;
        const int jk = meta[it.o_kout_j + k];
        float *pout = part + (int64_t)sp * it.o_ssize + jk;
        const int32_t *perm = meta + it.o_perm;
        const int32_t *clsj = meta + it.o_clsj;
        if (n_cls >= JT_WAVE) {
            for (int cls = lane; cls < n_cls; cls += JT_WAVE) {
                float s = 0.f;
                for (int n = 0; n < m_in; ++n) s += lds_red[perm[cls * m_in + n]];
                __hip_atomic_store(pout + clsj[cls], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            int P = JT_WAVE / n_cls;
            P = 1 << (31 - __clz(P));            // largest power of two <= 64 / n_cls
            const int cls = lane / P, part_i = lane - cls * P;
            float s = 0.f;
            if (cls < n_cls)
                for (int n = part_i; n < m_in; n += P) s += lds_red[perm[cls * m_in + n]];
            for (int off = P >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
            if (cls < n_cls && part_i == 0) __hip_atomic_store(pout + clsj[cls], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace

// Finalize: each block sums the split partials of jc separator entries
// (JT_BLOCK / jc split rows per column, fixed order), writes them, and adds a
// block sum to the message's scratch.  The block that arrives last forms
// sigma from the block sums in block order, updates the log-scales, and
// rescales the whole separator table (and forms new/old, 0/0 := 0).
// Returns true in the block that completed the message.
namespace {

struct FinPtrs {
    const JtMsg *__restrict__ msgs;
    const int32_t *__restrict__ child_edges;
    const float *__restrict__ partial;
    float *__restrict__ sep;
    double *__restrict__ lam;
    float *__restrict__ scale;
    int32_t *__restrict__ flag;
    double *__restrict__ fsig;
    int32_t *__restrict__ fcnt;
    int64_t partial_stride, sep_stride, lam_stride, scale_stride, fsig_stride, fcnt_stride;
    int32_t n_cliques;
};

// Given sigma (the sum of the new separator table), update the FP64
// log-scales and turn the raw table into the collect table (rescaled to mean
// one) or the distribute ratio new/old with 0/0 := 0.  All threads call it;
// thread tid owns entries tid, tid + JT_BLOCK, ...
__device__ void finish_message(const FinPtrs &F, const JtMsg &m, int slot, double sigma, float *sh_f) {
    const int tid = threadIdx.x;
    const int nc = F.n_cliques;
    float *sep = F.sep + (int64_t)slot * F.sep_stride;
    double *lam = F.lam + (int64_t)slot * F.lam_stride;
    float *scl = F.scale + (int64_t)slot * F.scale_stride;
    const int ssize = m.ssize;
    float *raw = nullptr;
    if (m.kind == JT_MSG_COLLECT) raw = sep + m.sepc_off;
    if (m.kind == JT_MSG_DIST || m.kind == JT_MSG_PLAIN) raw = sep + m.sepd_off;
    if (tid == 0) {
        const double ns = (double)ssize;
        double f = 0.0;
        switch (m.kind) {
            case JT_MSG_COLLECT: {
                double lc = 0.0;
                for (int a = 0; a < m.n_children; ++a) lc += lam[JT_LAM_SC(nc) + F.child_edges[m.child_base + a]];
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
                for (int a = 0; a < m.n_children; ++a) lc += lam[JT_LAM_SC(nc) + F.child_edges[m.child_base + a]];
                lam[JT_LAM_COLL(nc) + m.from] = lc;
                if (sigma > 0.0) {
                    lam[JT_LAM_LOGZ(nc)] = lc + log(sigma);
                    scl[m.from] = (float)(1.0 / sigma);
                    F.flag[slot] = 0;
                } else {
                    lam[JT_LAM_LOGZ(nc)] = -INFINITY;
                    scl[m.from] = 0.f;
                    F.flag[slot] = 1;
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
                    F.flag[slot] = sigma > 0.0 ? 0 : 1;
                }
                break;
            }
        }
        *sh_f = (float)f;
    }
    __syncthreads();
    const float f = *sh_f;
    if (m.kind == JT_MSG_COLLECT) {
        for (int jx = tid; jx < ssize; jx += JT_BLOCK) raw[jx] = raw[jx] * f;
    } else if (m.kind == JT_MSG_DIST) {
        const float *oldc = sep + m.sepc_off;
        for (int jx = tid; jx < ssize; jx += JT_BLOCK) {
            const float nw = raw[jx] * f;
            const float od = oldc[jx];
            raw[jx] = (od == 0.f) ? 0.f : nw / od;
        }
    } else if (m.kind == JT_MSG_PLAIN) {
        float *oldc = sep + m.sepc_off;
        for (int jx = tid; jx < ssize; jx += JT_BLOCK) {
            const float nw = raw[jx] * f;
            const float od = oldc[jx];
            raw[jx] = (od == 0.f) ? 0.f : nw / od;
            oldc[jx] = nw;
        }
    }
}

// The whole finalize of one message in one block: sum the split partials of
// every separator entry in a fixed order, sigma in a fixed order, then finish.
// Entry j is summed by thread j % JT_BLOCK (all splits), or, for separators
// of fewer than 64 entries, by JT_BLOCK / 64 threads over interleaved splits
// and a fixed LDS tree.  red: JT_BLOCK floats, dred: JT_BLOCK doubles.
__device__ __forceinline__ float ldp(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void finalize_whole(const FinPtrs &F, int mi, int slot, float *red, double *dred, float *sh_f) {
    const int tid = threadIdx.x;
    const JtMsg m = F.msgs[mi];
    const float *P = F.partial + (int64_t)slot * F.partial_stride + m.partial_off;
    float *sep = F.sep + (int64_t)slot * F.sep_stride;
    float *raw = nullptr;
    if (m.kind == JT_MSG_COLLECT) raw = sep + m.sepc_off;
    if (m.kind == JT_MSG_DIST || m.kind == JT_MSG_PLAIN) raw = sep + m.sepd_off;
    const int ssize = m.ssize, nsplit = m.nsplit;
    double local = 0.0;
    if (ssize >= 64) {
        for (int j = tid; j < ssize; j += JT_BLOCK) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
            int p = 0;
            for (; p + 3 < nsplit; p += 4) {
                a0 += ldp(P + (int64_t)p * ssize + j);
                a1 += ldp(P + (int64_t)(p + 1) * ssize + j);
                a2 += ldp(P + (int64_t)(p + 2) * ssize + j);
                a3 += ldp(P + (int64_t)(p + 3) * ssize + j);
            }
            for (; p < nsplit; ++p) a0 += ldp(P + (int64_t)p * ssize + j);
            const float v = (a0 + a1) + (a2 + a3);
            if (raw) raw[j] = v;
            local += (double)v;
        }
    } else {
        int sp2 = 1;
        while (sp2 < ssize) sp2 <<= 1;
        const int R = JT_BLOCK / sp2;
        const int jj = tid & (sp2 - 1), r = tid / sp2;
        float s = 0.f;
        if (jj < ssize) {
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
            int p = r;
            for (; p + 3 * R < nsplit; p += 4 * R) {
                a0 += ldp(P + (int64_t)p * ssize + jj);
                a1 += ldp(P + (int64_t)(p + R) * ssize + jj);
                a2 += ldp(P + (int64_t)(p + 2 * R) * ssize + jj);
                a3 += ldp(P + (int64_t)(p + 3 * R) * ssize + jj);
            }
            for (; p < nsplit; p += R) a0 += ldp(P + (int64_t)p * ssize + jj);
            s = (a0 + a1) + (a2 + a3);
        }
        red[tid] = s;
        __syncthreads();
        for (int h = R >> 1; h > 0; h >>= 1) {
            if (r < h) red[tid] += red[tid + h * sp2];
            __syncthreads();
        }
        if (r == 0 && jj < ssize) {
            const float v = red[jj];
            if (raw) raw[jj] = v;      // thread jj: the same thread rescales it
            local = (double)v;
        }
    }
    dred[tid] = local;
    __syncthreads();
    for (int h = JT_BLOCK >> 1; h > 0; h >>= 1) {
        if (tid < h) dred[tid] += dred[tid + h];
        __syncthreads();
    }
    const double sigma = dred[0];
    __syncthreads();
    finish_message(F, m, slot, sigma, sh_f);
}

__device__ bool finalize_block(const FinPtrs &F, const JtFTask &ft, int slot, float *red, double *dred, float *sh_f,
                               int *sh_last) {
    const int tid = threadIdx.x;
    const JtMsg m = F.msgs[ft.msg];
    const int nc = F.n_cliques;
    const float *P = F.partial + (int64_t)slot * F.partial_stride + m.partial_off;
    float *sep = F.sep + (int64_t)slot * F.sep_stride;
    double *lam = F.lam + (int64_t)slot * F.lam_stride;
    float *scl = F.scale + (int64_t)slot * F.scale_stride;
    double *fsig = F.fsig + (int64_t)slot * F.fsig_stride;
    int32_t *fcnt = F.fcnt + (int64_t)slot * F.fcnt_stride;
    const int ssize = m.ssize, nsplit = m.nsplit;
    float *raw = nullptr;
    if (m.kind == JT_MSG_COLLECT) raw = sep + m.sepc_off;
    if (m.kind == JT_MSG_DIST || m.kind == JT_MSG_PLAIN) raw = sep + m.sepd_off;

    const int jc = ft.jc, R = JT_BLOCK / jc;
    const int jj = tid & (jc - 1), r = tid / jc;
    const int j = ft.j0 + jj;
    float s = 0.f;
    if (j < ft.j1) {
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
        int p = r;
        for (; p + 3 * R < nsplit; p += 4 * R) {
            a0 += P[(int64_t)p * ssize + j];
            a1 += P[(int64_t)(p + R) * ssize + j];
            a2 += P[(int64_t)(p + 2 * R) * ssize + j];
            a3 += P[(int64_t)(p + 3 * R) * ssize + j];
        }
        for (; p < nsplit; p += R) a0 += P[(int64_t)p * ssize + j];
        s = (a0 + a1) + (a2 + a3);
    }
    red[tid] = s;
    __syncthreads();
    for (int h = R >> 1; h > 0; h >>= 1) {
        if (r < h) red[tid] += red[tid + h * jc];
        __syncthreads();
    }
    double v = 0.0;
    if (r == 0 && j < ft.j1) {
        const float x = red[jj];
        if (raw) raw[j] = x;
        v = (double)x;
    }
    dred[tid] = v;
    __syncthreads();
    for (int h = JT_BLOCK >> 1; h > 0; h >>= 1) {
        if (tid < h) dred[tid] += dred[tid + h];
        __syncthreads();
    }
    if (ft.nb > 1) {
        if (tid == 0) fsig[m.fbase + ft.b] = dred[0];
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            *sh_last = (atomicAdd(&fcnt[ft.msg], 1) == ft.nb - 1);
            __threadfence();
        }
        __syncthreads();
        if (!*sh_last) return false;
        __threadfence();
    }
    double sigma = dred[0];
    if (ft.nb > 1) {
        sigma = 0.0;
        for (int b = 0; b < ft.nb; ++b) sigma += fsig[m.fbase + b];
        __syncthreads();
        if (tid == 0) fcnt[ft.msg] = 0;    // ready for the next propagation
    }
    finish_message(F, m, slot, sigma, sh_f);
    return true;
}

__device__ __forceinline__ FinPtrs fin_ptrs(const JtDev &d) {
    FinPtrs F;
    F.msgs = d.msgs;
    F.child_edges = d.child_edges;
    F.partial = d.partial;
    F.sep = d.sep;
    F.lam = d.lam;
    F.scale = d.scale;
    F.flag = d.flag;
    F.fsig = d.fsig;
    F.fcnt = d.fcnt;
    F.partial_stride = d.partial_stride;
    F.sep_stride = d.sep_stride;
    F.lam_stride = d.lam_stride;
    F.scale_stride = d.scale_stride;
    F.fsig_stride = d.fsig_stride;
    F.fcnt_stride = d.fcnt_stride;
    F.n_cliques = d.n_cliques;
    return F;
}

}  // namespace

// One launch = the passes of one tree level (or one message) for every slot.
// Buffers are separate __restrict__ parameters so the compiler can prove the
// metadata is never written by the kernel and read it through the scalar
// unit (uniform loads that do not wait on the streaming vector loads).
//
// A pass that sums into a separator also finalizes that message: every block
// of the item counts its arrival after its partials are written, and the
// block that arrives last sums all split partials (fixed order), forms
// sigma, the log-scales and the new table or ratio.  No block ever waits for
// another, and the next level's launch sees finished messages.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_pass_kernel(
    const JtTask *__restrict__ tasks, const JtItem *__restrict__ items, const JtGather *__restrict__ gathers,
    const int32_t *__restrict__ meta, const int32_t *__restrict__ ev_idx, const JtEv *__restrict__ ev_ent,
    const float *__restrict__ init, float *__restrict__ coll, float *__restrict__ out, float *__restrict__ sep,
    float *__restrict__ scale, float *__restrict__ partial, const JtMsg *__restrict__ msgs,
    const int32_t *__restrict__ child_edges, double *__restrict__ lam, int32_t *__restrict__ flag,
    int32_t *__restrict__ icnt, PassStrides st, int64_t lam_stride, int64_t icnt_stride, int n_cliques,
    int task_begin, int n_tasks) {
    __shared__ __align__(16) float lds_ratio[JT_LDS_RATIO_FLOATS];   // also the finalize's double scratch
    __shared__ float lds_red[JT_WAVES_PER_BLOCK][JT_TILE_MAX];
    __shared__ float sh_f;
    __shared__ int sh_last;
    const int slot = blockIdx.x / n_tasks;
    const JtTask task = tasks[task_begin + (blockIdx.x - slot * n_tasks)];
    const JtItem it = items[task.item];
    // stage the ratio tables this pass multiplies in
    const float *sep_slot = sep + (int64_t)slot * st.sep;
    for (int g = 0; g < it.n_gather_lds; ++g) {
        const JtGather G = gathers[it.gather_base + g];
        for (int j = threadIdx.x; j < G.ssize; j += JT_BLOCK) lds_ratio[G.lds_off + j] = sep_slot[G.sep_off + j];
    }
    __syncthreads();
    float *red = lds_red[threadIdx.x / JT_WAVE];
    if (it.vec == 4)
        pass_body<4>(it, task, slot, gathers, meta, ev_idx, ev_ent, init, coll, out, sep, scale, partial, st, lds_ratio,
                     red);
    else
        pass_body<1>(it, task, slot, gathers, meta, ev_idx, ev_ent, init, coll, out, sep, scale, partial, st, lds_ratio,
                     red);
    if (it.msg < 0) return;
    int32_t *cnt = icnt + (int64_t)slot * icnt_stride + task.item;
    wait_vm_stores();   // this wave's partials are acknowledged
    __syncthreads();
    if (threadIdx.x == 0) sh_last = (atomicAdd(cnt, 1) == it.n_tasks - 1);
    __syncthreads();
    if (!sh_last) return;
    FinPtrs F;
    F.msgs = msgs;
    F.child_edges = child_edges;
    F.partial = partial;
    F.sep = sep;
    F.lam = lam;
    F.scale = scale;
    F.flag = flag;
    F.fsig = nullptr;
    F.fcnt = nullptr;
    F.partial_stride = st.partial;
    F.sep_stride = st.sep;
    F.lam_stride = lam_stride;
    F.scale_stride = st.scale;
    F.fsig_stride = 0;
    F.fcnt_stride = 0;
    F.n_cliques = n_cliques;
    finalize_whole(F, it.msg, slot, lds_red[0], reinterpret_cast<double *>(lds_ratio), &sh_f);
    if (threadIdx.x == 0) *cnt = 0;    // ready for the next propagation
}

extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_finalize_kernel(JtDev d, int ftask_begin, int n_ftasks) {
    __shared__ float red[JT_BLOCK];
    __shared__ double dred[JT_BLOCK];
    __shared__ float sh_f;
    __shared__ int sh_last;
    const int slot = blockIdx.x / n_ftasks;
    const JtFTask ft = d.ftasks[ftask_begin + (blockIdx.x - slot * n_ftasks)];
    finalize_block(fin_ptrs(d), ft, slot, red, dred, &sh_f, &sh_last);
}

// Dataflow schedule: one persistent launch for the whole propagation.  Blocks
// take units (a pass task or a finalize task, for one slot) from a global
// counter in topological order and wait only for what that unit reads: a
// pass task for the finalize of the messages whose tables it multiplies in
// (and whose scale it applies), a finalize task for every task of the pass
// that produced its partials.  A unit only ever waits for units taken
// before it, so the smallest unfinished unit can always run and every block
// reaches the end.  A wait that exceeds its bound sets df_err and gives up,
// so the launch still ends.
#define JT_SPIN_LIMIT (1 << 20)

__device__ __forceinline__ bool wait_at_least(int32_t *p, int32_t want) {
    for (int it = 0; it < JT_SPIN_LIMIT; ++it) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= want) return true;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_dataflow_kernel(
    const JtUnit *__restrict__ units, const int32_t *__restrict__ deps, const JtTask *__restrict__ tasks,
    const JtItem *__restrict__ items, const JtGather *__restrict__ gathers, const int32_t *__restrict__ meta,
    const int32_t *__restrict__ ev_idx, const JtEv *__restrict__ ev_ent, const float *__restrict__ init,
    float *__restrict__ coll, float *__restrict__ out, float *__restrict__ sep, float *__restrict__ scale,
    float *__restrict__ partial, const JtFTask *__restrict__ ftasks, const JtMsg *__restrict__ msgs,
    const int32_t *__restrict__ child_edges, double *__restrict__ lam, int32_t *__restrict__ flag,
    double *__restrict__ fsig, int32_t *__restrict__ fcnt, int32_t *__restrict__ df, int32_t *__restrict__ df_err,
    PassStrides st, int64_t lam_stride, int64_t fsig_stride, int64_t fcnt_stride, int64_t df_stride, int n_cliques,
    int n_items, int n_units, int n_slots) {
    __shared__ float lds_ratio[JT_LDS_RATIO_FLOATS];
    __shared__ float lds_red[JT_WAVES_PER_BLOCK][JT_TILE_MAX];
    __shared__ double dred[JT_BLOCK];
    __shared__ float sh_f;
    __shared__ int sh_last, sh_unit, sh_ok;
    FinPtrs F;
    F.msgs = msgs;
    F.child_edges = child_edges;
    F.partial = partial;
    F.sep = sep;
    F.lam = lam;
    F.scale = scale;
    F.flag = flag;
    F.fsig = fsig;
    F.fcnt = fcnt;
    F.partial_stride = st.partial;
    F.sep_stride = st.sep;
    F.lam_stride = lam_stride;
    F.scale_stride = st.scale;
    F.fsig_stride = fsig_stride;
    F.fcnt_stride = fcnt_stride;
    F.n_cliques = n_cliques;
    const int tid = threadIdx.x;
    const int total = n_units * n_slots;
    for (;;) {
        if (tid == 0) sh_unit = atomicAdd(&df[0], 1);
        __syncthreads();
        const int g = sh_unit;
        __syncthreads();
        if (g >= total) break;
        const int u = g / n_slots, slot = g - u * n_slots;
        const JtUnit U = units[u];
        int32_t *done = df + JT_WAVE + (int64_t)slot * df_stride;   // [0, n_items) items, then messages
        if (U.kind == 0) {
            const JtTask task = tasks[U.index];
            const JtItem it = items[task.item];
            if (tid == 0) {
                bool ok = true;
                for (int a = 0; a < it.n_dep && ok; ++a) ok = wait_at_least(done + n_items + deps[it.dep_base + a], 1);
                if (!ok) atomicExch(df_err, 1);
                sh_ok = ok;
                __threadfence();   // acquire: what the producers released is visible
            }
            __syncthreads();
            __threadfence();
            if (sh_ok) {
                const float *sep_slot = sep + (int64_t)slot * st.sep;
                for (int gg = 0; gg < it.n_gather_lds; ++gg) {
                    const JtGather G = gathers[it.gather_base + gg];
                    for (int j = tid; j < G.ssize; j += JT_BLOCK) lds_ratio[G.lds_off + j] = sep_slot[G.sep_off + j];
                }
                __syncthreads();
                float *red = lds_red[tid / JT_WAVE];
                if (it.vec == 4)
                    pass_body<4>(it, task, slot, gathers, meta, ev_idx, ev_ent, init, coll, out, sep, scale, partial,
                                 st, lds_ratio, red);
                else
                    pass_body<1>(it, task, slot, gathers, meta, ev_idx, ev_ent, init, coll, out, sep, scale, partial,
                                 st, lds_ratio, red);
            }
            __threadfence();   // release this block's table and partial writes
            __syncthreads();
            if (tid == 0) {
                __threadfence();
                atomicAdd(done + task.item, 1);
            }
        } else {
            const JtFTask ft = ftasks[U.index];
            const JtMsg m = msgs[ft.msg];
            if (tid == 0) {
                const bool ok = wait_at_least(done + m.item, items[m.item].n_tasks);
                if (!ok) atomicExch(df_err, 1);
                sh_ok = ok;
                __threadfence();
            }
            __syncthreads();
            __threadfence();
            bool last = false;
            if (sh_ok) last = finalize_block(F, ft, slot, lds_red[0], dred, &sh_f, &sh_last);
            if (!sh_ok) last = (ft.b == 0);   // a failed wait still releases the dependents
            __threadfence();
            __syncthreads();
            if (last && tid == 0) {
                __threadfence();
                atomicExch(done + n_items + ft.msg, 1);
            }
        }
    }
}

// Clears the dataflow counters before the persistent launch (a kernel, so
// the propagation can be captured in a graph without memset nodes).
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_dataflow_reset_kernel(int32_t *df, int64_t n, int32_t *fcnt,
                                                                                int64_t n_fcnt) {
    for (int64_t i = blockIdx.x * (int64_t)JT_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * JT_BLOCK) df[i] = 0;
    for (int64_t i = blockIdx.x * (int64_t)JT_BLOCK + threadIdx.x; i < n_fcnt; i += (int64_t)gridDim.x * JT_BLOCK)
        fcnt[i] = 0;
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
    PassStrides st;
    st.coll = d.coll_stride;
    st.out = d.out_stride;
    st.sep = d.sep_stride;
    st.partial = d.partial_stride;
    st.scale = d.scale_stride;
    st.ev_idx = d.ev_idx_stride;
    st.ev_ent = d.ev_ent_stride;
    hipLaunchKernelGGL(jt_pass_kernel, dim3((unsigned)n_tasks * (unsigned)n_slots), dim3(JT_BLOCK), 0, s, d.tasks,
                       d.items, d.gathers, d.meta, d.ev_idx, d.ev_ent, d.init, d.coll, d.out, d.sep, d.scale,
                       d.partial, d.msgs, d.child_edges, d.lam, d.flag, d.icnt, st, d.lam_stride, d.icnt_stride,
                       d.n_cliques, task_begin, n_tasks);
    return hipGetLastError();
}

hipError_t jt_launch_finalize(const JtDev &d, int ftask_begin, int n_ftasks, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(jt_finalize_kernel, dim3((unsigned)n_ftasks * (unsigned)n_slots), dim3(JT_BLOCK), 0, s, d,
                       ftask_begin, n_ftasks);
    return hipGetLastError();
}

hipError_t jt_launch_dataflow(const JtDev &d, int n_slots, int grid, hipStream_t s) {
    const int64_t n_df = JT_WAVE + (int64_t)n_slots * d.df_stride;
    hipLaunchKernelGGL(jt_dataflow_reset_kernel, dim3((unsigned)std::min<int64_t>(1024, (n_df + JT_BLOCK - 1) / JT_BLOCK)),
                       dim3(JT_BLOCK), 0, s, d.df, n_df, d.fcnt, (int64_t)n_slots * d.fcnt_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PassStrides st;
    st.coll = d.coll_stride;
    st.out = d.out_stride;
    st.sep = d.sep_stride;
    st.partial = d.partial_stride;
    st.scale = d.scale_stride;
    st.ev_idx = d.ev_idx_stride;
    st.ev_ent = d.ev_ent_stride;
    hipLaunchKernelGGL(jt_dataflow_kernel, dim3((unsigned)grid), dim3(JT_BLOCK), 0, s, d.units, d.deps, d.tasks,
                       d.items, d.gathers, d.meta, d.ev_idx, d.ev_ent, d.init, d.coll, d.out, d.sep, d.scale,
                       d.partial, d.ftasks, d.msgs, d.child_edges, d.lam, d.flag, d.fsig, d.fcnt, d.df, d.df + 1, st,
                       d.lam_stride, d.fsig_stride, d.fcnt_stride, d.df_stride, d.n_cliques, d.n_items, d.n_units,
                       n_slots);
    return hipGetLastError();
}

int jt_dataflow_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(jt_dataflow_kernel), JT_BLOCK,
                                                     0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

hipError_t jt_launch_plain_init(const JtDev &d, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(jt_plain_init_kernel, dim3((unsigned)n_slots), dim3(JT_BLOCK), 0, s, d);
    return hipGetLastError();
}
