// jt_kernels.hip -- gfx950 kernels of the junction-tree message engine.
//
// A message i -> k (eq. (1)-(3)) is computed by one streaming "pass" over a
// clique table whose last block also "finalizes" the message:
//
//   pass      v(r) = src[r] * [evidence] * prod_g ratio_g[j_g(r)] * scale
//             optionally dst[r] = v(r) (the scatter-multiply of eq. (3), fused
//             with everything absorbed so far) and/or a segmented sum of v
//             into the entries of one separator (the marginalization of
//             eq. (2)).
//   finalize  sum the pass's partial rows into the new separator table,
//             rescale it to mean one, form new/old with 0/0 := 0 (the rule
//             stated after eq. (3)), update the FP64 log-scales.
//
// The separator index of an entry is j(r) = Jin[r % T] + Jout[r / T]
// (factored cluster-separator mapping, Sec. 3.2).  A block streams one
// "group" of tiles (T <= 256 entries each) at a time, its four waves taking
// a quarter each; each lane holds the same 4 in-tile positions for every
// tile, so its Jin values sit in registers, and the tile offsets and Jout
// values of up to 64 tiles are fetched lane-parallel and read back with
// readlane (tiles of at most 128 entries go two to a wave, one per
// half-wave).  The segmented reduction is atomics-free and has a fixed order:
// a wave sums its tiles position by position in registers, the block adds
// its four waves position by position in LDS, folds the positions of each
// class (the separator configurations inside a tile) and writes one partial
// row per group; the finalize adds the rows in order.  Every result is
// therefore bit-identical from run to run.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "jt_internal.h"

namespace {
typedef float jt_f4 __attribute__((ext_vector_type(4)));

// Wait until this wave's memory operations are acknowledged (vmcnt(0);
// expcnt and lgkmcnt left open).  Partials are written with agent-coherent
// stores, so once acknowledged any block of the chip reads them with
// agent-coherent loads -- no L2 write-back or invalidate is needed.
__device__ __forceinline__ void wait_vm_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Staging copies into LDS with global->LDS loads: the data does not pass
// through registers, so every load of a staging step is in flight at once and
// the block waits once (vmcnt(0), then the barrier) instead of once per round
// of 256 entries.  One instruction moves 64 lanes' data to consecutive LDS
// addresses from the (wave-uniform) destination.
//  lds_copy_f4: n floats, 16 B per lane (256 per instruction); the source is
//    16-byte aligned and readable up to n rounded up to a multiple of 4, and so
//    is the LDS slot (the last lane may copy up to three floats of padding).
//  lds_copy_i1: n int32, 4 B per lane (64 per instruction), exact.
// Instruction c goes to wave (c + rot) mod 4, so small tables staged together
// are spread over the waves.
__device__ __forceinline__ void lds_copy_f4(const float *src, float *dst, int n, int wave, int lane, int rot) {
    for (int c = (wave - rot) & (JT_WAVES_PER_BLOCK - 1); c * 256 < n; c += JT_WAVES_PER_BLOCK)
        if (c * 256 + 4 * lane < n) __builtin_amdgcn_global_load_lds(src + c * 256 + 4 * lane, dst + c * 256, 16, 0, 0);
}
__device__ __forceinline__ void lds_copy_i1(const int32_t *src, int32_t *dst, int n, int wave, int lane, int rot) {
    for (int c = (wave - rot) & (JT_WAVES_PER_BLOCK - 1); c * 64 < n; c += JT_WAVES_PER_BLOCK)
        if (c * 64 + lane < n) __builtin_amdgcn_global_load_lds(src + c * 64 + lane, dst + c * 64, 4, 0, 0);
}

// Agent-coherent load of a value written by another block of the same launch.
__device__ __forceinline__ float ldp(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void stp(float *p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over the 64 lanes in a fixed tree; the total is valid in lane 0.
__device__ __forceinline__ double wave_sum_lane0(double v) {
#pragma unroll
    for (int off = JT_WAVE / 2; off > 0; off >>= 1) v += __shfl_down(v, off);
    return v;
}

struct GatherReg {
    int32_t jout_off;  // Jout table of the gather's view (meta offsets stay below 2^30)
    int32_t off;       // LDS float offset, or float offset in the slot's separator region
    int32_t in_lds;
};

// Per-tile context of the tiles a wave has in flight.
struct TileBatch {
    int o[JT_UNROLL];
    float x[JT_UNROLL][4];
};

// The value that the lane owning this lane's tile of step uu holds in `v`:
// chunk tile uu, or with PAIR chunk tile 2 uu + h for half-wave h.
template <int PAIR>
__device__ __forceinline__ int step_val(int v, int uu, int hl) {
    if (!PAIR) return __builtin_amdgcn_readlane(v, uu);
    const int v0 = __builtin_amdgcn_readlane(v, 2 * uu), v1 = __builtin_amdgcn_readlane(v, 2 * uu + 1);
    return hl ? v1 : v0;
}

// Strides of the per-slot regions (values only, passed by value).
struct PassStrides {
    int64_t coll, out, sep, partial, scale, ev_idx, ev_ent;
};

// LDS of one pass block besides the staged ratio tables.
struct PassLds {
    float red[JT_WAVES_PER_BLOCK][JT_TILE_MAX];   // per-wave position sums
    float pos[JT_TILE_MAX];                       // block position sums
    int32_t perm[JT_TILE_MAX];                    // output view: positions grouped by class
    int32_t clsj[JT_TILE_MAX];                    // output view: separator offset of each class
    double wsum[JT_WAVES_PER_BLOCK];
    float f;
    int last;
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of the four waves' position sums at in-tile position t, in a fixed
// order (with PAIR each wave's two half-wave sums first).
template <int PAIR>
__device__ __forceinline__ float block_pos_sum(const PassLds &L, int t) {
    if (!PAIR) return (L.red[0][t] + L.red[1][t]) + (L.red[2][t] + L.red[3][t]);
    constexpr int H = JT_TILE_MAX / 2;
    return ((L.red[0][t] + L.red[0][H + t]) + (L.red[1][t] + L.red[1][H + t])) +
           ((L.red[2][t] + L.red[2][H + t]) + (L.red[3][t] + L.red[3][H + t]));
}

// One wave folds the T position sums in `row` into the classes of the output
// view (fixed order) and stores the partial row: pout[clsj[cls]].
__device__ __forceinline__ void fold_store(const float *row, const PassLds &L, int n_cls, int m_in, float *pout,
                                           int lane) {
    if (n_cls >= JT_WAVE) {
        for (int cls = lane; cls < n_cls; cls += JT_WAVE) {
            float s = 0.f;
            for (int n = 0; n < m_in; ++n) s += row[L.perm[cls * m_in + n]];
            stp(pout + L.clsj[cls], s);
        }
    } else {
        int P = JT_WAVE / n_cls;
        P = 1 << (31 - __clz(P));            // largest power of two <= 64 / n_cls
        const int cls = lane / P, part_i = lane - cls * P;
        float s = 0.f;
        if (cls < n_cls)
            for (int n = part_i; n < m_in; n += P) s += row[L.perm[cls * m_in + n]];
        for (int off = P >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (cls < n_cls && part_i == 0) stp(pout + L.clsj[cls], s);
    }
}

// Streaming (non-temporal) stores of table entries: a table is written once
// per pass, and stores that bypass L2 leave no dirty lines for the
// end-of-kernel write-back.
__device__ __forceinline__ void st_nt4(float *p, float a, float b, float c, float d) {
    const jt_f4 w = {a, b, c, d};
    __builtin_nontemporal_store(w, reinterpret_cast<jt_f4 *>(p));
}

// One block's share of a pass: groups [task.g0, task.g1) of item `it`.
// VEC: the lane layout of a tile (4 consecutive entries per lane as one
// float4 when T % 4 == 0, else entries lane + 64 q).  PAIR: tiles of at most
// 128 entries are taken two at a time, one per half-wave (lanes 32 h + l
// hold position 4 l + q, or l + 32 q, of the pair's tile h), so a load
// instruction moves a whole wave's width; the two halves keep separate
// position sums, added in a fixed order at the end of the group.
template <int VEC, int PAIR>
__device__ __forceinline__ void pass_block(const JtItem &it, const JtTask &task, int slot,
                                           const JtGather *__restrict__ gfirst,
                                           const JtGather *__restrict__ gathers, const int32_t *__restrict__ meta,
                                           const int32_t *__restrict__ ev_idx, const JtEv *__restrict__ ev_ent,
                                           const float *__restrict__ src, float *__restrict__ dst,
                                           const float *__restrict__ sep, const int32_t *__restrict__ cs_row,
                                           const float *__restrict__ scale_arr, float *__restrict__ partial,
                                           const PassStrides &st, float *__restrict__ lds_ratio, PassLds &L) {
    const int lane = threadIdx.x & (JT_WAVE - 1);
    // wave-uniform by construction; saying so lets the compiler keep the
    // group / tile bookkeeping and the metadata loads on the scalar unit
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / JT_WAVE);
    const int T = it.T;
    const int hl = PAIR ? lane >> 5 : 0;   // the half-wave's tile of a pair

    int pos[4];
    bool valid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int pl = PAIR ? lane & 31 : lane;
        pos[q] = (VEC == 4) ? 4 * pl + q : pl + (PAIR ? 32 : JT_WAVE) * q;
        valid[q] = pos[q] < T;
    }

    // gathers: per-lane Jin in registers, Jout offset and table location
    const int ng = it.n_gather;
    const int ngr = ng < JT_NG_REG ? ng : JT_NG_REG;
    GatherReg gr[JT_NG_REG];
    int32_t gglob[JT_NG_REG];   // float offset of each gathered table in `sep`
    int jin[JT_NG_REG][4];
    // float offset of a gathered table in `sep` (all slot regions of the
    // separator area stay below 2^31 floats): a collect message is read from
    // its sender's collect source, a distribute ratio from this slot
    auto gather_off = [&](const JtGather &G) -> int32_t {
        const int32_t gs = (cs_row && G.src_clique >= 0) ? cs_row[G.src_clique] : slot;
        return gs * (int32_t)st.sep + G.sep_off;
    };
#pragma unroll
    for (int g = 0; g < JT_NG_REG; ++g) {
        gr[g].jout_off = 0;
        gr[g].in_lds = 0;
        gr[g].off = 0;
        gglob[g] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) jin[g][q] = 0;
        if (g < ngr) {
            const JtGather G = gfirst[g];
            gr[g].jout_off = G.jout_off;
            gr[g].in_lds = G.lds_off >= 0;
            gglob[g] = gather_off(G);
            gr[g].off = G.lds_off >= 0 ? G.lds_off : gglob[g];
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

    // written by the finalize of an earlier launch
    const float scale = it.scale_clique >= 0 ? scale_arr[(int64_t)slot * st.scale + it.scale_clique] : 1.0f;

    const bool has_out = it.out_view >= 0;
    const int32_t rout_off = it.o_rout_tile;
    float *part = partial + (int64_t)slot * st.partial + it.partial_off;

    // issue the loads of steps [u0, min(u0 + U, nst)) of a chunk of nt tiles
    // (a step is one tile, or with PAIR two)
    auto issue = [&](TileBatch &B, int u0, int nst, int nt, int my_o) {
#pragma unroll
        for (int u = 0; u < JT_UNROLL; ++u) {
            const int uu = u0 + u;
            B.o[u] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) B.x[u][q] = 0.f;
            if (uu < nst) {
                // loaded even when evidence zeroes the tile (masked in
                // consume), so the load does not wait for the evidence test
                const int o = step_val<PAIR>(my_o, uu, hl);
                B.o[u] = o;
                const bool tv = !PAIR || 2 * uu + hl < nt;
                const float *base = src + (int64_t)o * T;
                if (VEC == 4) {
                    if (valid[0] && tv) {
                        const float4 v4 = *reinterpret_cast<const float4 *>(base + pos[0]);
                        B.x[u][0] = v4.x;
                        B.x[u][1] = v4.y;
                        B.x[u][2] = v4.z;
                        B.x[u][3] = v4.w;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (valid[q] && tv) B.x[u][q] = base[pos[q]];
                }
            }
        }
    };
    // entry u of batch B (step uu): multiply in the gathers, mask, scale,
    // store, accumulate
    auto consume_one = [&](const TileBatch &B, int u, int uu, int nt, uint64_t zmask,
                           const int (&my_jo)[JT_NG_REG], float (&acc)[4]) {
        {
            const int ti = PAIR ? 2 * uu + hl : uu;   // this lane's chunk tile
            const bool tv = !PAIR || ti < nt;
            const bool zt = (zmask >> ti) & 1ull;    // outer evidence zeroes the whole tile
            const int o = B.o[u];
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = B.x[u][q];
#pragma unroll
            for (int gg = 0; gg < JT_NG_REG; ++gg) {
                if (gg < ngr) {
                    const int jo = step_val<PAIR>(my_jo[gg], uu, hl);
                    if (gr[gg].in_lds) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] *= lds_ratio[gr[gg].off + jo + jin[gg][q]];
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] *= sep[gr[gg].off + jo + jin[gg][q]];
                    }
                }
            }
            for (int gg = JT_NG_REG; gg < ng; ++gg) {
                const JtGather G = gathers[it.gather_base + gg];
                const int jo = meta[G.jout_off + o];
                const int32_t go = gather_off(G);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = jo + (valid[q] ? meta[G.jin_off + pos[q]] : 0);
                    v[q] *= G.lds_off >= 0 ? lds_ratio[G.lds_off + j] : sep[go + j];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (keep[q] && !zt && tv) ? v[q] * scale : 0.f;
            if (dst && tv) {
                float *b = dst + (int64_t)o * T;
                if (VEC == 4) {
                    if (valid[0]) st_nt4(b + pos[0], v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (valid[q]) __builtin_nontemporal_store(v[q], b + pos[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] += v[q];
        }
    };
    auto consume = [&](const TileBatch &B, int u0, int nst, int nt, uint64_t zmask, const int (&my_jo)[JT_NG_REG],
                       float (&acc)[4]) {
#pragma unroll
        for (int u = 0; u < JT_UNROLL; ++u) {
            if (u0 + u >= nst) break;
            consume_one(B, u, u0 + u, nt, zmask, my_jo, acc);
        }
    };

    // LDS staging (ratio tables, the output view's class tables); every wave
    // calls it once, after its first chunk's tile loads are in flight.  The
    // ratio tables sit 16-byte aligned in the separator region (padded to 64
    // floats) and in LDS (slots rounded up to 4 floats).
    auto stage = [&]() {
        const int ngl = it.n_gather_lds;
#pragma unroll
        for (int g = 0; g < JT_NG_REG; ++g)
            if (g < ngl && g < ngr)
                lds_copy_f4(sep + gglob[g], lds_ratio + gfirst[g].lds_off, gfirst[g].ssize, wave, lane, g);
        for (int gg = JT_NG_REG; gg < ngl; ++gg) {
            const JtGather G = gathers[it.gather_base + gg];
            lds_copy_f4(sep + gather_off(G), lds_ratio + G.lds_off, G.ssize, wave, lane, gg);
        }
        if (has_out) {
            lds_copy_i1(meta + it.o_perm, L.perm, T, wave, lane, 0);
            lds_copy_i1(meta + it.o_clsj, L.clsj, it.o_n_cls, wave, lane, 2);
        }
        wait_vm_stores();   // this wave's loads into LDS have landed
        __syncthreads();
    };
    TileBatch A, B;

    if (!PAIR && it.wave_groups) {
        // Short groups (one kept-outer configuration with its n_rout tiles
        // each): a wave streams a contiguous run of whole groups back to back,
        // metadata of 64 tiles at a time across group boundaries, and folds
        // its position sums into the group's partial row whenever the group
        // changes -- without stalling the loads already in flight.
        const int ngrp = task.g1 - task.g0;
        const int per = (ngrp + JT_WAVES_PER_BLOCK - 1) / JT_WAVES_PER_BLOCK;
        const int gw0 = task.g0 + min(ngrp, wave * per), gw1 = task.g0 + min(ngrp, wave * per + per);
        const int nr = it.tpg;
        const int n_my = (gw1 - gw0) * nr;
        float *row = L.red[wave];
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        int cur_g = -1, cur_jk = 0;
        auto flush = [&]() {
            wave_sync();
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (valid[q]) row[pos[q]] = acc[q];
            wave_sync();
            fold_store(row, L, it.o_n_cls, it.o_m_in, part + cur_jk, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = 0.f;
        };
        auto consume_w = [&](const TileBatch &Bt, int u0, int nt, int my_g, int my_jk, uint64_t zmask,
                             const int (&my_jo)[JT_NG_REG]) {
#pragma unroll
            for (int u = 0; u < JT_UNROLL; ++u) {
                const int uu = u0 + u;
                if (uu >= nt) break;
                const int gt = __builtin_amdgcn_readlane(my_g, uu);
                if (gt != cur_g) {
                    if (cur_g >= 0) flush();
                    cur_g = gt;
                    cur_jk = __builtin_amdgcn_readlane(my_jk, uu);
                }
                consume_one(Bt, u, uu, nt, zmask, my_jo, acc);
            }
        };
        bool staged = false;
        int cb = 0;
        do {
            const int nt = max(0, min(JT_WAVE, n_my - cb));
            const bool live = lane < nt;
            int my_o = 0, my_g = 0, my_jk = 0;
            if (live) {
                const int t = cb + lane;
                const int gi = t / nr;
                my_g = gw0 + gi;
                my_o = meta[it.o_kout_tile + my_g] + meta[rout_off + (t - gi * nr)];
                my_jk = meta[it.o_kout_j + my_g];
            }
            bool my_zero = false;
            for (int e = ev0; e < ev1; ++e) {
                const JtEv E = evs[e];
                if (E.outer && ((my_o / E.stride) % E.card) != E.digit) my_zero = true;
            }
            const uint64_t zmask = __ballot(live && my_zero);
            int my_jo[JT_NG_REG];
#pragma unroll
            for (int gg = 0; gg < JT_NG_REG; ++gg) my_jo[gg] = (gg < ngr && live) ? meta[gr[gg].jout_off + my_o] : 0;
            issue(A, 0, nt, nt, my_o);
            if (!staged) {
                stage();
                staged = true;
            }
            for (int uq = 0; uq < nt; uq += 2 * JT_UNROLL) {
                if (uq + JT_UNROLL < nt) issue(B, uq + JT_UNROLL, nt, nt, my_o);
                consume_w(A, uq, nt, my_g, my_jk, zmask, my_jo);
                if (uq + 2 * JT_UNROLL < nt) issue(A, uq + 2 * JT_UNROLL, nt, nt, my_o);
                if (uq + JT_UNROLL < nt) consume_w(B, uq + JT_UNROLL, nt, my_g, my_jk, zmask, my_jo);
            }
            cb += JT_WAVE;
        } while (cb < n_my);
        if (cur_g >= 0) flush();
        return;
    }

    bool staged = false;
    for (int g = task.g0; g < task.g1; ++g) {
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
        // this wave's quarter of the group
        const int per = (q1 - q0 + JT_WAVES_PER_BLOCK - 1) / JT_WAVES_PER_BLOCK;
        const int a = min(q1, q0 + wave * per), b = min(q1, a + per);
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        int cb = a;
        do {   // every wave runs at least one chunk (possibly empty): the staging barrier
            const int nt = max(0, min(JT_WAVE, b - cb));
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
            const int nst = PAIR ? (nt + 1) >> 1 : nt;
            issue(A, 0, nst, nt, my_o);
            if (!staged) {
                stage();
                staged = true;
            }
            // two batches of tiles in flight: load one while the other is consumed
            for (int uq = 0; uq < nst; uq += 2 * JT_UNROLL) {
                if (uq + JT_UNROLL < nst) issue(B, uq + JT_UNROLL, nst, nt, my_o);
                consume(A, uq, nst, nt, zmask, my_jo, acc);
                if (uq + 2 * JT_UNROLL < nst) issue(A, uq + 2 * JT_UNROLL, nst, nt, my_o);
                if (uq + JT_UNROLL < nst) consume(B, uq + JT_UNROLL, nst, nt, zmask, my_jo, acc);
            }
            cb += JT_WAVE;
        } while (cb < b);
        if (!has_out) continue;

        // the block's position sums (waves in order), then the classes of
        // the output view folded in a fixed order into one partial row
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (valid[q]) L.red[wave][hl * (JT_TILE_MAX / 2) + pos[q]] = acc[q];
        __syncthreads();
        for (int t = threadIdx.x; t < T; t += JT_BLOCK) L.pos[t] = block_pos_sum<PAIR>(L, t);
        __syncthreads();
        if (wave == 0)
            fold_store(L.pos, L, it.o_n_cls, it.o_m_in, part + (int64_t)sp * it.o_ssize + meta[it.o_kout_j + k], lane);
    }
}

// Multi-slot distribute pass: up to JT_MS slots whose pass over this
// clique reads the same source table (the evidence-free absorbed table, or
// the initial table of a leaf without evidence in any of them).  Every tile
// is loaded once; for each slot k it is multiplied by that slot's parent ratio
// (staged in LDS at k * ldsz) and scale, stored as the slot's posterior and
// summed into the slot's partial rows -- in the same order, with the same
// groups and folds, as the single-slot pass, so each slot's bits equal those
// of its own pass (PAIR as in pass_block).
template <int VEC, int PAIR>
__device__ __forceinline__ void pass_multi(const JtItem &it, const JtTask &task, const int32_t *ms_slot, int ns,
                                           const JtGather &G, const int32_t *__restrict__ meta,
                                           const float *__restrict__ src, float *__restrict__ out,
                                           const float *__restrict__ sep, const float *__restrict__ scale_arr,
                                           float *__restrict__ partial, const PassStrides &st,
                                           float *__restrict__ lds_ratio, PassLds &L,
                                           float (*__restrict__ posk)[JT_TILE_MAX], const int64_t *ms_part,
                                           const int64_t *ms_dst, const float *ms_scl) {
    const int lane = threadIdx.x & (JT_WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / JT_WAVE);
    const int T = it.T;
    const int hl = PAIR ? lane >> 5 : 0;
    int pos[4];
    bool valid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int pl = PAIR ? lane & 31 : lane;
        pos[q] = (VEC == 4) ? 4 * pl + q : pl + (PAIR ? 32 : JT_WAVE) * q;
        valid[q] = pos[q] < T;
    }
    int jin[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) jin[q] = valid[q] ? meta[G.jin_off + pos[q]] : 0;
    // per slot (in LDS, read as broadcasts): scale ms_scl[k], posterior
    // offset ms_dst[k], partial-row offset ms_part[k]
    const int ldsz = (G.ssize + 3) & ~3;
    const bool has_dst = it.dst_kind == JT_DST_OUT;
    const bool has_out = it.out_view >= 0;
    const int32_t rout_off = it.o_rout_tile;

    auto issue = [&](TileBatch &B, int u0, int nst, int nt, int my_o) {
#pragma unroll
        for (int u = 0; u < JT_UNROLL; ++u) {
            const int uu = u0 + u;
            B.o[u] = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) B.x[u][q] = 0.f;
            if (uu < nst) {
                const int o = step_val<PAIR>(my_o, uu, hl);
                B.o[u] = o;
                const bool tv = !PAIR || 2 * uu + hl < nt;
                const float *base = src + (int64_t)o * T;
                if (VEC == 4) {
                    if (valid[0] && tv) {
                        const float4 v4 = *reinterpret_cast<const float4 *>(base + pos[0]);
                        B.x[u][0] = v4.x;
                        B.x[u][1] = v4.y;
                        B.x[u][2] = v4.z;
                        B.x[u][3] = v4.w;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (valid[q] && tv) B.x[u][q] = base[pos[q]];
                }
            }
        }
    };
    auto consume_one = [&](const TileBatch &B, int u, int uu, int nt, int my_jo, float (&acc)[JT_MS][4]) {
        const int o = B.o[u];
        const bool tv = !PAIR || 2 * uu + hl < nt;   // the lane's tile of the step exists
        const int jo = step_val<PAIR>(my_jo, uu, hl);
#pragma unroll
        for (int k = 0; k < JT_MS; ++k) {
            if (k >= ns) break;
            const float *__restrict__ rk = lds_ratio + k * ldsz + jo;
            const float sk = ms_scl[k];
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v[q] = B.x[u][q] * rk[jin[q]];
                v[q] = v[q] * sk;
            }
            if (has_dst && tv) {
                float *b = out + ms_dst[k] + (int64_t)o * T;
                if (VEC == 4) {
                    if (valid[0]) st_nt4(b + pos[0], v[0], v[1], v[2], v[3]);
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (valid[q]) __builtin_nontemporal_store(v[q], b + pos[q]);
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[k][q] += tv ? v[q] : 0.f;
        }
    };
    auto consume = [&](const TileBatch &B, int u0, int nst, int nt, int my_jo, float (&acc)[JT_MS][4]) {
#pragma unroll
        for (int u = 0; u < JT_UNROLL; ++u) {
            if (u0 + u >= nst) break;
            consume_one(B, u, u0 + u, nt, my_jo, acc);
        }
    };
    auto stage = [&]() {
        // every slot's ratio table (16-byte aligned in the separator region
        // and, at k * ldsz, in LDS), then the output view's class tables
#pragma unroll
        for (int k = 0; k < JT_MS; ++k)
            if (k < ns)
                lds_copy_f4(sep + (int64_t)ms_slot[k] * st.sep + G.sep_off, lds_ratio + k * ldsz, G.ssize, wave, lane, k);
        if (has_out) {
            lds_copy_i1(meta + it.o_perm, L.perm, T, wave, lane, 0);
            lds_copy_i1(meta + it.o_clsj, L.clsj, it.o_n_cls, wave, lane, 2);
        }
        wait_vm_stores();   // this wave's loads into LDS have landed
        __syncthreads();
    };
    TileBatch A, B;
    float acc[JT_MS][4];
#pragma unroll
    for (int k = 0; k < JT_MS; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[k][q] = 0.f;

    if (!PAIR && it.wave_groups) {
        const int ngrp = task.g1 - task.g0;
        const int per = (ngrp + JT_WAVES_PER_BLOCK - 1) / JT_WAVES_PER_BLOCK;
        const int gw0 = task.g0 + min(ngrp, wave * per), gw1 = task.g0 + min(ngrp, wave * per + per);
        const int nr = it.tpg;
        const int n_my = (gw1 - gw0) * nr;
        float *row = L.red[wave];
        int cur_g = -1, cur_jk = 0;
        auto flush = [&]() {
#pragma unroll
            for (int k = 0; k < JT_MS; ++k) {
                if (k >= ns) break;
                wave_sync();
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (valid[q]) row[pos[q]] = acc[k][q];
                wave_sync();
                fold_store(row, L, it.o_n_cls, it.o_m_in, partial + ms_part[k] + cur_jk, lane);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[k][q] = 0.f;
            }
        };
        auto consume_w = [&](const TileBatch &Bt, int u0, int nt, int my_g, int my_jk, int my_jo) {
#pragma unroll
            for (int u = 0; u < JT_UNROLL; ++u) {
                const int uu = u0 + u;
                if (uu >= nt) break;
                const int gt = __builtin_amdgcn_readlane(my_g, uu);
                if (gt != cur_g) {
                    if (cur_g >= 0) flush();
                    cur_g = gt;
                    cur_jk = __builtin_amdgcn_readlane(my_jk, uu);
                }
                consume_one(Bt, u, uu, nt, my_jo, acc);
            }
        };
        bool staged = false;
        int cb = 0;
        do {
            const int nt = max(0, min(JT_WAVE, n_my - cb));
            const bool live = lane < nt;
            int my_o = 0, my_g = 0, my_jk = 0;
            if (live) {
                const int t = cb + lane;
                const int gi = t / nr;
                my_g = gw0 + gi;
                my_o = meta[it.o_kout_tile + my_g] + meta[rout_off + (t - gi * nr)];
                my_jk = meta[it.o_kout_j + my_g];
            }
            const int my_jo = live ? meta[G.jout_off + my_o] : 0;
            issue(A, 0, nt, nt, my_o);
            if (!staged) {
                stage();
                staged = true;
            }
            for (int uq = 0; uq < nt; uq += 2 * JT_UNROLL) {
                if (uq + JT_UNROLL < nt) issue(B, uq + JT_UNROLL, nt, nt, my_o);
                consume_w(A, uq, nt, my_g, my_jk, my_jo);
                if (uq + 2 * JT_UNROLL < nt) issue(A, uq + 2 * JT_UNROLL, nt, nt, my_o);
                if (uq + JT_UNROLL < nt) consume_w(B, uq + JT_UNROLL, nt, my_g, my_jk, my_jo);
            }
            cb += JT_WAVE;
        } while (cb < n_my);
        if (cur_g >= 0) flush();
        return;
    }

    bool staged = false;
    for (int g = task.g0; g < task.g1; ++g) {
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
        const int per = (q1 - q0 + JT_WAVES_PER_BLOCK - 1) / JT_WAVES_PER_BLOCK;
        const int a = min(q1, q0 + wave * per), b = min(q1, a + per);
#pragma unroll
        for (int kk = 0; kk < JT_MS; ++kk)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[kk][q] = 0.f;
        int cb = a;
        do {
            const int nt = max(0, min(JT_WAVE, b - cb));
            const bool live = lane < nt;
            int my_o = 0;
            if (live) my_o = has_out ? tile_k + meta[rout_off + cb + lane] : cb + lane;
            const int my_jo = live ? meta[G.jout_off + my_o] : 0;
            const int nst = PAIR ? (nt + 1) >> 1 : nt;
            issue(A, 0, nst, nt, my_o);
            if (!staged) {
                stage();
                staged = true;
            }
            for (int uq = 0; uq < nst; uq += 2 * JT_UNROLL) {
                if (uq + JT_UNROLL < nst) issue(B, uq + JT_UNROLL, nst, nt, my_o);
                consume(A, uq, nst, nt, my_jo, acc);
                if (uq + 2 * JT_UNROLL < nst) issue(A, uq + 2 * JT_UNROLL, nst, nt, my_o);
                if (uq + JT_UNROLL < nst) consume(B, uq + JT_UNROLL, nst, nt, my_jo, acc);
            }
            cb += JT_WAVE;
        } while (cb < b);
        if (!has_out) continue;
        // per slot: the block's position sums (waves in order) into posk[k],
        // then every wave folds the classes of its share of the slots
#pragma unroll
        for (int kk = 0; kk < JT_MS; ++kk) {
            if (kk >= ns) break;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (valid[q]) L.red[wave][hl * (JT_TILE_MAX / 2) + pos[q]] = acc[kk][q];
            __syncthreads();
            for (int t = threadIdx.x; t < T; t += JT_BLOCK) posk[kk][t] = block_pos_sum<PAIR>(L, t);
            __syncthreads();
        }
        const int jk = meta[it.o_kout_j + k];
        for (int kk = wave; kk < ns; kk += JT_WAVES_PER_BLOCK)
            fold_store(posk[kk], L, it.o_n_cls, it.o_m_in, partial + ms_part[kk] + (int64_t)sp * it.o_ssize + jk, lane);
        __syncthreads();
    }
}

struct FinPtrs {
    const int32_t *__restrict__ child_edges;   // pairs (edge id, child clique)
    const int32_t *__restrict__ cs_row;        // this slot's collect sources, NULL: the slot itself
    const float *__restrict__ partial;
    float *__restrict__ sep;
    double *__restrict__ lam;
    float *__restrict__ scale;
    int32_t *__restrict__ flag;
    int64_t partial_stride, sep_stride, lam_stride, scale_stride;
    int32_t n_cliques;
};

// Keep the loads above this point from being moved below it and the uses
// below from being moved above (a volatile asm with a memory clobber bounds
// the scheduling region).  With the loads of a batch free of branches, they
// are all in flight before the first one is waited for.
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

// Column sums of the partial rows for columns j = jj + CT*(c0 + c), c < CB,
// rows s = r + R*i: four accumulators per column (i mod 4) combined as
// (a0 + a1) + (a2 + a3); RB rows per batch, so each batch issues CB*RB loads
// before any is used.  Writes the sums to raw and returns their FP64 total.
template <int CB, int RB>
__device__ __forceinline__ double column_sums(const float *P, float *stage, int ssize, int CT, int R, int jj, int r,
                                              int c0, int ncol, int nrow, float *first) {
    float a[CB][4];
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) a[c][q] = 0.f;
    for (int i0 = 0; i0 < nrow; i0 += RB) {
        // every load is issued (out-of-range ones read element 0 and are
        // dropped after the fence): no branch separates the loads, so none
        // of them waits for another
        float x[CB][RB];
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const bool ok = c0 + c < ncol && i0 + q < nrow;
                // 32-bit offset from the uniform base (partial regions stay below 2^31 floats)
                const uint32_t off = ok ? (uint32_t)((r + R * (i0 + q)) * ssize + jj + CT * (c0 + c)) : 0u;
                x[c][q] = ldp(P + off);
            }
        issue_fence();
#pragma unroll
        for (int c = 0; c < CB; ++c)
#pragma unroll
            for (int q = 0; q < RB; ++q)   // row i0 + q into accumulator (i0 + q) % 4 (RB is 1, 2 or a multiple of 4)
                a[c][q & 3] += (c0 + c < ncol && i0 + q < nrow) ? x[c][q] : 0.f;
    }
    double local = 0.0;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const float v = (a[c][0] + a[c][1]) + (a[c][2] + a[c][3]);
        if (c0 + c < ncol) {
            if (R == 1) {
                if (stage) stage[jj + CT * (c0 + c)] = v;
                local += (double)v;
            } else {
                *first = v;   // one column per thread when R > 1
            }
        }
    }
    return local;
}

// The finalize of one message, in the block of its pass that arrived last.
//  1. raw[j] = sum over the partial rows s of P[s][j], in a fixed order:
//     thread (jj, r) owns columns j = jj + CT*c and rows s = r + R*i (see
//     column_sums); with R > 1 row groups the columns are combined in a fixed
//     LDS tree;
//  2. sigma = sum_j raw[j] in FP64 (fixed wave trees, waves in order);
//  3. log-scales from sigma, then the separator table is rewritten as the
//     collect table (rescaled to mean one) or the distribute ratio new/old
//     with 0/0 := 0.
// The loads that do not depend on the partials (the log-scales the update
// reads) are issued first; steps 1 and 3 each issue their loads in batches
// before using them, so the finalize costs a few memory round trips.
// Log-scales a finalize combines (written by earlier launches).
struct FinScalars {
    double lc;           // sum of the children's collect log-scales (collect, total)
    double l0, l1, l2;   // distribute: log Z, collect scale of the target, collect scale of the edge;
                         // one-at-a-time: scale of the edge, collect scale of the source
};

// The slot whose collect data hold clique c's (the evidence-free slot when c
// has no evidence of this slot below it).
__device__ __forceinline__ int64_t coll_slot(const int32_t *__restrict__ cs_row, int c, int slot) {
    return cs_row ? (int64_t)cs_row[c] : (int64_t)slot;
}

__device__ __forceinline__ FinScalars load_fin_scalars(const FinPtrs &F, const JtMsg &m, int slot) {
    const int nc = F.n_cliques;
    const double *lam = F.lam + (int64_t)slot * F.lam_stride;
    FinScalars q{0.0, 0.0, 0.0, 0.0};
    if (m.kind == JT_MSG_COLLECT || m.kind == JT_MSG_TOTAL) {
        // children in order, two interleaved partial sums (even-numbered
        // children into s0, odd into s1); eight children per batch: their
        // edge ids and cliques, then their log-scales (from each child's
        // collect source), each batch of loads in flight together
        double s0 = 0.0, s1 = 0.0;
        for (int b = 0; b < m.n_children; b += 8) {
            int e[8], ch[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = m.child_base + (b + u < m.n_children ? b + u : b);
                e[u] = F.child_edges[2 * k];
                ch[u] = F.child_edges[2 * k + 1];
            }
            issue_fence();
            int64_t cs[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) cs[u] = coll_slot(F.cs_row, ch[u], slot);
            issue_fence();
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = F.lam[cs[u] * F.lam_stride + JT_LAM_SC(nc) + e[u]];
            issue_fence();
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (b + u >= m.n_children) break;
                if ((u & 1) == 0) s0 += v[u];
                else s1 += v[u];
            }
        }
        q.lc = s0 + s1;
    } else if (m.kind == JT_MSG_DIST) {
        // the target's collect scale and the collect message's scale belong
        // to the target's collect source
        const double *lt = F.lam + coll_slot(F.cs_row, m.to, slot) * F.lam_stride;
        q.l0 = lam[JT_LAM_LOGZ(nc)];
        q.l1 = lt[JT_LAM_COLL(nc) + m.to];
        q.l2 = lt[JT_LAM_SC(nc) + m.edge];
    } else if (m.kind == JT_MSG_PLAIN) {
        q.l0 = lam[JT_LAM_SC(nc) + m.edge];
        q.l1 = lam[JT_LAM_COLL(nc) + m.from];
    } else if (m.kind == JT_MSG_PLAIN_TOTAL) {
        q.l1 = lam[JT_LAM_COLL(nc) + m.from];
    }
    return q;
}

__device__ __forceinline__ void finalize_message(const FinPtrs &F, const JtMsg &m, const FinScalars &fs, int slot,
                                                 PassLds &L, float *lds_dyn, int lds_floats) {
    const int tid = threadIdx.x;
    const int lane = tid & (JT_WAVE - 1), wave = tid / JT_WAVE;
    const int nc = F.n_cliques;
    const float *P = F.partial + (int64_t)slot * F.partial_stride + m.partial_off;
    float *sep = F.sep + (int64_t)slot * F.sep_stride;
    double *lam = F.lam + (int64_t)slot * F.lam_stride;
    float *scl = F.scale + (int64_t)slot * F.scale_stride;
    const int ssize = m.ssize, nsplit = m.nsplit;
    float *raw = nullptr;
    if (m.kind == JT_MSG_COLLECT) raw = sep + m.sepc_off;
    if (m.kind == JT_MSG_DIST || m.kind == JT_MSG_PLAIN) raw = sep + m.sepd_off;
    // the old table of a distribute message is the target's collect message
    float *oldc = nullptr;
    if (m.kind == JT_MSG_DIST) oldc = F.sep + coll_slot(F.cs_row, m.to, slot) * F.sep_stride + m.sepc_off;
    if (m.kind == JT_MSG_PLAIN) oldc = sep + m.sepc_off;

    int CT = JT_BLOCK;
    if (ssize < JT_BLOCK) {
        CT = 1;
        while (CT < ssize) CT <<= 1;
    }
    const int R = JT_BLOCK / CT;
    const int jj = tid & (CT - 1), r = tid / CT;
    const int ncol = jj < ssize ? (ssize - jj + CT - 1) / CT : 0;
    const int nrow = r < nsplit ? (nsplit - r + R - 1) / R : 0;

    const double l0 = fs.l0, l1 = fs.l1, l2 = fs.l2;
    // old separator entries of the thread's first columns, in flight with
    // the partial rows
    float od[4] = {0.f, 0.f, 0.f, 0.f};
    if (oldc) {
        const int nod = R == 1 ? ncol : (r == 0 ? ncol : 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) od[q] = oldc[q < nod ? jj + CT * q : 0];   // unused when q >= nod
    }
    // column sums are staged in LDS when the separator fits (the block's
    // reduction rows, or the launch's ratio staging area, free by now), else
    // in the separator table itself
    float *stage = raw;
    if (R == 1 && ssize <= JT_WAVES_PER_BLOCK * JT_TILE_MAX) stage = &L.red[0][0];
    else if (R == 1 && ssize <= lds_floats) stage = lds_dyn;

    // 1. column sums; batch shape by the rows per thread (the shape depends
    //    on the message only, so the order is fixed)
    double local = 0.0;
    float first = 0.f;
    for (int c0 = 0; c0 < ncol;) {
        if (nrow <= 1) {
            local += column_sums<8, 1>(P, stage, ssize, CT, R, jj, r, c0, ncol, nrow, &first);
            c0 += 8;
        } else if (nrow <= 2) {
            local += column_sums<8, 2>(P, stage, ssize, CT, R, jj, r, c0, ncol, nrow, &first);
            c0 += 8;
        } else if (ncol - c0 <= 1) {
            // one column, many rows: 12 rows per batch (a 4 x 4 batch would
            // leave three of its four columns empty and take three times the
            // round trips); rows reach the same accumulators in the same order
            local += column_sums<1, 12>(P, stage, ssize, CT, R, jj, r, c0, ncol, nrow, &first);
            c0 += 1;
        } else {
            local += column_sums<4, 4>(P, stage, ssize, CT, R, jj, r, c0, ncol, nrow, &first);
            c0 += 4;
        }
    }
    if (R > 1) {
        // combine the R row groups of each column (fixed tree)
        float *red = &L.red[0][0];
        red[tid] = first;
        __syncthreads();
        for (int h = R >> 1; h > 0; h >>= 1) {
            if (r < h) red[tid] += red[tid + h * CT];
            __syncthreads();
        }
        first = red[jj];
        local = (r == 0 && jj < ssize) ? (double)first : 0.0;
    }
    // 2. sigma: wave trees, then the waves in order
    local = wave_sum_lane0(local);
    if (lane == 0) L.wsum[wave] = local;
    const double lc = fs.lc;
    __syncthreads();
    if (tid == 0) {
        const double sigma = ((L.wsum[0] + L.wsum[1]) + (L.wsum[2] + L.wsum[3]));
        const double ns = (double)ssize;
        double f = 0.0;
        switch (m.kind) {
            case JT_MSG_COLLECT: {
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
                const double logz = l0;
                double lsd = 0.0;
                if (sigma > 0.0) {
                    f = ns / sigma;
                    lsd = logz + log(sigma / ns);
                }
                lam[JT_LAM_SD(nc) + m.edge] = lsd;
                const double lcal = l1 + lsd - l2;
                scl[m.to] = (float)exp(lcal - logz);
                break;
            }
            case JT_MSG_PLAIN: {
                const double lold = l0;
                double lnew = lold;
                if (sigma > 0.0) {
                    f = ns / sigma;
                    lnew = l1 + log(sigma / ns);
                }
                lam[JT_LAM_COLL(nc) + m.to] += lnew - lold;
                lam[JT_LAM_SC(nc) + m.edge] = lnew;
                break;
            }
            case JT_MSG_PLAIN_TOTAL: {
                scl[m.from] = sigma > 0.0 ? (float)(1.0 / sigma) : 0.f;
                if (m.to == -2) {
                    lam[JT_LAM_LOGZ(nc)] = sigma > 0.0 ? l1 + log(sigma) : -INFINITY;
                    F.flag[slot] = sigma > 0.0 ? 0 : 1;
                }
                break;
            }
        }
        L.f = (float)f;
    }
    __syncthreads();
    if (!raw) return;
    const float f = L.f;
    // 3. rewrite the thread's columns, eight at a time (loads before stores)
    auto put = [&](int j, float v, float o) {
        const float nw = v * f;
        if (m.kind == JT_MSG_COLLECT) {
            raw[j] = nw;
        } else {
            raw[j] = (o == 0.f) ? 0.f : nw / o;
            if (m.kind == JT_MSG_PLAIN) oldc[j] = nw;
        }
    };
    if (R > 1) {
        if (r == 0 && jj < ssize) put(jj, first, od[0]);
        return;
    }
    for (int q0 = 0; q0 < ncol; q0 += 8) {
        float v8[8], o8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = q0 + u < ncol ? jj + CT * (q0 + u) : jj;   // out of range: re-read column jj, unused
            v8[u] = stage[j];   // this thread's own column sums
            o8[u] = oldc ? ((q0 == 0 && u < 4) ? od[u & 3] : oldc[j]) : 0.f;
        }
        issue_fence();
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (q0 + u < ncol) put(jj + CT * (q0 + u), v8[u], o8[u]);
    }
}


// Distribute messages with small separators and few partial rows are
// finalized by a single wave (no block barriers): lane l owns separator
// entries j = l + 64c.  Both pass kernels use this for exactly these
// messages, so a slot's bits do not depend on which kernel ran its pass.
#define JT_WFIN_MAX_SEP 255   // below the large-clique tree's smallest separators (256), where a block finalize is faster
#define JT_WFIN_MAX_ROWS 4
__device__ __forceinline__ bool wave_finalized(const JtMsg &m) {
    return m.kind == JT_MSG_DIST && m.ssize <= JT_WFIN_MAX_SEP && m.nsplit <= JT_WFIN_MAX_ROWS;
}

//  1. raw[j] = ((0 + P[0][j]) + P[1][j]) + ... in row order;
//  2. sigma = sum_j raw[j] in FP64: each lane its entries in ascending c,
//     then a fixed wave tree;
//  3. lane 0 updates the log-scales and the target's output scale;
//  4. ratio[j] = (raw[j] * |S| / sigma) / old[j], 0 where old[j] = 0.
__device__ __forceinline__ void wave_finalize_dist(const FinPtrs &F, const JtMsg &m, const FinScalars &fs, int slot,
                                                   int lane) {
    const int nc = F.n_cliques;
    const float *P = F.partial + (int64_t)slot * F.partial_stride + m.partial_off;
    float *raw = F.sep + (int64_t)slot * F.sep_stride + m.sepd_off;
    const float *oldc = F.sep + coll_slot(F.cs_row, m.to, slot) * F.sep_stride + m.sepc_off;
    double *lam = F.lam + (int64_t)slot * F.lam_stride;
    float *scl = F.scale + (int64_t)slot * F.scale_stride;
    const int ssize = m.ssize, nsplit = m.nsplit;
    constexpr int C = (JT_WFIN_MAX_SEP + JT_WAVE - 1) / JT_WAVE;
    float v[C], od[C];
    double local = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = lane + JT_WAVE * c;
        float x[JT_WFIN_MAX_ROWS];
        od[c] = 0.f;
        v[c] = 0.f;
        if (JT_WAVE * c >= ssize) continue;      // uniform: no column of this round exists
        const bool ok = j < ssize;
#pragma unroll
        for (int r = 0; r < JT_WFIN_MAX_ROWS; ++r) x[r] = (ok && r < nsplit) ? ldp(P + r * ssize + j) : 0.f;
        od[c] = ok ? oldc[j] : 0.f;
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < JT_WFIN_MAX_ROWS; ++r)
            if (r < nsplit) a += x[r];
        v[c] = a;
        if (ok) local += (double)a;
    }
    const double sigma = wave_sum_lane0(local);
    float f = 0.f;
    if (lane == 0) {
        const double ns = (double)ssize;
        const double logz = fs.l0;
        double lsd = 0.0, fd = 0.0;
        if (sigma > 0.0) {
            fd = ns / sigma;
            lsd = logz + log(sigma / ns);
        }
        lam[JT_LAM_SD(nc) + m.edge] = lsd;
        const double lcal = fs.l1 + lsd - fs.l2;
        scl[m.to] = (float)exp(lcal - logz);
        f = (float)fd;
    }
    f = __shfl(f, 0);
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int j = lane + JT_WAVE * c;
        if (JT_WAVE * c >= ssize) continue;
        if (j < ssize) {
            const float nw = v[c] * f;
            raw[j] = (od[c] == 0.f) ? 0.f : nw / od[c];
        }
    }
}
}  // namespace

// One launch = the passes of one tree level (or one message) for every slot.
// Buffers are separate __restrict__ parameters so the compiler can prove the
// metadata is never written by the kernel and read it through the scalar
// unit (uniform loads that do not wait on the streaming vector loads).
//
// A pass that sums into a separator also finalizes that message: every block
// of the item counts its arrival after its partials are written, and the
// block that arrives last sums all partial rows (fixed order), forms sigma,
// the log-scales and the new table or ratio.  No block ever waits for
// another, and the next level's launch sees finished messages.
//
// Work: a plain launch has n_tasks blocks per slot (block b: slot b / n_tasks,
// task b % n_tasks).  A listed launch reads its (task, slot) entries from
// `work`, one per block; its grid is at least the entry count (*work_count)
// and the blocks beyond it, and padding entries (task -1), return at once.
// Five waves per SIMD (five blocks per CU): the register budget that keeps
// enough tile loads in flight per CU (measured: 4 waves per SIMD costs 5 % on
// the large-clique tree and 10 % on the batched one).
extern "C" __global__ __launch_bounds__(JT_BLOCK) __attribute__((amdgpu_waves_per_eu(5, 8))) void jt_pass_kernel(
    const JtBlock *__restrict__ blocks, const JtGather *__restrict__ gathers,
    const int32_t *__restrict__ meta, const int32_t *__restrict__ ev_idx, const JtEv *__restrict__ ev_ent,
    const float *__restrict__ init, float *__restrict__ coll, float *__restrict__ out, float *__restrict__ sep,
    float *__restrict__ scale, float *__restrict__ partial, const JtMsg *__restrict__ msgs,
    const int32_t *__restrict__ child_edges, double *__restrict__ lam, int32_t *__restrict__ flag,
    int32_t *__restrict__ icnt, const int32_t *__restrict__ csrc, const JtWork *__restrict__ work,
    const int32_t *__restrict__ work_count, PassStrides st, int64_t lam_stride, int64_t icnt_stride,
    int64_t csrc_stride, int n_cliques, int task_begin, int n_tasks, int n_plain, int lds_floats, int flags) {
    // staged ratio tables, sized per launch
    extern __shared__ __align__(16) float lds_ratio[];
    __shared__ PassLds L;
    {
        const int w = blockIdx.x;
        int slot, tix;
        if (work) {
            // the entry is read whether or not the block is past the count
            // (the list holds work_cap >= grid entries, so the read stays
            // inside it either way)
            const JtWork e = work[w];
            // past the count, or per-XCD padding
            const int cnt = *work_count;
            if ((w >= cnt) | (e.task < 0)) return;
            tix = e.task;
            slot = e.slot;
        } else {
            if (w >= n_plain) return;
            slot = w / n_tasks;
            tix = w - slot * n_tasks;
        }
        const JtBlock *__restrict__ rec = blocks + task_begin + tix;
        const JtItem it = rec->it;
        const int32_t *__restrict__ cs_row = (flags & JT_PF_SHARE) ? csrc + (int64_t)slot * csrc_stride : nullptr;
        FinPtrs F;
        F.child_edges = child_edges;
        F.cs_row = cs_row;
        F.partial = partial;
        F.sep = sep;
        F.lam = lam;
        F.scale = scale;
        F.flag = flag;
        F.partial_stride = st.partial;
        F.sep_stride = st.sep;
        F.lam_stride = lam_stride;
        F.scale_stride = st.scale;
        F.n_cliques = n_cliques;
        JtTask task;
        task.item = rec->item;
        task.g0 = rec->g0;
        task.g1 = rec->g1;
        task.pad = 0;
        // source and destination tables of this slot; an absorbed collect
        // table is read from the clique's collect source
        const float *src;
        if (it.src_kind == JT_SRC_INIT)
            src = init + it.src_off;
        else if (it.src_kind == JT_SRC_COLL)
            src = coll + coll_slot(cs_row, it.clique, slot) * st.coll + it.src_off;
        else
            src = out + (int64_t)slot * st.out + it.src_off;
        float *dst = nullptr;
        if (it.dst_kind == JT_DST_COLL) dst = coll + (int64_t)slot * st.coll + it.dst_off;
        if (it.dst_kind == JT_DST_OUT) dst = out + (int64_t)slot * st.out + it.dst_off;
        // table entries are loaded through the caches (initial and
        // evidence-free tables are read by many slots) and stored
        // non-temporally; one instance per lane layout keeps the kernel's
        // code small
        if (it.pair)
            pass_block<4, 1>(it, task, slot, rec->g, gathers, meta, ev_idx, ev_ent, src, dst, sep, cs_row, scale,
                             partial, st, lds_ratio, L);
        else if (it.vec == 4)
            pass_block<4, 0>(it, task, slot, rec->g, gathers, meta, ev_idx, ev_ent, src, dst, sep, cs_row, scale,
                             partial, st, lds_ratio, L);
        else
            pass_block<1, 0>(it, task, slot, rec->g, gathers, meta, ev_idx, ev_ent, src, dst, sep, cs_row, scale,
                             partial, st, lds_ratio, L);
        if (it.msg >= 0) {
            int32_t *cnt = icnt + (int64_t)slot * icnt_stride + task.item;
            // Hand-off to the finalizing block, ordered by the hardware:
            //  1. partial rows are stored with agent-scope atomic stores, which
            //     on gfx950 write through the XCD's L2 to the device-coherent
            //     level (no dirty copy stays in a cache another XCD cannot see);
            //  2. every wave waits until its stores are acknowledged (vmcnt 0:
            //     the write has reached that level) before the barrier;
            //  3. thread 0 then counts the block's arrival with a device atomic,
            //     performed at that same level, so the count can only reach
            //     n_tasks after every block's rows are there;
            //  4. the last block's loads of the rows are issued after its atomic
            //     returned (barrier, branch on the result) and are agent-scope
            //     atomic loads, which bypass the non-coherent caches.
            // An acquire-release count (L2 write-back per block, L2 invalidate in
            // the last) gives the same results at a measured 1.6x the time of a
            // propagation, so the count stays relaxed.
            // The message record is issued here, in flight with the count; only
            // the finalizing block uses it (loaded at a block's start, its
            // scalar registers would be held -- and spilled -- through the pass).
            const JtMsg m = msgs[it.msg];
            wait_vm_stores();
            __syncthreads();
            bool last = true;
            if (it.n_tasks > 1) {
                if (threadIdx.x == 0) L.last = atomicAdd(cnt, 1) == it.n_tasks - 1;
                __syncthreads();
                last = L.last;
            }
            if (last) {
                const FinScalars fs = load_fin_scalars(F, m, slot);
                if (wave_finalized(m)) {
                    if (threadIdx.x < JT_WAVE) wave_finalize_dist(F, m, fs, slot, threadIdx.x);
                } else {
                    finalize_message(F, m, fs, slot, L, lds_ratio, lds_floats);
                }
                if (it.n_tasks > 1 && threadIdx.x == 0) *cnt = 0;    // ready for the next propagation
            }
        }
    }
}

// Multi-slot distribute launch (four blocks per CU, each serving up to JT_MS
// slots): entry e of `work` is (task, chunk): the task
// of every slot of chunks[chunk] (up to JT_MS slots reading the same source
// table).  task = -1 pads the per-XCD lists; such blocks return at once.
// After the pass each slot of the set counts its arrival, and the block
// finalizes the messages of the slots it arrived last for, one after the
// other (same hand-off as the single-slot kernel).
extern "C" __global__ __launch_bounds__(JT_BLOCK) __attribute__((amdgpu_waves_per_eu(4, 8))) void jt_pass_multi_kernel(
    const JtBlock *__restrict__ blocks, const int32_t *__restrict__ meta, const float *__restrict__ init,
    const float *__restrict__ coll, float *__restrict__ out, float *__restrict__ sep, float *__restrict__ scale,
    float *__restrict__ partial, const JtMsg *__restrict__ msgs, const int32_t *__restrict__ child_edges,
    double *__restrict__ lam, int32_t *__restrict__ flag, int32_t *__restrict__ icnt,
    const int32_t *__restrict__ csrc, const JtWork *__restrict__ work, const int32_t *__restrict__ work_count,
    const JtChunk *__restrict__ chunks, PassStrides st, int64_t lam_stride, int64_t icnt_stride, int64_t csrc_stride,
    int n_cliques, int task_begin, int lds_floats) {
    extern __shared__ __align__(16) float lds_ratio[];
    __shared__ PassLds L;
    __shared__ float posk[JT_MS][JT_TILE_MAX];
    __shared__ int64_t ms_part[JT_MS];
    __shared__ int64_t ms_dst[JT_MS];
    __shared__ float ms_scl[JT_MS];
    __shared__ int32_t ms_slot[JT_MS];
    __shared__ int32_t ms_last[JT_MS];
    const int w = blockIdx.x;
    const JtWork e = work[w];
    const int cnt = *work_count;
    if ((w >= cnt) | (e.task < 0)) return;
    const JtChunk chk = chunks[e.slot];
    int ns = 0;
#pragma unroll
    for (int k = 0; k < JT_MS; ++k) ns += chk.s[k] >= 0 ? 1 : 0;
    const JtBlock *__restrict__ rec = blocks + task_begin + e.task;
    const JtItem it = rec->it;
    const JtGather G = rec->g[0];
    JtTask task;
    task.item = rec->item;
    task.g0 = rec->g0;
    task.g1 = rec->g1;
    task.pad = 0;
    if (threadIdx.x < JT_MS) {
        const int k = threadIdx.x;
        const int32_t sk = chunks[e.slot].s[k];   // per-thread element: read from memory, not the register copy
        ms_slot[k] = sk;
        ms_part[k] = sk >= 0 ? (int64_t)sk * st.partial + it.partial_off : 0;
        ms_dst[k] = sk >= 0 ? (int64_t)sk * st.out + it.dst_off : 0;
        ms_scl[k] = sk >= 0 ? scale[(int64_t)sk * st.scale + it.scale_clique] : 0.f;
    }
    // every slot of the set reads the clique's collect data from the same
    // (evidence-free) slot, or the shared initial table
    const float *src = it.src_kind == JT_SRC_INIT
                           ? init + it.src_off
                           : coll + (int64_t)csrc[(int64_t)chk.s[0] * csrc_stride + it.clique] * st.coll + it.src_off;
    __syncthreads();
    if (it.pair)
        pass_multi<4, 1>(it, task, ms_slot, ns, G, meta, src, out, sep, scale, partial, st, lds_ratio, L, posk,
                         ms_part, ms_dst, ms_scl);
    else if (it.vec == 4)
        pass_multi<4, 0>(it, task, ms_slot, ns, G, meta, src, out, sep, scale, partial, st, lds_ratio, L, posk,
                         ms_part, ms_dst, ms_scl);
    else
        pass_multi<1, 0>(it, task, ms_slot, ns, G, meta, src, out, sep, scale, partial, st, lds_ratio, L, posk,
                         ms_part, ms_dst, ms_scl);
    if (it.msg < 0) return;
    const JtMsg m = msgs[it.msg];
    wait_vm_stores();   // this wave's partials are acknowledged (see jt_pass_kernel)
    __syncthreads();
    if (threadIdx.x < ns) {
        const int k = threadIdx.x;
        ms_last[k] = it.n_tasks > 1
                         ? atomicAdd(icnt + (int64_t)ms_slot[k] * icnt_stride + task.item, 1) == it.n_tasks - 1
                         : 1;
    }
    __syncthreads();
    FinPtrs F;
    F.child_edges = child_edges;
    F.partial = partial;
    F.sep = sep;
    F.lam = lam;
    F.scale = scale;
    F.flag = flag;
    F.partial_stride = st.partial;
    F.sep_stride = st.sep;
    F.lam_stride = lam_stride;
    F.scale_stride = st.scale;
    F.n_cliques = n_cliques;
    if (wave_finalized(m)) {
        // one wave per slot, four slots at a time
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / JT_WAVE);
        for (int k = wave; k < ns; k += JT_WAVES_PER_BLOCK) {
            if (!ms_last[k]) continue;
            const int slot = ms_slot[k];
            F.cs_row = csrc + (int64_t)slot * csrc_stride;
            const FinScalars fs = load_fin_scalars(F, m, slot);
            wave_finalize_dist(F, m, fs, slot, threadIdx.x & (JT_WAVE - 1));
            if (it.n_tasks > 1 && (threadIdx.x & (JT_WAVE - 1)) == 0) icnt[(int64_t)slot * icnt_stride + task.item] = 0;
        }
        return;
    }
    for (int k = 0; k < ns; ++k) {
        if (!ms_last[k]) continue;
        const int slot = ms_slot[k];
        F.cs_row = csrc + (int64_t)slot * csrc_stride;
        const FinScalars fs = load_fin_scalars(F, m, slot);
        finalize_message(F, m, fs, slot, L, lds_ratio, lds_floats);
        if (it.n_tasks > 1 && threadIdx.x == 0) icnt[(int64_t)slot * icnt_stride + task.item] = 0;
        __syncthreads();
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

// A plain launch: n_tasks blocks for each of n_slots slots.  A listed launch
// (work_off >= 0): `grid` blocks, at least the count d.work_count[work_idx]
// of entries d.work[work_off ..] and at most the list's capacity.
hipError_t jt_launch_pass(const JtDev &d, int task_begin, int n_tasks, int n_slots, int lds_floats, int flags,
                          int64_t work_off, int work_idx, int grid, hipStream_t s) {
    PassStrides st;
    st.coll = d.coll_stride;
    st.out = d.out_stride;
    st.sep = d.sep_stride;
    st.partial = d.partial_stride;
    st.scale = d.scale_stride;
    st.ev_idx = d.ev_idx_stride;
    st.ev_ent = d.ev_ent_stride;
    const bool listed = work_off >= 0;
    const unsigned blocks = listed ? (unsigned)grid : (unsigned)n_tasks * (unsigned)n_slots;
    hipLaunchKernelGGL(jt_pass_kernel, dim3(blocks), dim3(JT_BLOCK), (size_t)lds_floats * sizeof(float), s, d.blocks,
                       d.gathers, d.meta, d.ev_idx, d.ev_ent, d.init, d.coll, d.out, d.sep, d.scale, d.partial, d.msgs,
                       d.child_edges, d.lam, d.flag, d.icnt, d.csrc, listed ? d.work + work_off : nullptr,
                       listed ? d.work_count + work_idx : nullptr, st, d.lam_stride, d.icnt_stride, d.csrc_stride,
                       d.n_cliques, task_begin, n_tasks, n_tasks * n_slots, lds_floats, flags);
    return hipGetLastError();
}

hipError_t jt_launch_pass_multi(const JtDev &d, int task_begin, int lds_floats, int64_t work_off, int work_idx,
                                int grid, hipStream_t s) {
    PassStrides st;
    st.coll = d.coll_stride;
    st.out = d.out_stride;
    st.sep = d.sep_stride;
    st.partial = d.partial_stride;
    st.scale = d.scale_stride;
    st.ev_idx = d.ev_idx_stride;
    st.ev_ent = d.ev_ent_stride;
    hipLaunchKernelGGL(jt_pass_multi_kernel, dim3((unsigned)grid), dim3(JT_BLOCK), (size_t)lds_floats * sizeof(float), s,
                       d.blocks, d.meta, d.init, d.coll, d.out, d.sep, d.scale, d.partial, d.msgs, d.child_edges,
                       d.lam, d.flag, d.icnt, d.csrc, d.work + work_off, d.work_count + work_idx, d.chunks, st,
                       d.lam_stride, d.icnt_stride, d.csrc_stride, d.n_cliques, task_begin, lds_floats);
    return hipGetLastError();
}

hipError_t jt_launch_plain_init(const JtDev &d, int n_slots, hipStream_t s) {
    hipLaunchKernelGGL(jt_plain_init_kernel, dim3((unsigned)n_slots), dim3(JT_BLOCK), 0, s, d);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Read-out (Sec. 2.1: posteriors from the calibrated tables): the posteriors
// of slots [slot0, slot0 + n) packed in clique order, slot after slot, and
// their log Z (-inf when the evidence has probability zero).  Block
// (slot, clique) copies one table, float4 at a time when both ends allow.
// Read-out: the posteriors of slots [slot0, slot0 + n) packed in clique
// order, slot after slot, and each slot's log Z.  Block b copies a fixed
// chunk of one slot's packed range (blocks spread over every clique, however
// large): it finds the first clique overlapping its chunk by binary search
// over the packed offsets, then copies clique segment by clique segment, each
// thread four entries per round (loads before stores).
#define JT_RO_CHUNK 8192
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_read_out_kernel(
    const float *__restrict__ out, int64_t out_stride, const int64_t *__restrict__ cltab, int n_cliques,
    int slot0, int64_t packed_total, int n_chunks, const double *__restrict__ lam, int64_t lam_stride,
    const int32_t *__restrict__ flag, float *__restrict__ dst, double *__restrict__ log_z) {
    const int k = blockIdx.x / n_chunks, ch = blockIdx.x - k * n_chunks;
    const int slot = slot0 + k;
    const int64_t i0 = (int64_t)ch * JT_RO_CHUNK;
    const int64_t i1 = min(packed_total, i0 + (int64_t)JT_RO_CHUNK);
    if (ch == 0 && threadIdx.x == 0)
        log_z[k] = flag[slot] ? -INFINITY : lam[(int64_t)slot * lam_stride + JT_LAM_LOGZ(n_cliques)];
    // last clique whose packed offset is <= i0 (offsets ascend with the clique)
    int lo = 0, hi = n_cliques - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cltab[3 * mid + 2] <= i0) lo = mid;
        else hi = mid - 1;
    }
    const float *__restrict__ src = out + (int64_t)slot * out_stride;
    float *__restrict__ b = dst + (int64_t)k * packed_total;
    for (int c = lo; c < n_cliques; ++c) {
        const int64_t off = cltab[3 * c], n = cltab[3 * c + 1], po = cltab[3 * c + 2];
        if (po >= i1) break;
        const int64_t j0 = max(i0, po), j1 = min(i1, po + n);
        const int64_t shift = off - po;   // packed entry j of this clique is src[j + shift]
        for (int64_t j = j0 + threadIdx.x; j < j1; j += 4 * JT_BLOCK) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = j + u * JT_BLOCK < j1 ? src[j + u * JT_BLOCK + shift] : 0.f;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j + u * JT_BLOCK < j1) b[j + u * JT_BLOCK] = v[u];
        }
    }
}

hipError_t jt_launch_read_out(const JtDev &d, int slot0, int n_slots, int64_t packed_total, float *dst,
                              double *log_z, hipStream_t s) {
    const int64_t n_chunks = std::max<int64_t>(1, (packed_total + JT_RO_CHUNK - 1) / JT_RO_CHUNK);
    if (n_chunks * n_slots > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(jt_read_out_kernel, dim3((unsigned)(n_slots * n_chunks)), dim3(JT_BLOCK), 0, s, d.out,
                       d.out_stride, d.cltab, d.n_cliques, slot0, packed_total, (int)n_chunks, d.lam, d.lam_stride,
                       d.flag, dst, log_z);
    return hipGetLastError();
}
