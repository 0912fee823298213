// jt_paper.hip -- the paper's own kernel design, kept as an ablation of the
// tiled engine: one message at a time in the depth-first order of
// Algorithms 2-3, and per message one thread per separator entry j that
// reads its explicit mapping lists (Sec. 3.2, Algorithm 1):
//   marginalize  new[j] = sum_n phi_from[mu_from(j, n)]      (eq. (2))
//   ratio        sigma = sum_j new[j]; ratio[j] = (new[j]*|S|/sigma) / old[j],
//                0 where old[j] = 0; old[j] = new[j]*|S|/sigma; log-scales
//   scatter      phi_to[mu_to(j, n)] *= ratio[j]               (eq. (3))
// Algorithm 1 runs the first and last step in one thread; the normalization
// between them (FP32 would overflow without it) needs sigma over all j, so
// the message is three launches.  The mapping lists are stored naive (list j
// contiguous) or interleaved (entry n of all lists contiguous: consecutive
// threads read consecutive words), the two layouts of Fig. 8.
#include <hip/hip_runtime.h>
#include <math.h>

#include "jt_internal.h"

namespace {

__device__ __forceinline__ int32_t mu_at(const int32_t *__restrict__ mu, int64_t base, int32_t layout, int32_t S,
                                          int32_t m, int32_t j, int32_t n) {
    return layout == JT_LAYOUT_INTERLEAVED_ ? mu[base + (int64_t)n * S + j] : mu[base + (int64_t)j * m + n];
}

}  // namespace

// Initialization (Algorithm 4) of one slot: posterior tables := initial
// tables with the slot's hard evidence entered (digit conditions of the
// tiled layout: an outer digit of tile r / T, an inner one of entry r % T).
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_paper_reset_kernel(
    const JtPaperBlk *__restrict__ blocks, const float *__restrict__ init, float *__restrict__ out,
    const int32_t *__restrict__ ev_idx, const JtEv *__restrict__ ev_ent) {
    const JtPaperBlk b = blocks[blockIdx.x];
    const int e0 = ev_idx[b.clique], e1 = ev_idx[b.clique + 1];
    for (int64_t r = b.start + threadIdx.x; r < b.end; r += JT_BLOCK) {
        float x = init[b.init_off + r];
        const int64_t o = r / b.T, i = r - o * b.T;
        for (int e = e0; e < e1; ++e) {
            const JtEv E = ev_ent[e];
            const int64_t d = E.outer ? o : i;
            if ((d / E.stride) % E.card != E.digit) x = 0.f;
        }
        out[b.out_off + r] = x;
    }
}

extern "C" __global__ void jt_paper_marg_kernel(JtPaperMsg m, const int32_t *__restrict__ mu, int32_t layout,
                                                const float *__restrict__ out, float *__restrict__ sep) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m.ssize) return;
    const float *__restrict__ phi = out + m.from_off;
    float s = 0.f;
    for (int32_t n = 0; n < m.m_from; ++n) s += phi[mu_at(mu, m.mu_from, layout, m.ssize, m.m_from, j, n)];
    sep[m.sepd_off + j] = s;
}

// One block: sigma (FP64, fixed order), the log-scales and the ratio, with
// the semantics of the one-message-at-a-time schedule.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_paper_ratio_kernel(JtPaperMsg m, float *__restrict__ sep,
                                                                            double *__restrict__ lam, int n_cliques) {
    __shared__ double ws[JT_BLOCK / JT_WAVE];
    __shared__ float fsh;
    const int tid = threadIdx.x, lane = tid & (JT_WAVE - 1), wave = tid / JT_WAVE;
    float *__restrict__ nw = sep + m.sepd_off;
    float *__restrict__ old = sep + m.sepc_off;
    double local = 0.0;
    for (int j = tid; j < m.ssize; j += JT_BLOCK) local += (double)nw[j];
#pragma unroll
    for (int off = JT_WAVE / 2; off > 0; off >>= 1) local += __shfl_down(local, off);
    if (lane == 0) ws[wave] = local;
    __syncthreads();
    if (tid == 0) {
        const double sigma = (ws[0] + ws[1]) + (ws[2] + ws[3]);
        const double ns = (double)m.ssize;
        const double lold = lam[JT_LAM_SC(n_cliques) + m.edge];
        double lnew = lold, f = 0.0;
        if (sigma > 0.0) {
            f = ns / sigma;
            lnew = lam[JT_LAM_COLL(n_cliques) + m.from] + log(sigma / ns);
        }
        lam[JT_LAM_COLL(n_cliques) + m.to] += lnew - lold;
        lam[JT_LAM_SC(n_cliques) + m.edge] = lnew;
        fsh = (float)f;
    }
    __syncthreads();
    const float f = fsh;
    for (int j = tid; j < m.ssize; j += JT_BLOCK) {
        const float v = nw[j] * f, o = old[j];
        nw[j] = (o == 0.f) ? 0.f : v / o;
        old[j] = v;
    }
}

extern "C" __global__ void jt_paper_scatter_kernel(JtPaperMsg m, const int32_t *__restrict__ mu, int32_t layout,
                                                   float *__restrict__ out, const float *__restrict__ sep) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m.ssize) return;
    float *__restrict__ phi = out + m.to_off;
    const float r = sep[m.sepd_off + j];
    for (int32_t n = 0; n < m.m_to; ++n) {
        const int32_t k = mu_at(mu, m.mu_to, layout, m.ssize, m.m_to, j, n);
        phi[k] = phi[k] * r;
    }
}

// Read-out (Sec. 2.1): block c sums clique c's calibrated table (FP64, fixed
// order) into its scale 1/sigma; the root's block also writes log Z.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_paper_total_kernel(
    const int64_t *__restrict__ cltab, const float *__restrict__ out, float *__restrict__ scale,
    double *__restrict__ lam, int32_t *__restrict__ flag, int n_cliques, int root) {
    __shared__ double ws[JT_BLOCK / JT_WAVE];
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & (JT_WAVE - 1), wave = tid / JT_WAVE;
    const float *__restrict__ t = out + cltab[3 * c];
    const int64_t n = cltab[3 * c + 1];
    double local = 0.0;
    for (int64_t r = tid; r < n; r += JT_BLOCK) local += (double)t[r];
#pragma unroll
    for (int off = JT_WAVE / 2; off > 0; off >>= 1) local += __shfl_down(local, off);
    if (lane == 0) ws[wave] = local;
    __syncthreads();
    if (tid == 0) {
        const double sigma = (ws[0] + ws[1]) + (ws[2] + ws[3]);
        scale[c] = sigma > 0.0 ? (float)(1.0 / sigma) : 0.f;
        if (c == root) {
            lam[JT_LAM_LOGZ(n_cliques)] = sigma > 0.0 ? lam[JT_LAM_COLL(n_cliques) + c] + log(sigma) : -INFINITY;
            flag[0] = sigma > 0.0 ? 0 : 1;
        }
    }
}

extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_paper_norm_kernel(const JtPaperBlk *__restrict__ blocks,
                                                                           float *__restrict__ out,
                                                                           const float *__restrict__ scale) {
    const JtPaperBlk b = blocks[blockIdx.x];
    const float f = scale[b.clique];
    for (int64_t r = b.start + threadIdx.x; r < b.end; r += JT_BLOCK) out[b.out_off + r] *= f;
}

// One propagation of slot `slot` (after the separators := 1 and log-scales
// := 0 set-up of the one-at-a-time schedule).
hipError_t jt_launch_paper_slot(const JtDev &d, const JtPaperMsg *host_msgs, int n_msgs, const JtPaperBlk *dev_blocks,
                                int n_blocks, const int32_t *dev_mu, int32_t layout, int32_t tpb, int32_t root,
                                int slot, hipStream_t s) {
    float *out = d.out + (int64_t)slot * d.out_stride;
    float *sep = d.sep + (int64_t)slot * d.sep_stride;
    double *lam = d.lam + (int64_t)slot * d.lam_stride;
    hipLaunchKernelGGL(jt_paper_reset_kernel, dim3((unsigned)n_blocks), dim3(JT_BLOCK), 0, s, dev_blocks, d.init, out,
                       d.ev_idx + (int64_t)slot * d.ev_idx_stride, d.ev_ent + (int64_t)slot * d.ev_ent_stride);
    for (int k = 0; k < n_msgs; ++k) {
        const JtPaperMsg &m = host_msgs[k];
        const unsigned g = (unsigned)((m.ssize + tpb - 1) / tpb);
        hipLaunchKernelGGL(jt_paper_marg_kernel, dim3(g), dim3((unsigned)tpb), 0, s, m, dev_mu, layout,
                           (const float *)out, sep);
        hipLaunchKernelGGL(jt_paper_ratio_kernel, dim3(1), dim3(JT_BLOCK), 0, s, m, sep, lam, d.n_cliques);
        hipLaunchKernelGGL(jt_paper_scatter_kernel, dim3(g), dim3((unsigned)tpb), 0, s, m, dev_mu, layout, out,
                           (const float *)sep);
    }
    hipLaunchKernelGGL(jt_paper_total_kernel, dim3((unsigned)d.n_cliques), dim3(JT_BLOCK), 0, s, d.cltab,
                       (const float *)out, d.scale + (int64_t)slot * d.scale_stride, lam, d.flag + slot, d.n_cliques,
                       root);
    hipLaunchKernelGGL(jt_paper_norm_kernel, dim3((unsigned)n_blocks), dim3(JT_BLOCK), 0, s, dev_blocks, out,
                       (const float *)(d.scale + (int64_t)slot * d.scale_stride));
    return hipGetLastError();
}
