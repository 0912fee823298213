// jt_bn.hip -- device side of the Bayesian-network front end:
//   * Initialization (Algorithm 4): every clique table is the product of the
//     conditional tables of the families assigned to it;
//   * expected counts (the E-step of EM over a batch of evidence sets): the
//     family marginals of the calibrated cliques summed over the slots.
#include <hip/hip_runtime.h>

#include "jt_internal.h"

#define JT_BN_TILES_PER_BLOCK 16

// Block (chunk, clique): tiles [chunk * 16, chunk * 16 + 16) of the clique;
// thread i < T owns in-tile position i.  The families are multiplied in
// ascending variable order (1 for a clique without one).
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_bn_init_kernel(
    const int32_t *__restrict__ meta, const JtFamily *__restrict__ fam, const int32_t *__restrict__ fam_rng,
    const JtCliqueShape *__restrict__ shape, const float *__restrict__ cpts, float *__restrict__ init) {
    const int c = blockIdx.y;
    const JtCliqueShape sh = shape[c];
    const int T = sh.T;
    const int64_t n_tiles = sh.n_tiles;
    const int64_t o0 = (int64_t)blockIdx.x * JT_BN_TILES_PER_BLOCK;
    const int i = threadIdx.x;
    if (o0 >= n_tiles || i >= T) return;
    const int f0 = fam_rng[c], f1 = fam_rng[c + 1];
    const int64_t o1 = o0 + JT_BN_TILES_PER_BLOCK < n_tiles ? o0 + JT_BN_TILES_PER_BLOCK : n_tiles;
    float *__restrict__ dst = init + sh.init_off;
    for (int64_t o = o0; o < o1; ++o) {
        float v = 1.f;
        for (int f = f0; f < f1; ++f) {
            const JtFamily F = fam[f];
            v *= cpts[F.cpt_off + meta[F.jin_off + i] + meta[F.jout_off + o]];
        }
        dst[o * T + i] = v;
    }
}

// Block (entry chunk, family fam0 + y): thread j sums entry j of the family's
// marginal of the calibrated clique over slots [s0, s0 + n_slots), then over
// the clique entries of list j in ascending order, in FP64, into
// dst[cpt_off - dst_base + j].  Expected counts (all active slots) and the
// read-out of merged cliques' original cliques (one slot) both use it.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_family_marginal_kernel(
    const JtFamily *__restrict__ fam, int fam0, const int32_t *__restrict__ mu, const int64_t *__restrict__ cltab,
    const float *__restrict__ out, int64_t out_stride, int s0, int n_slots, const JtCliqueShape *__restrict__ shape,
    float *__restrict__ dst, int64_t dst_base) {
    const JtFamily F = fam[fam0 + blockIdx.y];
    const int64_t j = (int64_t)blockIdx.x * JT_BLOCK + threadIdx.x;
    if (j >= F.fsize) return;
    const int64_t m = shape[F.clique].size / F.fsize;
    const int32_t *__restrict__ list = mu + F.mu_off + j * m;
    double acc = 0.0;
    for (int s = s0; s < s0 + n_slots; ++s) {
        const float *__restrict__ post = out + (int64_t)s * out_stride + cltab[3 * F.clique];
        for (int64_t n = 0; n < m; ++n) acc += (double)post[list[n]];
    }
    dst[F.cpt_off - dst_base + j] = (float)acc;
}

hipError_t jt_launch_bn_init(const JtDev &d, const JtFamily *fam, const int32_t *fam_rng, const JtCliqueShape *shape,
                             int n_cliques, int64_t max_tiles, const float *cpts, hipStream_t s) {
    const unsigned gx = (unsigned)((max_tiles + JT_BN_TILES_PER_BLOCK - 1) / JT_BN_TILES_PER_BLOCK);
    hipLaunchKernelGGL(jt_bn_init_kernel, dim3(gx, (unsigned)n_cliques), dim3(JT_BLOCK), 0, s, d.meta, fam, fam_rng,
                       shape, cpts, const_cast<float *>(d.init));
    return hipGetLastError();
}

hipError_t jt_launch_family_marginal(const JtDev &d, const JtFamily *fam, int fam0, int n_fam, int64_t max_fsize,
                                     const int32_t *mu, const JtCliqueShape *shape, int s0, int n_slots, float *dst,
                                     int64_t dst_base, hipStream_t s) {
    const unsigned gx = (unsigned)((max_fsize + JT_BLOCK - 1) / JT_BLOCK);
    hipLaunchKernelGGL(jt_family_marginal_kernel, dim3(gx, (unsigned)n_fam), dim3(JT_BLOCK), 0, s, fam, fam0, mu,
                       d.cltab, d.out, d.out_stride, s0, n_slots, shape, dst, dst_base);
    return hipGetLastError();
}

// M-step of EM: every row of every conditional table (the card[v] entries of
// one parent configuration, contiguous) becomes (counts + alpha) / sum of
// (counts + alpha) over the row, summed in FP64 in entry order.  Thread per
// row; rows of family k start at its cpt_off.
extern "C" __global__ __launch_bounds__(JT_BLOCK) void jt_bn_mstep_kernel(const JtFamily *__restrict__ fam,
                                                                         const int32_t *__restrict__ card,
                                                                         const float *__restrict__ counts, float alpha,
                                                                         float *__restrict__ cpts) {
    const JtFamily F = fam[blockIdx.y];
    const int k = card[F.var];
    const int64_t row = (int64_t)blockIdx.x * JT_BLOCK + threadIdx.x;
    if (row * k >= F.fsize) return;
    const int64_t b = F.cpt_off + row * k;
    double s = 0.0;
    for (int x = 0; x < k; ++x) s += (double)counts[b + x] + (double)alpha;
    for (int x = 0; x < k; ++x)
        cpts[b + x] = s > 0.0 ? (float)(((double)counts[b + x] + (double)alpha) / s) : 1.0f / (float)k;
}

hipError_t jt_launch_bn_mstep(const JtFamily *fam, int n_fam, int64_t max_rows, const int32_t *card,
                              const float *counts, float alpha, float *cpts, hipStream_t s) {
    const unsigned gx = (unsigned)((max_rows + JT_BLOCK - 1) / JT_BLOCK);
    hipLaunchKernelGGL(jt_bn_mstep_kernel, dim3(gx, (unsigned)n_fam), dim3(JT_BLOCK), 0, s, fam, card, counts, alpha,
                       cpts);
    return hipGetLastError();
}
