/*
 * jt_oracle.c -- plain, slow, sequential FP64 reference for junction-tree
 * belief propagation (Zheng, Mengshoel, Chong, "Belief Propagation by Message
 * Passing in Junction Trees: Computing Each Message Faster Using GPU
 * Parallelization").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or helper with the GPU
 * path; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg load it.  Nothing in the product path may call it.
 *
 * What it computes, in the paper's order and notation:
 *   - Index mapping tables mu_{X, phi_S(j)} (Sec. 3.2): the set of entries r
 *     of a clique table phi_X whose state string agrees with the separator
 *     entry j on the separator variables.  Built by decoding every r into
 *     its state string and projecting it onto S (the mapping rule of Sec. 3.1),
 *     so each list comes out in ascending r.  A literal per-entry scan (for
 *     each j, scan all r) is kept beside it so tests can check the two agree.
 *   - Message passing (eq. (1)-(3), Algorithm 1): marginalize phi_Xi into the
 *     new separator table, then multiply every entry of phi_Xk by new/old of
 *     its separator entry, with 0/0 := 0 (the rule stated after eq. (3)).
 *   - Collect_Evidence / Distribute_Evidence / Belief_Propagation
 *     (Algorithms 2-4): depth-first Hugin propagation from the root, children
 *     visited in ascending clique id; messages go child->parent in collect and
 *     parent->child in distribute.
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - tables are row-major with the last-listed variable fastest (Fig. 2);
 *   - separator variables are ordered by ascending global variable id;
 *   - the separator keeps the new table after each message (Hugin keeps the
 *     old and new separator tables, Sec. 3 step 2);
 *   - hard evidence zeroes the inconsistent entries of the lowest-id clique
 *     that contains the observed variable ("Initialization", Algorithm 4);
 *   - scaling: each new separator table is divided by its sum sigma and
 *     log(sigma) is carried in a per-table FP64 log-scale lambda; the
 *     represented joint prod T_C / prod T_S with T = phi * exp(lambda) is
 *     unchanged, so marginals and log Z do not depend on it.
 *
 * Op counting follows Sec. 3.4: a message i->k costs |phi_Xi| - |phi_S|
 * additions and |phi_Xk| + |phi_S| multiplications; the extra work of the
 * scaling (the sum sigma and the division by it) is counted separately.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define JO_OK 0
#define JO_ZERO_EVIDENCE 1
#define JO_E_ARG (-1)
#define JO_E_NOT_JT (-2)
#define JO_E_TOO_LARGE (-3)
#define JO_E_NOMEM (-4)

typedef struct {
    int n_vars;
    int32_t *card;
    int n_cliques;
    int64_t *clique_off;
    int32_t *clique_vars;
    int32_t *parent;
    int root;
    int64_t *tsize;       /* |phi_X| per clique */
    int64_t *toff;        /* offset of each table in the concatenation */
    /* separator of edge (c, parent(c)), variables in ascending id */
    int *sep_n;
    int32_t **sep_vars;
    int64_t *ssize;       /* |phi_S| per edge (index = child clique) */
    /* mu lists, concatenated: mu[c][side][j * m + n], side 0 = child clique,
       side 1 = parent clique; m = |phi_X| / |phi_S| */
    int32_t **mu_child;
    int32_t **mu_parent;
    int *home;            /* lowest clique id containing each variable */
    /* children lists in ascending id */
    int *child_off;
    int *child_list;
} jo_plan;

/* ------------------------------------------------------------------------- */
/* state strings (Sec. 3.1): index <-> per-variable states, last var fastest */

static void decode_index(int64_t r, int n, const int32_t *vars, const int32_t *card,
                         int32_t *states) {
    for (int i = n - 1; i >= 0; --i) {
        int32_t s = card[vars[i]];
        states[i] = (int32_t)(r % s);
        r /= s;
    }
}

static int64_t encode_index(int n, const int32_t *vars, const int32_t *card,
                            const int32_t *states) {
    int64_t r = 0;
    for (int i = 0; i < n; ++i) r = r * card[vars[i]] + states[i];
    return r;
}

/* mu lists of clique table X onto separator S by one pass over the table:
   decode r, project the state string onto S, encode j, append r to list j.
   Lists come out in ascending r.  out has |phi_X| entries. */
static int build_mu(int nx, const int32_t *xv, int64_t xsize, int ns, const int32_t *sv,
                    int64_t ssize, const int32_t *card, int32_t *out) {
    int64_t m = xsize / ssize;
    int *pos = (int *)malloc(sizeof(int) * (ns > 0 ? ns : 1));
    int32_t *xs = (int32_t *)malloc(sizeof(int32_t) * (nx > 0 ? nx : 1));
    int32_t *ss = (int32_t *)malloc(sizeof(int32_t) * (ns > 0 ? ns : 1));
    int64_t *fill = (int64_t *)calloc((size_t)ssize, sizeof(int64_t));
    if (!pos || !xs || !ss || !fill) {
        free(pos); free(xs); free(ss); free(fill);
        return JO_E_NOMEM;
    }
    for (int a = 0; a < ns; ++a) {
        pos[a] = -1;
        for (int b = 0; b < nx; ++b)
            if (xv[b] == sv[a]) pos[a] = b;
    }
    for (int64_t r = 0; r < xsize; ++r) {
        decode_index(r, nx, xv, card, xs);
        for (int a = 0; a < ns; ++a) ss[a] = xs[pos[a]];
        int64_t j = encode_index(ns, sv, card, ss);
        out[j * m + fill[j]] = (int32_t)r;
        fill[j]++;
    }
    free(pos); free(xs); free(ss); free(fill);
    return JO_OK;
}

/* The literal procedure of Sec. 3.1: for every separator entry j, convert j
   into its state string Y^j and scan all entries r of the clique table,
   keeping those whose state string agrees with Y^j on the separator
   variables.  Quadratic; used only on small tables to check build_mu. */
int jo_mu_scan_literal(int n_vars, const int32_t *card, int nx, const int32_t *xv, int ns,
                       const int32_t *sv, int32_t *out) {
    int64_t xsize = 1, ssize = 1;
    for (int i = 0; i < nx; ++i) {
        if (xv[i] < 0 || xv[i] >= n_vars) return JO_E_ARG;
        xsize *= card[xv[i]];
    }
    for (int i = 0; i < ns; ++i) {
        if (sv[i] < 0 || sv[i] >= n_vars) return JO_E_ARG;
        ssize *= card[sv[i]];
    }
    int32_t xs[64], ys[64];
    if (nx > 64 || ns > 64) return JO_E_ARG;
    int64_t k = 0;
    for (int64_t j = 0; j < ssize; ++j) {
        decode_index(j, ns, sv, card, ys);
        for (int64_t r = 0; r < xsize; ++r) {
            decode_index(r, nx, xv, card, xs);
            int agree = 1;
            for (int a = 0; a < ns && agree; ++a)
                for (int b = 0; b < nx; ++b)
                    if (xv[b] == sv[a] && xs[b] != ys[a]) { agree = 0; break; }
            if (agree) out[k++] = (int32_t)r;
        }
    }
    return JO_OK;
}

/* ------------------------------------------------------------------------- */

void jo_free(jo_plan *p) {
    if (!p) return;
    if (p->sep_vars)
        for (int c = 0; c < p->n_cliques; ++c) free(p->sep_vars[c]);
    if (p->mu_child)
        for (int c = 0; c < p->n_cliques; ++c) free(p->mu_child[c]);
    if (p->mu_parent)
        for (int c = 0; c < p->n_cliques; ++c) free(p->mu_parent[c]);
    free(p->card); free(p->clique_off); free(p->clique_vars); free(p->parent);
    free(p->tsize); free(p->toff); free(p->sep_n); free(p->sep_vars); free(p->ssize);
    free(p->mu_child); free(p->mu_parent); free(p->home); free(p->child_off);
    free(p->child_list);
    free(p);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Validate the tree and build separators and mu lists for every edge. */
int jo_create(int n_vars, const int32_t *card, int n_cliques, const int64_t *clique_off,
              const int32_t *clique_vars, const int32_t *parent, jo_plan **out) {
    if (!out || n_vars < 0 || n_cliques < 1 || !card || !clique_off || !clique_vars || !parent)
        return JO_E_ARG;
    *out = NULL;
    for (int v = 0; v < n_vars; ++v)
        if (card[v] < 1) return JO_E_ARG;
    jo_plan *p = (jo_plan *)calloc(1, sizeof(jo_plan));
    if (!p) return JO_E_NOMEM;
    int rc = JO_OK;
    p->n_vars = n_vars;
    p->n_cliques = n_cliques;
    int64_t nflat = clique_off[n_cliques];
    p->card = (int32_t *)malloc(sizeof(int32_t) * (n_vars > 0 ? n_vars : 1));
    p->clique_off = (int64_t *)malloc(sizeof(int64_t) * (n_cliques + 1));
    p->clique_vars = (int32_t *)malloc(sizeof(int32_t) * (nflat > 0 ? nflat : 1));
    p->parent = (int32_t *)malloc(sizeof(int32_t) * n_cliques);
    p->tsize = (int64_t *)calloc(n_cliques, sizeof(int64_t));
    p->toff = (int64_t *)calloc(n_cliques + 1, sizeof(int64_t));
    p->sep_n = (int *)calloc(n_cliques, sizeof(int));
    p->sep_vars = (int32_t **)calloc(n_cliques, sizeof(int32_t *));
    p->ssize = (int64_t *)calloc(n_cliques, sizeof(int64_t));
    p->mu_child = (int32_t **)calloc(n_cliques, sizeof(int32_t *));
    p->mu_parent = (int32_t **)calloc(n_cliques, sizeof(int32_t *));
    p->home = (int *)malloc(sizeof(int) * (n_vars > 0 ? n_vars : 1));
    p->child_off = (int *)calloc(n_cliques + 1, sizeof(int));
    p->child_list = (int *)calloc(n_cliques > 0 ? n_cliques : 1, sizeof(int));
    if (!p->card || !p->clique_off || !p->clique_vars || !p->parent || !p->tsize || !p->toff ||
        !p->sep_n || !p->sep_vars || !p->ssize || !p->mu_child || !p->mu_parent || !p->home ||
        !p->child_off || !p->child_list) {
        jo_free(p);
        return JO_E_NOMEM;
    }
    memcpy(p->card, card, sizeof(int32_t) * n_vars);
    memcpy(p->clique_off, clique_off, sizeof(int64_t) * (n_cliques + 1));
    if (nflat > 0) memcpy(p->clique_vars, clique_vars, sizeof(int32_t) * nflat);
    memcpy(p->parent, parent, sizeof(int32_t) * n_cliques);

    /* clique variable lists: in range, no duplicates; table sizes */
    if (clique_off[0] != 0) { rc = JO_E_ARG; goto fail; }
    for (int c = 0; c < n_cliques; ++c) {
        if (clique_off[c + 1] < clique_off[c]) { rc = JO_E_ARG; goto fail; }
        int64_t sz = 1;
        for (int64_t a = clique_off[c]; a < clique_off[c + 1]; ++a) {
            int32_t v = clique_vars[a];
            if (v < 0 || v >= n_vars) { rc = JO_E_ARG; goto fail; }
            for (int64_t b = clique_off[c]; b < a; ++b)
                if (clique_vars[b] == v) { rc = JO_E_ARG; goto fail; }
            sz *= card[v];
            if (sz > 2147483647LL) { rc = JO_E_TOO_LARGE; goto fail; }
        }
        p->tsize[c] = sz;
        p->toff[c + 1] = p->toff[c] + sz;
    }
    /* exactly one root, parents in range, no cycles */
    p->root = -1;
    for (int c = 0; c < n_cliques; ++c) {
        if (parent[c] == -1) {
            if (p->root >= 0) { rc = JO_E_NOT_JT; goto fail; }
            p->root = c;
        } else if (parent[c] < 0 || parent[c] >= n_cliques || parent[c] == c) {
            rc = JO_E_NOT_JT; goto fail;
        }
    }
    if (p->root < 0) { rc = JO_E_NOT_JT; goto fail; }
    for (int c = 0; c < n_cliques; ++c) {
        int x = c, steps = 0;
        while (x != p->root) {
            x = parent[x];
            if (++steps > n_cliques) { rc = JO_E_NOT_JT; goto fail; }
        }
    }
    /* children in ascending id */
    for (int c = 0; c < n_cliques; ++c)
        if (parent[c] >= 0) p->child_off[parent[c] + 1]++;
    for (int c = 0; c < n_cliques; ++c) p->child_off[c + 1] += p->child_off[c];
    {
        int *fill = (int *)calloc(n_cliques, sizeof(int));
        if (!fill) { rc = JO_E_NOMEM; goto fail; }
        for (int c = 0; c < n_cliques; ++c)
            if (parent[c] >= 0) {
                int q = parent[c];
                p->child_list[p->child_off[q] + fill[q]++] = c;
            }
        free(fill);
    }
    /* running intersection: the cliques holding a variable form a connected
       subtree, i.e. exactly one of them has a parent that lacks it */
    {
        int *tops = (int *)calloc(n_vars > 0 ? n_vars : 1, sizeof(int));
        if (!tops) { rc = JO_E_NOMEM; goto fail; }
        for (int v = 0; v < n_vars; ++v) p->home[v] = -1;
        for (int c = 0; c < n_cliques; ++c)
            for (int64_t a = clique_off[c]; a < clique_off[c + 1]; ++a) {
                int32_t v = clique_vars[a];
                if (p->home[v] < 0) p->home[v] = c;
                int q = parent[c], inpar = 0;
                if (q >= 0)
                    for (int64_t b = clique_off[q]; b < clique_off[q + 1]; ++b)
                        if (clique_vars[b] == v) inpar = 1;
                if (!inpar) tops[v]++;
            }
        for (int v = 0; v < n_vars; ++v)
            if (tops[v] > 1) { free(tops); rc = JO_E_NOT_JT; goto fail; }
        free(tops);
    }
    /* separators and mu lists, both sides of every edge */
    for (int c = 0; c < n_cliques; ++c) {
        int q = parent[c];
        if (q < 0) continue;
        int nx = (int)(clique_off[c + 1] - clique_off[c]);
        const int32_t *xv = clique_vars + clique_off[c];
        int nq = (int)(clique_off[q + 1] - clique_off[q]);
        const int32_t *qv = clique_vars + clique_off[q];
        int32_t *sv = (int32_t *)malloc(sizeof(int32_t) * (nx > 0 ? nx : 1));
        if (!sv) { rc = JO_E_NOMEM; goto fail; }
        int ns = 0;
        for (int a = 0; a < nx; ++a)
            for (int b = 0; b < nq; ++b)
                if (xv[a] == qv[b]) sv[ns++] = xv[a];
        qsort(sv, ns, sizeof(int32_t), cmp_i32);
        p->sep_vars[c] = sv;
        p->sep_n[c] = ns;
        int64_t ss = 1;
        for (int a = 0; a < ns; ++a) ss *= card[sv[a]];
        p->ssize[c] = ss;
        p->mu_child[c] = (int32_t *)malloc(sizeof(int32_t) * p->tsize[c]);
        p->mu_parent[c] = (int32_t *)malloc(sizeof(int32_t) * p->tsize[q]);
        if (!p->mu_child[c] || !p->mu_parent[c]) { rc = JO_E_NOMEM; goto fail; }
        rc = build_mu(nx, xv, p->tsize[c], ns, sv, ss, card, p->mu_child[c]);
        if (rc) goto fail;
        rc = build_mu(nq, qv, p->tsize[q], ns, sv, ss, card, p->mu_parent[c]);
        if (rc) goto fail;
    }
    *out = p;
    return JO_OK;
fail:
    jo_free(p);
    return rc;
}

/* Copy the mu lists of edge (child, parent(child)): side 0 = child's table,
   side 1 = parent's table.  out has |phi_X| entries: list j at [j*m, (j+1)*m). */
int jo_mu(const jo_plan *p, int child, int side, int32_t *out) {
    if (!p || child < 0 || child >= p->n_cliques || p->parent[child] < 0 || !out) return JO_E_ARG;
    int c = side ? p->parent[child] : child;
    memcpy(out, side ? p->mu_parent[child] : p->mu_child[child], sizeof(int32_t) * p->tsize[c]);
    return JO_OK;
}

/* The single cluster-sepset mapping table of CSM (the inverse of the mu
   lists): out[r] = j for every entry r of the table. */
int jo_map(const jo_plan *p, int child, int side, int32_t *out) {
    if (!p || child < 0 || child >= p->n_cliques || p->parent[child] < 0 || !out) return JO_E_ARG;
    int c = side ? p->parent[child] : child;
    const int32_t *mu = side ? p->mu_parent[child] : p->mu_child[child];
    int64_t m = p->tsize[c] / p->ssize[child];
    for (int64_t j = 0; j < p->ssize[child]; ++j)
        for (int64_t n = 0; n < m; ++n) out[mu[j * m + n]] = (int32_t)j;
    return JO_OK;
}

int64_t jo_sep_size(const jo_plan *p, int child) {
    if (!p || child < 0 || child >= p->n_cliques || p->parent[child] < 0) return -1;
    return p->ssize[child];
}

int jo_sep_vars(const jo_plan *p, int child, int32_t *out) {
    if (!p || child < 0 || child >= p->n_cliques || p->parent[child] < 0 || !out) return JO_E_ARG;
    memcpy(out, p->sep_vars[child], sizeof(int32_t) * p->sep_n[child]);
    return p->sep_n[child];
}

/* ------------------------------------------------------------------------- */
/* propagation state for one evidence set */

typedef struct {
    const jo_plan *p;
    double **phi;       /* clique tables */
    double **sep;       /* separator tables (old), one per edge */
    double *lam_c;      /* log-scale of every clique table */
    double *lam_s;      /* log-scale of every separator table */
    double *scratch;    /* new separator table */
    int zero;           /* some message had sigma == 0 */
    int64_t adds, muls, scale_adds, scale_muls;
} jo_state;

/* One message through the separator of edge `e` (e = the child clique),
   from clique `from` to clique `to` (eq. (1)-(3), Algorithm 1). */
static void message(jo_state *st, int e, int from, int to) {
    const jo_plan *p = st->p;
    int64_t ns = p->ssize[e];
    const int32_t *mu_from = (from == e) ? p->mu_child[e] : p->mu_parent[e];
    const int32_t *mu_to = (to == e) ? p->mu_child[e] : p->mu_parent[e];
    int64_t m_from = p->tsize[from] / ns;
    int64_t m_to = p->tsize[to] / ns;
    double *phi_from = st->phi[from];
    double *phi_to = st->phi[to];
    double *old = st->sep[e];
    double *nw = st->scratch;

    /* marginalization, eq. (2): sum phi_from over each mu list */
    for (int64_t j = 0; j < ns; ++j) {
        const int32_t *mu = mu_from + j * m_from;
        double s = phi_from[mu[0]];
        for (int64_t n = 1; n < m_from; ++n) s += phi_from[mu[n]];
        nw[j] = s;
        st->adds += m_from - 1;
    }
    /* scaling: divide by sigma, carry log(sigma) */
    double sigma = 0.0;
    for (int64_t j = 0; j < ns; ++j) sigma += nw[j];
    st->scale_adds += ns - 1;
    double lam_new;
    if (sigma > 0.0) {
        for (int64_t j = 0; j < ns; ++j) nw[j] /= sigma;
        st->scale_muls += ns;
        lam_new = st->lam_c[from] + log(sigma);
    } else {
        st->zero = 1;
        lam_new = st->lam_s[e];
    }
    /* scattering, eq. (3): multiply by new/old, 0/0 := 0 */
    for (int64_t j = 0; j < ns; ++j) {
        double ratio = (old[j] == 0.0) ? 0.0 : nw[j] / old[j];
        st->muls += 1;
        const int32_t *mu = mu_to + j * m_to;
        for (int64_t n = 0; n < m_to; ++n) phi_to[mu[n]] *= ratio;
        st->muls += m_to;
    }
    st->lam_c[to] += lam_new - st->lam_s[e];
    st->lam_s[e] = lam_new;
    memcpy(old, nw, sizeof(double) * ns);
}

/* Algorithm 2: children first, then the child's message to this clique. */
static void collect(jo_state *st, int c) {
    const jo_plan *p = st->p;
    for (int k = p->child_off[c]; k < p->child_off[c + 1]; ++k) {
        int ch = p->child_list[k];
        collect(st, ch);
        message(st, ch, ch, c);
    }
}

/* Algorithm 3: message to each child, then recurse into it. */
static void distribute(jo_state *st, int c) {
    const jo_plan *p = st->p;
    for (int k = p->child_off[c]; k < p->child_off[c + 1]; ++k) {
        int ch = p->child_list[k];
        message(st, ch, c, ch);
        distribute(st, ch);
    }
}

/* Algorithm 4 for one evidence set.
 *   potentials: FP32 tables concatenated in clique order (converted to FP64);
 *   ev_vars/ev_states: n_obs hard observations;
 *   marg_out: normalized calibrated tables P(X_C | e), concatenated (may be NULL);
 *   logz_out: log Z_e read at the root;
 *   logz_per_clique: lambda_C + log(sum phi_C) for every clique (may be NULL);
 *   counts[4]: adds, muls (Sec. 3.4), scaling adds, scaling muls (may be NULL).
 * Returns JO_OK, JO_ZERO_EVIDENCE (then logz = -inf and marg_out is zeroed),
 * or a negative error. */
int jo_run(const jo_plan *p, const float *potentials, int n_obs, const int32_t *ev_vars,
           const int32_t *ev_states, double *marg_out, double *logz_out, double *logz_per_clique,
           int64_t *counts) {
    if (!p || !potentials || !logz_out || n_obs < 0 || (n_obs > 0 && (!ev_vars || !ev_states)))
        return JO_E_ARG;
    for (int a = 0; a < n_obs; ++a) {
        int32_t v = ev_vars[a];
        if (v < 0 || v >= p->n_vars) return JO_E_ARG;
        if (ev_states[a] < 0 || ev_states[a] >= p->card[v]) return JO_E_ARG;
        for (int b = 0; b < a; ++b)
            if (ev_vars[b] == v && ev_states[b] != ev_states[a]) return JO_E_ARG;
    }
    int nc = p->n_cliques;
    jo_state st;
    memset(&st, 0, sizeof(st));
    st.p = p;
    st.phi = (double **)calloc(nc, sizeof(double *));
    st.sep = (double **)calloc(nc, sizeof(double *));
    st.lam_c = (double *)calloc(nc, sizeof(double));
    st.lam_s = (double *)calloc(nc, sizeof(double));
    int64_t maxs = 1;
    for (int c = 0; c < nc; ++c)
        if (p->parent[c] >= 0 && p->ssize[c] > maxs) maxs = p->ssize[c];
    st.scratch = (double *)malloc(sizeof(double) * maxs);
    int rc = JO_OK;
    if (!st.phi || !st.sep || !st.lam_c || !st.lam_s || !st.scratch) { rc = JO_E_NOMEM; goto out; }
    /* Initialization: tables from the (FP32) potentials, separators = 1 */
    for (int c = 0; c < nc; ++c) {
        st.phi[c] = (double *)malloc(sizeof(double) * p->tsize[c]);
        if (!st.phi[c]) { rc = JO_E_NOMEM; goto out; }
        const float *src = potentials + p->toff[c];
        for (int64_t r = 0; r < p->tsize[c]; ++r) st.phi[c][r] = (double)src[r];
        if (p->parent[c] >= 0) {
            st.sep[c] = (double *)malloc(sizeof(double) * p->ssize[c]);
            if (!st.sep[c]) { rc = JO_E_NOMEM; goto out; }
            for (int64_t j = 0; j < p->ssize[c]; ++j) st.sep[c][j] = 1.0;
        }
    }
    /* evidence: zero the entries of the home clique that disagree */
    {
        int32_t xs[64];
        for (int a = 0; a < n_obs; ++a) {
            int32_t v = ev_vars[a];
            int c = p->home[v];
            if (c < 0) continue;   /* variable in no clique: nothing to enter */
            int nx = (int)(p->clique_off[c + 1] - p->clique_off[c]);
            const int32_t *xv = p->clique_vars + p->clique_off[c];
            if (nx > 64) { rc = JO_E_ARG; goto out; }
            int pos = 0;
            for (int b = 0; b < nx; ++b)
                if (xv[b] == v) pos = b;
            for (int64_t r = 0; r < p->tsize[c]; ++r) {
                decode_index(r, nx, xv, p->card, xs);
                if (xs[pos] != ev_states[a]) st.phi[c][r] = 0.0;
            }
        }
    }
    collect(&st, p->root);
    distribute(&st, p->root);
    {
        double zroot = 0.0;
        for (int c = 0; c < nc; ++c) {
            double s = 0.0;
            for (int64_t r = 0; r < p->tsize[c]; ++r) s += st.phi[c][r];
            double lz = (s > 0.0) ? st.lam_c[c] + log(s) : -INFINITY;
            if (logz_per_clique) logz_per_clique[c] = lz;
            if (c == p->root) zroot = s;
            if (marg_out) {
                double *o = marg_out + p->toff[c];
                for (int64_t r = 0; r < p->tsize[c]; ++r) o[r] = (s > 0.0) ? st.phi[c][r] / s : 0.0;
            }
        }
        if (st.zero || !(zroot > 0.0)) {
            rc = JO_ZERO_EVIDENCE;
            *logz_out = -INFINITY;
            if (marg_out) memset(marg_out, 0, sizeof(double) * p->toff[nc]);
        } else {
            *logz_out = st.lam_c[p->root] + log(zroot);
        }
    }
    if (counts) {
        counts[0] = st.adds;
        counts[1] = st.muls;
        counts[2] = st.scale_adds;
        counts[3] = st.scale_muls;
    }
out:
    if (st.phi)
        for (int c = 0; c < nc; ++c) free(st.phi[c]);
    if (st.sep)
        for (int c = 0; c < nc; ++c) free(st.sep[c]);
    free(st.phi); free(st.sep); free(st.lam_c); free(st.lam_s); free(st.scratch);
    return rc;
}
