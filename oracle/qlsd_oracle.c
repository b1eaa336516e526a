/*
 * qlsd_oracle.c -- plain, slow, obviously-correct CPU reference for BP + LSD.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP decoder is
 * checked against.  It shares no code, header, table or helper with the HIP
 * path.  Only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.
 *
 * Everything is float64 and single-shot; decode_batch only loops over shots
 * (optionally with OpenMP).  Paper references are to Hillmann et al.,
 * "Localized statistics decoding" (arXiv:2406.18655):
 *
 *   - decoding problem s = H e, minimum-weight goal ............ Sec. 2.1
 *   - min-sum BP, scaling 0.625, parallel (flooding) schedule .. Sec. 4.3 (Methods)
 *   - BP first; LSD on BP's soft output only if BP fails ...... Sec. 2.3
 *   - clusters, sub-matrix, validity, boundary, candidates .... Defs. 4.1-4.3
 *   - collisions / merges ..................................... Def. 4.4
 *   - LSD steps 1-6 and the serial loop ....................... Sec. 4.1, Alg. 1
 *   - synchronous growth rounds (all invalid clusters pick on
 *     the round-start state, then one union, then elimination) Appendix B, Alg. 2
 *   - local solve e_[C] = H_[C]^{-1} s_[C] .................... Eq. (2), Sec. 4.1 step 6
 *   - higher-order LSD-mu (mu extra growth steps, then local
 *     exhaustive OSD of order w per cluster) .................. Appendix D
 *   - OSD-0 (global reliability-ordered inversion) ............ Sec. 2.2 "Inversion decoding"
 *   - global OSD-CS of order w (the comparator of Sec. 2.3 and Appendix C, the global
 *     counterpart of LSD-mu's local OSD-CS) ................... Sec. 2.2, Sec. 2.3
 *
 * Readings where the paper is silent (the same ones the HIP path implements):
 *   BP   : r_{i->j} = (-1)^{s_i} * alpha * prod_{j'!=j} sgn(q_{j'->i}) * min_{j'!=j} |q_{j'->i}|,
 *          sgn(0)=+1; L_j = lambda_j + sum_i r_{i->j}; q_{j->i} = lambda_j + sum_{i'!=i} r_{i'->j}
 *          (exclusive sum written out); |q|,|L| clamped to 2^64; e_j = [L_j < 0];
 *          convergence tested after every iteration (>= 1 iteration).
 *   LSD  : key order (llr_j, j) ascending (index breaks ties, -0 == +0);
 *          Lambda(C) = N(rows(C)) \ cols(C); rows(C) = seed check + all checks of its
 *          columns; synchronous rounds; collisions through owned or simultaneously
 *          claimed checks; a merged group keeps its members' columns and appends the
 *          round's distinct new columns in ascending key; valid clusters do not grow
 *          but can be merged into; an invalid cluster with empty Lambda is frozen and
 *          flags UNSAT (its faults stay zero).
 *          The local solution is the unique x supported on the greedy pivot set of the
 *          cluster's columns (in cluster column order) with H_[rows,P] x = s_[rows].
 *   LSD-mu: after LSD-0, mu further rounds in which every non-frozen cluster grows;
 *          then per cluster: T = its non-pivot columns in ascending key, T_w its first
 *          w = min(mu,|T|); every pattern t over T_w is scored by the integer weight
 *          sum_{x_j=1} omega_j of x = (x_P(t), t); strict minimum, smaller t on ties.
 *   LSD-mu with local OSD-CS of order w (the combination sweep of the cited OSD work, used
 *          by Appendix D's bivariate bicycle study with growth steps and OSD order chosen
 *          separately): candidates in this order -- the zero pattern, every single column
 *          of T in key order, every pair (a, b), a < b < w' = min(w, |T|), of the first w'
 *          columns of T in lexicographic order; the strictly smallest integer weight wins,
 *          so ties go to the candidate met first.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ST_BP_CONVERGED 1u
#define ST_LSD_RUN 2u
#define ST_UNSAT 4u
#define ST_BAD_LLR 8u

/* ------------------------------------------------------------------ code */

typedef struct {
    int m, n, nnz;
    int32_t *row_ptr, *col_idx;            /* CSR (checks -> faults), edge id = CSR position */
    int32_t *col_ptr, *row_idx, *col_edge; /* CSC (faults -> checks) and the CSR edge id of each */
} ocode;

void *oracle_code_new(int m, int n, const int32_t *row_ptr, const int32_t *col_idx) {
    ocode *c = (ocode *)calloc(1, sizeof(ocode));
    int nnz = row_ptr[m];
    c->m = m; c->n = n; c->nnz = nnz;
    c->row_ptr = (int32_t *)malloc(sizeof(int32_t) * (m + 1));
    c->col_idx = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    memcpy(c->row_ptr, row_ptr, sizeof(int32_t) * (m + 1));
    memcpy(c->col_idx, col_idx, sizeof(int32_t) * nnz);
    c->col_ptr = (int32_t *)calloc(n + 1, sizeof(int32_t));
    c->row_idx = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    c->col_edge = (int32_t *)malloc(sizeof(int32_t) * (nnz > 0 ? nnz : 1));
    for (int e = 0; e < nnz; e++) c->col_ptr[col_idx[e] + 1]++;
    for (int j = 0; j < n; j++) c->col_ptr[j + 1] += c->col_ptr[j];
    int *fill = (int *)calloc(n, sizeof(int));
    for (int i = 0; i < m; i++)
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; e++) {
            int j = col_idx[e];
            int k = c->col_ptr[j] + fill[j]++;
            c->row_idx[k] = i;
            c->col_edge[k] = e;
        }
    free(fill);
    return c;
}

void oracle_code_free(void *p) {
    ocode *c = (ocode *)p;
    if (!c) return;
    free(c->row_ptr); free(c->col_idx); free(c->col_ptr); free(c->row_idx); free(c->col_edge);
    free(c);
}

/* prior log-likelihood ratios lambda_j = ln((1-p_j)/p_j); -1 if some p_j is not in (0,1) */
int oracle_lambda(const double *p, int n, double *lam) {
    for (int j = 0; j < n; j++) {
        if (!(p[j] > 0.0 && p[j] < 1.0)) return -1;
        lam[j] = log((1.0 - p[j]) / p[j]);
    }
    return 0;
}

/* integer OSD-E weights omega_j = round(2^20 * lambda_j) */
void oracle_omega(const double *lam, int n, int64_t *omega) {
    for (int j = 0; j < n; j++) omega[j] = (int64_t)llround(ldexp(lam[j], 20));
}

static int syndrome_ok(const ocode *c, const uint8_t *e, const uint8_t *s) {
    for (int i = 0; i < c->m; i++) {
        int par = 0;
        for (int k = c->row_ptr[i]; k < c->row_ptr[i + 1]; k++) par ^= e[c->col_idx[k]];
        if (par != (s[i] & 1)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------- BP */

static double clamp64(double x) {
    const double C = 18446744073709551616.0; /* 2^64 */
    return x > C ? C : (x < -C ? -C : x);
}

/*
 * Min-sum BP with the parallel schedule.  Returns 1 if H e = s was reached.
 * With early_exit == 0 all max_iter iterations run (the return value then says
 * whether the last one satisfies the syndrome).  *iters_out = iterations run.
 * *min_mag_out (nullable) receives the smallest |q_{j->i}| and |L_j| met over the iterations
 * run: a float32 run cannot be expected to reproduce the sign of a value that close to zero,
 * so shots whose trajectory passes near zero are where the two may part.  oracle_bp is the
 * same without it.
 */
int oracle_bp_traj(const void *code, const double *lam, const uint8_t *s, int max_iter, double alpha,
                   int early_exit, double *L_out, uint8_t *hard_out, int32_t *iters_out,
                   double *min_mag_out) {
    const ocode *c = (const ocode *)code;
    double min_mag = INFINITY;
    int E = c->nnz;
    double *q = (double *)malloc(sizeof(double) * (E > 0 ? E : 1));
    double *r = (double *)malloc(sizeof(double) * (E > 0 ? E : 1));
    double *L = (double *)malloc(sizeof(double) * (c->n > 0 ? c->n : 1));
    uint8_t *hard = (uint8_t *)malloc(c->n > 0 ? c->n : 1);
    for (int e = 0; e < E; e++) q[e] = lam[c->col_idx[e]];
    int it = 0, conv = 0;
    if (max_iter < 1) max_iter = 1;
    for (it = 1; it <= max_iter; it++) {
        /* check-node update: every outgoing message excludes its own edge */
        for (int i = 0; i < c->m; i++) {
            for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; e++) {
                double sgn = (s[i] & 1) ? -1.0 : 1.0;
                double mn = INFINITY;
                for (int e2 = c->row_ptr[i]; e2 < c->row_ptr[i + 1]; e2++) {
                    if (e2 == e) continue;
                    if (q[e2] < 0.0) sgn = -sgn;
                    double a = fabs(q[e2]);
                    if (a < mn) mn = a;
                }
                r[e] = sgn * alpha * mn;
            }
        }
        /* variable-node update: posterior and exclusive sums */
        for (int j = 0; j < c->n; j++) {
            double tot = lam[j];
            for (int k = c->col_ptr[j]; k < c->col_ptr[j + 1]; k++) tot += r[c->col_edge[k]];
            L[j] = clamp64(tot);
            if (fabs(L[j]) < min_mag) min_mag = fabs(L[j]);
            for (int k = c->col_ptr[j]; k < c->col_ptr[j + 1]; k++) {
                double x = lam[j];
                for (int k2 = c->col_ptr[j]; k2 < c->col_ptr[j + 1]; k2++)
                    if (k2 != k) x += r[c->col_edge[k2]];
                q[c->col_edge[k]] = clamp64(x);
                if (fabs(q[c->col_edge[k]]) < min_mag) min_mag = fabs(q[c->col_edge[k]]);
            }
            hard[j] = L[j] < 0.0 ? 1 : 0;
        }
        conv = syndrome_ok(c, hard, s);
        if (conv && early_exit) break;
    }
    if (it > max_iter) it = max_iter;
    if (L_out) memcpy(L_out, L, sizeof(double) * c->n);
    if (hard_out) memcpy(hard_out, hard, c->n);
    if (iters_out) *iters_out = it;
    if (min_mag_out) *min_mag_out = min_mag;
    free(q); free(r); free(L); free(hard);
    return conv;
}

int oracle_bp(const void *code, const double *lam, const uint8_t *s, int max_iter, double alpha,
              int early_exit, double *L_out, uint8_t *hard_out, int32_t *iters_out) {
    return oracle_bp_traj(code, lam, s, max_iter, alpha, early_exit, L_out, hard_out, iters_out, NULL);
}

/* ---------------------------------------------------- GF(2) elimination */

/*
 * Echelon elimination of a column list restricted to a row list (Gaussian
 * elimination, processed column by column in the given order).  A column is a
 * pivot iff it is independent of the columns before it.  comb[p] records which
 * of the listed columns sum to the reduced pivot vector, so that a right-hand
 * side in the span can be expressed in the original columns.
 */
typedef struct {
    int nr, nc, W, Wc, npiv;
    uint64_t *vec;   /* npiv x W  reduced pivot vectors      */
    uint64_t *comb;  /* npiv x Wc combination over listed cols */
    int *prow;       /* pivot row (local) of each pivot        */
    int *pcol;       /* listed-column index of each pivot      */
    uint8_t *is_piv; /* per listed column                      */
} elim_t;

static void bit_set(uint64_t *v, int k) { v[k >> 6] |= 1ull << (k & 63); }
static int bit_get(const uint64_t *v, int k) { return (int)((v[k >> 6] >> (k & 63)) & 1ull); }

static int lowest_bit(const uint64_t *v, int W) {
    for (int w = 0; w < W; w++)
        if (v[w]) return w * 64 + __builtin_ctzll(v[w]);
    return -1;
}

/* rowpos[i] = local index of check i inside the cluster, or -1 */
static void col_bits(const ocode *c, int j, const int *rowpos, uint64_t *out, int W) {
    memset(out, 0, sizeof(uint64_t) * W);
    for (int k = c->col_ptr[j]; k < c->col_ptr[j + 1]; k++) {
        int lp = rowpos[c->row_idx[k]];
        if (lp >= 0) bit_set(out, lp);
    }
}

static void elim_build(elim_t *el, const ocode *c, const int *rowpos, int nr, const int *cols, int nc) {
    el->nr = nr; el->nc = nc;
    el->W = (nr + 63) / 64; if (el->W < 1) el->W = 1;
    el->Wc = (nc + 63) / 64; if (el->Wc < 1) el->Wc = 1;
    el->npiv = 0;
    int cap = nc > 0 ? nc : 1;
    el->vec = (uint64_t *)calloc((size_t)cap * el->W, sizeof(uint64_t));
    el->comb = (uint64_t *)calloc((size_t)cap * el->Wc, sizeof(uint64_t));
    el->prow = (int *)malloc(sizeof(int) * cap);
    el->pcol = (int *)malloc(sizeof(int) * cap);
    el->is_piv = (uint8_t *)calloc(cap, 1);
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * el->W);
    uint64_t *cb = (uint64_t *)malloc(sizeof(uint64_t) * el->Wc);
    for (int t = 0; t < nc; t++) {
        col_bits(c, cols[t], rowpos, v, el->W);
        memset(cb, 0, sizeof(uint64_t) * el->Wc);
        bit_set(cb, t);
        for (int p = 0; p < el->npiv; p++) {
            if (bit_get(v, el->prow[p])) {
                for (int w = 0; w < el->W; w++) v[w] ^= el->vec[(size_t)p * el->W + w];
                for (int w = 0; w < el->Wc; w++) cb[w] ^= el->comb[(size_t)p * el->Wc + w];
            }
        }
        int r = lowest_bit(v, el->W);
        if (r >= 0) {
            int p = el->npiv++;
            memcpy(el->vec + (size_t)p * el->W, v, sizeof(uint64_t) * el->W);
            memcpy(el->comb + (size_t)p * el->Wc, cb, sizeof(uint64_t) * el->Wc);
            el->prow[p] = r;
            el->pcol[p] = t;
            el->is_piv[t] = 1;
        }
    }
    free(v); free(cb);
}

/* rhs (local rows, W words) -> x over listed columns (Wc words); returns 1 iff rhs is in the span */
static int elim_solve(const elim_t *el, const uint64_t *rhs, uint64_t *x) {
    uint64_t *v = (uint64_t *)malloc(sizeof(uint64_t) * el->W);
    memcpy(v, rhs, sizeof(uint64_t) * el->W);
    memset(x, 0, sizeof(uint64_t) * el->Wc);
    for (int p = 0; p < el->npiv; p++) {
        if (bit_get(v, el->prow[p])) {
            for (int w = 0; w < el->W; w++) v[w] ^= el->vec[(size_t)p * el->W + w];
            for (int w = 0; w < el->Wc; w++) x[w] ^= el->comb[(size_t)p * el->Wc + w];
        }
    }
    int ok = lowest_bit(v, el->W) < 0;
    free(v);
    return ok;
}

static void elim_free(elim_t *el) {
    free(el->vec); free(el->comb); free(el->prow); free(el->pcol); free(el->is_piv);
}

/* ------------------------------------------------------------------ LSD */

typedef struct {
    int *rows, nrows, *cols, ncols;
    int alive, valid, frozen;
} cluster_t;

static int key_less(const double *llr, int a, int b) {
    /* ascending (llr_j, j); -0.0 == +0.0 under C comparison, so the index decides */
    if (llr[a] < llr[b]) return 1;
    if (llr[a] > llr[b]) return 0;
    return a < b;
}

static int dsu_find(int *par, int x) {
    while (par[x] != x) { par[x] = par[par[x]]; x = par[x]; }
    return x;
}

static void dsu_union(int *par, int a, int b) {
    a = dsu_find(par, a); b = dsu_find(par, b);
    if (a == b) return;
    if (a < b) par[b] = a; else par[a] = b; /* the smaller id represents the group */
}

/* rowpos scratch must be all -1 on entry and is restored on exit */
static int cluster_is_valid(const ocode *c, const cluster_t *cl, const uint8_t *s, int *rowpos) {
    for (int t = 0; t < cl->nrows; t++) rowpos[cl->rows[t]] = t;
    elim_t el;
    elim_build(&el, c, rowpos, cl->nrows, cl->cols, cl->ncols);
    uint64_t *rhs = (uint64_t *)calloc(el.W, sizeof(uint64_t));
    uint64_t *x = (uint64_t *)calloc(el.Wc, sizeof(uint64_t));
    for (int t = 0; t < cl->nrows; t++) if (s[cl->rows[t]] & 1) bit_set(rhs, t);
    int ok = elim_solve(&el, rhs, x);
    free(rhs); free(x);
    elim_free(&el);
    for (int t = 0; t < cl->nrows; t++) rowpos[cl->rows[t]] = -1;
    return ok;
}

/*
 * Local solution of one valid cluster.  mu == 0: x on the pivot set, zero
 * elsewhere.  mu > 0: exhaustive search over the first w = min(mu,|T|) non-pivot
 * columns in key order, keeping the pattern of strictly smallest integer weight.
 */
static void cluster_solve(const ocode *c, const cluster_t *cl, const uint8_t *s, const double *llr,
                          int mu, int cs_order, const int64_t *omega, int *rowpos, uint8_t *corr) {
    for (int t = 0; t < cl->nrows; t++) rowpos[cl->rows[t]] = t;
    elim_t el;
    elim_build(&el, c, rowpos, cl->nrows, cl->cols, cl->ncols);
    uint64_t *rhs0 = (uint64_t *)calloc(el.W, sizeof(uint64_t));
    uint64_t *rhs = (uint64_t *)calloc(el.W, sizeof(uint64_t));
    uint64_t *x = (uint64_t *)calloc(el.Wc, sizeof(uint64_t));
    uint64_t *best = (uint64_t *)calloc(el.Wc, sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)calloc(el.W, sizeof(uint64_t));
    for (int t = 0; t < cl->nrows; t++) if (s[cl->rows[t]] & 1) bit_set(rhs0, t);

    /* T: non-pivot listed columns, ascending key */
    int nt = 0;
    int *T = (int *)malloc(sizeof(int) * (cl->ncols > 0 ? cl->ncols : 1));
    for (int t = 0; t < cl->ncols; t++) if (!el.is_piv[t]) T[nt++] = t;
    for (int a = 1; a < nt; a++) { /* insertion sort by key */
        int v = T[a], b = a - 1;
        while (b >= 0 && key_less(llr, cl->cols[v], cl->cols[T[b]])) { T[b + 1] = T[b]; b--; }
        T[b + 1] = v;
    }
    int64_t best_cost = 0;
    int have = 0;
    /* score one candidate: the columns T[sel[0..ns-1]] set, the pivot part solved */
    int sel[2];
    #define TRY_CANDIDATE(ns)                                                                    \
    do {                                                                                         \
        memcpy(rhs, rhs0, sizeof(uint64_t) * el.W);                                              \
        for (int q_ = 0; q_ < (ns); q_++) {                                                      \
            col_bits(c, cl->cols[T[sel[q_]]], rowpos, tmp, el.W);                                \
            for (int r_ = 0; r_ < el.W; r_++) rhs[r_] ^= tmp[r_];                                \
        }                                                                                        \
        if (elim_solve(&el, rhs, x)) {                                                           \
            for (int q_ = 0; q_ < (ns); q_++) bit_set(x, T[sel[q_]]);                            \
            int64_t cost_ = 0;                                                                   \
            for (int t_ = 0; t_ < cl->ncols; t_++)                                               \
                if (bit_get(x, t_)) cost_ += omega ? omega[cl->cols[t_]] : 1;                    \
            if (!have || cost_ < best_cost) {                                                    \
                have = 1; best_cost = cost_;                                                     \
                memcpy(best, x, sizeof(uint64_t) * el.Wc);                                       \
            }                                                                                    \
        }                                                                                        \
    } while (0)
    if (cs_order > 0) {
        /* combination sweep: zero pattern, all singles of T, pairs among its first w' */
        int w = cs_order < nt ? cs_order : nt;
        TRY_CANDIDATE(0);
        for (int a = 0; a < nt; a++) { sel[0] = a; TRY_CANDIDATE(1); }
        for (int a = 0; a < w; a++)
            for (int b = a + 1; b < w; b++) { sel[0] = a; sel[1] = b; TRY_CANDIDATE(2); }
    } else {
        int w = mu < nt ? mu : nt;
        if (w > 24) w = 24;
        for (uint64_t pat = 0; pat < (1ull << w); pat++) {
            memcpy(rhs, rhs0, sizeof(uint64_t) * el.W);
            for (int k = 0; k < w; k++)
                if ((pat >> k) & 1) {
                    col_bits(c, cl->cols[T[k]], rowpos, tmp, el.W);
                    for (int q = 0; q < el.W; q++) rhs[q] ^= tmp[q];
                }
            int ok = elim_solve(&el, rhs, x);
            if (!ok) continue; /* cannot happen for a valid cluster; kept for plainness */
            for (int k = 0; k < w; k++) if ((pat >> k) & 1) bit_set(x, T[k]);
            int64_t cost = 0;
            for (int t = 0; t < cl->ncols; t++) if (bit_get(x, t)) cost += omega ? omega[cl->cols[t]] : 1;
            if (!have || cost < best_cost) {
                have = 1; best_cost = cost;
                memcpy(best, x, sizeof(uint64_t) * el.Wc);
            }
        }
    }
    #undef TRY_CANDIDATE
    if (have)
        for (int t = 0; t < cl->ncols; t++) if (bit_get(best, t)) corr[cl->cols[t]] = 1;
    free(T); free(rhs0); free(rhs); free(x); free(best); free(tmp);
    elim_free(&el);
    for (int t = 0; t < cl->nrows; t++) rowpos[cl->rows[t]] = -1;
}

/*
 * One synchronous growth round (Alg. 2's find_candidate / parallel_union /
 * on-the-fly elimination, with Alg. 1's order: grow, then merge, then validate).
 * grow_all == 0: only invalid clusters grow (LSD-0); grow_all == 1: every
 * non-frozen cluster grows (the extra steps of LSD-mu).  Returns the number of
 * clusters that selected a column.
 */
static int lsd_round(const ocode *c, cluster_t *cl, int ncl, int *owner, int *incl, const uint8_t *s,
                     const double *llr, int grow_all, int force_merge, int *sel, int *dsu, int *claim,
                     int *rowpos, uint32_t *status) {
    int nsel = 0;
    for (int a = 0; a < ncl; a++) {
        sel[a] = -1;
        if (!cl[a].alive || cl[a].frozen) continue;
        if (!grow_all && cl[a].valid) continue;
        int best = -1;
        if (force_merge) {
            for (int j = 0; j < c->n; j++)
                if (incl[j] != a && (best < 0 || key_less(llr, j, best))) best = j;
        } else {
            for (int t = 0; t < cl[a].nrows; t++) {
                int i = cl[a].rows[t];
                for (int k = c->row_ptr[i]; k < c->row_ptr[i + 1]; k++) {
                    int j = c->col_idx[k];
                    if (incl[j] == a) continue;           /* already a column of this cluster */
                    if (best < 0 || key_less(llr, j, best)) best = j;
                }
            }
        }
        if (best < 0) {
            if (!cl[a].valid) { cl[a].frozen = 1; *status |= ST_UNSAT; }
            continue;
        }
        sel[a] = best;
        nsel++;
    }
    if (nsel == 0) return 0;

    for (int a = 0; a < ncl; a++) dsu[a] = a;
    for (int a = 0; a < ncl; a++) {
        if (sel[a] < 0) continue;
        int g = sel[a];
        for (int k = c->col_ptr[g]; k < c->col_ptr[g + 1]; k++) {
            int i = c->row_idx[k];
            if (owner[i] >= 0) dsu_union(dsu, a, owner[i]);
            else if (claim[i] >= 0) dsu_union(dsu, a, claim[i]);
            else claim[i] = a;
        }
    }

    /* rebuild every group that grew or merged */
    int *newcols = (int *)malloc(sizeof(int) * (ncl > 0 ? ncl : 1));
    for (int root = 0; root < ncl; root++) {
        if (dsu_find(dsu, root) != root || !cl[root].alive) continue;
        int members = 0, grew = 0;
        for (int a = root; a < ncl; a++)
            if (dsu_find(dsu, a) == root && cl[a].alive) { members++; if (sel[a] >= 0) grew = 1; }
        if (members < 2 && !grew) continue;

        int nr = 0, nc = 0;
        for (int a = root; a < ncl; a++)
            if (cl[a].alive && dsu_find(dsu, a) == root) { nr += cl[a].nrows; nc += cl[a].ncols; }
        int extra_rows = 0;
        for (int i = 0; i < c->m; i++) if (claim[i] >= 0 && dsu_find(dsu, claim[i]) == root) extra_rows++;
        int nnew = 0;
        for (int a = root; a < ncl; a++) {
            if (!cl[a].alive || dsu_find(dsu, a) != root || sel[a] < 0) continue;
            int g = sel[a], dup = 0;
            for (int t = 0; t < nnew; t++) if (newcols[t] == g) dup = 1;
            if (!dup) newcols[nnew++] = g;
        }
        for (int x = 1; x < nnew; x++) { /* ascending key */
            int v = newcols[x], y = x - 1;
            while (y >= 0 && key_less(llr, v, newcols[y])) { newcols[y + 1] = newcols[y]; y--; }
            newcols[y + 1] = v;
        }
        int *rows = (int *)malloc(sizeof(int) * (nr + extra_rows + 1));
        int *cols = (int *)malloc(sizeof(int) * (nc + nnew + 1));
        int pr = 0, pc = 0;
        for (int a = root; a < ncl; a++) {
            if (!cl[a].alive || dsu_find(dsu, a) != root) continue;
            memcpy(rows + pr, cl[a].rows, sizeof(int) * cl[a].nrows); pr += cl[a].nrows;
            memcpy(cols + pc, cl[a].cols, sizeof(int) * cl[a].ncols); pc += cl[a].ncols;
            if (a != root) {
                cl[a].alive = 0;
                free(cl[a].rows); free(cl[a].cols);
                cl[a].rows = cl[a].cols = NULL;
                cl[a].nrows = cl[a].ncols = 0;
            }
        }
        for (int i = 0; i < c->m; i++) if (claim[i] >= 0 && dsu_find(dsu, claim[i]) == root) rows[pr++] = i;
        for (int t = 0; t < nnew; t++) cols[pc++] = newcols[t];
        free(cl[root].rows); free(cl[root].cols);
        cl[root].rows = rows; cl[root].nrows = pr;
        cl[root].cols = cols; cl[root].ncols = pc;
        for (int t = 0; t < pr; t++) owner[rows[t]] = root;
        for (int t = 0; t < pc; t++) incl[cols[t]] = root;
        cl[root].valid = cluster_is_valid(c, &cl[root], s, rowpos);
    }
    free(newcols);
    for (int i = 0; i < c->m; i++) claim[i] = -1;
    return nsel;
}

/*
 * LSD (order mu) on soft information llr.  corr (n bytes) receives e_hat.
 * stats (nullable, 7 ints): final cluster count, largest cluster column count,
 * growth rounds, total clustered columns, total clustered checks, largest cluster
 * check count, sum over clusters of the squared column count.  Returns status bits.
 * force_merge != 0 puts every check into one cluster that may grow by any column:
 * the result is then global OSD-0.
 */
static int lsd_impl(const void *code, const uint8_t *s, const double *llr, int mu, int cs_order,
                    const int64_t *omega, int force_merge, uint8_t *corr, int32_t *stats);

int oracle_lsd(const void *code, const uint8_t *s, const double *llr, int mu, const int64_t *omega,
               int force_merge, uint8_t *corr, int32_t *stats) {
    return lsd_impl(code, s, llr, mu, 0, omega, force_merge, corr, stats);
}

/* LSD-mu whose local reprocessing is OSD-CS of order cs_order >= 1 instead of OSD-E (mu = 0:
 * LSD-0, no reprocessing). */
int oracle_lsd_cs(const void *code, const uint8_t *s, const double *llr, int mu, int cs_order,
                  const int64_t *omega, uint8_t *corr, int32_t *stats) {
    return lsd_impl(code, s, llr, mu, cs_order < 1 ? 1 : cs_order, omega, 0, corr, stats);
}

static int lsd_impl(const void *code, const uint8_t *s, const double *llr, int mu, int cs_order,
                    const int64_t *omega, int force_merge, uint8_t *corr, int32_t *stats) {
    const ocode *c = (const ocode *)code;
    uint32_t status = 0;
    memset(corr, 0, c->n);
    if (stats) memset(stats, 0, sizeof(int32_t) * 7);
    for (int j = 0; j < c->n; j++)
        if (isnan(llr[j])) return (int)ST_BAD_LLR;

    int m = c->m, n = c->n;
    int *owner = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    int *claim = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    int *rowpos = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    int *incl = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < m; i++) { owner[i] = -1; claim[i] = -1; rowpos[i] = -1; }
    for (int j = 0; j < n; j++) incl[j] = -1;

    /* step 1: one cluster per flipped detector (or one cluster over all checks) */
    int ncl = 0;
    cluster_t *cl = (cluster_t *)calloc(m > 0 ? m : 1, sizeof(cluster_t));
    int any = 0;
    for (int i = 0; i < m; i++) any |= s[i] & 1;
    if (!any) goto done;
    if (force_merge) {
        cl[0].rows = (int *)malloc(sizeof(int) * m);
        cl[0].cols = (int *)malloc(sizeof(int));
        for (int i = 0; i < m; i++) { cl[0].rows[i] = i; owner[i] = 0; }
        cl[0].nrows = m; cl[0].ncols = 0; cl[0].alive = 1; cl[0].valid = 0;
        ncl = 1;
    } else {
        for (int i = 0; i < m; i++) {
            if (!(s[i] & 1)) continue;
            cl[ncl].rows = (int *)malloc(sizeof(int));
            cl[ncl].cols = (int *)malloc(sizeof(int));
            cl[ncl].rows[0] = i; cl[ncl].nrows = 1; cl[ncl].ncols = 0;
            cl[ncl].alive = 1; cl[ncl].valid = 0; cl[ncl].frozen = 0;
            owner[i] = ncl;
            ncl++;
        }
    }

    {
        int *sel = (int *)malloc(sizeof(int) * ncl);
        int *dsu = (int *)malloc(sizeof(int) * ncl);
        int rounds = 0;
        /* steps 2-5: grow invalid clusters until none is left */
        for (;;) {
            int invalid = 0;
            for (int a = 0; a < ncl; a++) if (cl[a].alive && !cl[a].valid && !cl[a].frozen) invalid = 1;
            if (!invalid) break;
            lsd_round(c, cl, ncl, owner, incl, s, llr, 0, force_merge, sel, dsu, claim, rowpos, &status);
            rounds++;
        }
        /* LSD-mu: mu additional steps for every cluster */
        for (int t = 0; t < mu && !force_merge; t++) {
            if (!lsd_round(c, cl, ncl, owner, incl, s, llr, 1, 0, sel, dsu, claim, rowpos, &status)) break;
            rounds++;
        }
        /* step 6: local solutions, united into one correction */
        int nalive = 0, maxc = 0, tot = 0, totr = 0, maxr = 0, sumsq = 0;
        for (int a = 0; a < ncl; a++) {
            if (!cl[a].alive) continue;
            nalive++;
            tot += cl[a].ncols;
            sumsq += cl[a].ncols * cl[a].ncols;
            totr += cl[a].nrows;
            if (cl[a].ncols > maxc) maxc = cl[a].ncols;
            if (cl[a].nrows > maxr) maxr = cl[a].nrows;
            if (cl[a].frozen) continue;
            cluster_solve(c, &cl[a], s, llr, force_merge ? 0 : mu, (force_merge || mu == 0) ? 0 : cs_order, omega,
                          rowpos, corr);
        }
        if (stats) {
            stats[0] = nalive; stats[1] = maxc; stats[2] = rounds; stats[3] = tot;
            stats[4] = totr; stats[5] = maxr; stats[6] = sumsq;
        }
        free(sel); free(dsu);
    }
done:
    for (int a = 0; a < ncl; a++) { free(cl[a].rows); free(cl[a].cols); }
    free(cl); free(owner); free(claim); free(rowpos); free(incl);
    return (int)status;
}

/*
 * Global OSD-0: all columns in ascending key order, greedy pivot set over all
 * checks, e_hat on the pivot set solves H_[I] e = s.  Returns ST_UNSAT if s is
 * not in the image of H (then corr is all zero).
 */
int oracle_osd0(const void *code, const uint8_t *s, const double *llr, uint8_t *corr) {
    const ocode *c = (const ocode *)code;
    int m = c->m, n = c->n;
    memset(corr, 0, n);
    int *order = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int j = 0; j < n; j++) order[j] = j;
    for (int a = 1; a < n; a++) {
        int v = order[a], b = a - 1;
        while (b >= 0 && key_less(llr, v, order[b])) { order[b + 1] = order[b]; b--; }
        order[b + 1] = v;
    }
    int *rowpos = (int *)calloc(m > 0 ? m : 1, sizeof(int));
    for (int i = 0; i < m; i++) rowpos[i] = i;
    elim_t el;
    elim_build(&el, c, rowpos, m, order, n);
    uint64_t *rhs = (uint64_t *)calloc(el.W, sizeof(uint64_t));
    uint64_t *x = (uint64_t *)calloc(el.Wc, sizeof(uint64_t));
    for (int i = 0; i < m; i++) if (s[i] & 1) bit_set(rhs, i);
    int ok = elim_solve(&el, rhs, x);
    if (ok)
        for (int t = 0; t < n; t++) if (bit_get(x, t)) corr[order[t]] = 1;
    free(rhs); free(x); elim_free(&el); free(rowpos); free(order);
    return ok ? 0 : (int)ST_UNSAT;
}

/*
 * Global OSD-CS of order w: OSD-0's reliability order and greedy pivot set over all columns and
 * all checks, then the combination sweep of the local OSD-CS reading applied to the whole
 * matrix -- candidates in the order: the zero pattern (OSD-0), every single non-pivot column in
 * key order, every pair among the first min(w, |T|) non-pivot columns in lexicographic order;
 * each fixes those columns to one, solves the pivot part, and is scored by the integer weight
 * sum_{x_j=1} omega_j; the strictly smallest weight wins (ties to the candidate met first).
 * Returns ST_UNSAT (zero correction) if s is not in the image of H.
 */
int oracle_osd_cs(const void *code, const uint8_t *s, const double *llr, int cs_order, const int64_t *omega,
                  uint8_t *corr) {
    const ocode *c = (const ocode *)code;
    int m = c->m, n = c->n;
    memset(corr, 0, n);
    int *order = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *rows = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    for (int j = 0; j < n; j++) order[j] = j;
    for (int a = 1; a < n; a++) {
        int v = order[a], b = a - 1;
        while (b >= 0 && key_less(llr, v, order[b])) { order[b + 1] = order[b]; b--; }
        order[b + 1] = v;
    }
    for (int i = 0; i < m; i++) rows[i] = i;
    /* solvability first, on the same elimination OSD-0 uses */
    int *rowpos = (int *)calloc(m > 0 ? m : 1, sizeof(int));
    for (int i = 0; i < m; i++) rowpos[i] = i;
    elim_t el;
    elim_build(&el, c, rowpos, m, order, n);
    uint64_t *rhs = (uint64_t *)calloc(el.W, sizeof(uint64_t));
    uint64_t *x = (uint64_t *)calloc(el.Wc, sizeof(uint64_t));
    for (int i = 0; i < m; i++) if (s[i] & 1) bit_set(rhs, i);
    int ok = elim_solve(&el, rhs, x);
    free(rhs); free(x); elim_free(&el);
    if (ok) {
        /* the whole matrix as one cluster whose columns are listed in key order */
        cluster_t all;
        memset(&all, 0, sizeof(all));
        all.rows = rows; all.nrows = m; all.cols = order; all.ncols = n;
        all.alive = 1; all.valid = 1;
        for (int i = 0; i < m; i++) rowpos[i] = -1;
        cluster_solve(c, &all, s, llr, 0, cs_order < 1 ? 1 : cs_order, omega, rowpos, corr);
    }
    free(rowpos); free(rows); free(order);
    return ok ? 0 : (int)ST_UNSAT;
}

/* ------------------------------------------------------ cluster statistics */

/*
 * The optimal factorization of Appendix A: the clusters of an error are the connected
 * components of its faults in the fault graph (two faults adjacent iff they share a
 * detector).  out (4 values): number of clusters nu, largest cluster kappa (faults), total
 * faults, sum over clusters of the squared size (kappa_alpha = that / total).  Breadth-first
 * search from every unvisited faulty node.
 */
void oracle_error_clusters(const void *code, const uint8_t *e, int64_t *out) {
    const ocode *c = (const ocode *)code;
    int n = c->n;
    int *seen = (int *)calloc(n > 0 ? n : 1, sizeof(int));
    int *queue = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int64_t nu = 0, kappa = 0, tot = 0, sq = 0;
    for (int j0 = 0; j0 < n; j0++) {
        if (!(e[j0] & 1) || seen[j0]) continue;
        int head = 0, tail = 0;
        queue[tail++] = j0;
        seen[j0] = 1;
        while (head < tail) {
            int j = queue[head++];
            for (int k = c->col_ptr[j]; k < c->col_ptr[j + 1]; k++) {
                int i = c->row_idx[k];
                for (int q = c->row_ptr[i]; q < c->row_ptr[i + 1]; q++) {
                    int j2 = c->col_idx[q];
                    if ((e[j2] & 1) && !seen[j2]) { seen[j2] = 1; queue[tail++] = j2; }
                }
            }
        }
        nu++;
        tot += tail;
        sq += (int64_t)tail * tail;
        if (tail > kappa) kappa = tail;
    }
    out[0] = nu; out[1] = kappa; out[2] = tot; out[3] = sq;
    free(seen); free(queue);
}

/* ---------------------------------------------------------------- BP+LSD */

/*
 * Decode a batch: BP; if it converged its hard decision is the answer, else
 * LSD-mu on BP's final posterior LLRs.  status[b] gets ST_* bits, iters[b] the
 * BP iteration count.  llr_out (nullable, B x n) receives BP's final posterior.
 * nthreads <= 0 uses the OpenMP default.
 */
void oracle_decode_batch(const void *code, const double *lam, const uint8_t *S, int B, int max_iter,
                         double alpha, int mu, const int64_t *omega, uint8_t *corr, uint8_t *status,
                         int32_t *iters, double *llr_out, int nthreads) {
    const ocode *c = (const ocode *)code;
    int n = c->n, m = c->m;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *L = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
        uint8_t *hard = (uint8_t *)malloc(n > 0 ? n : 1);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int b = 0; b < B; b++) {
            const uint8_t *s = S + (size_t)b * m;
            int32_t it = 0;
            int conv = oracle_bp(code, lam, s, max_iter, alpha, 1, L, hard, &it);
            uint32_t st = 0;
            if (conv) {
                st |= ST_BP_CONVERGED;
                memcpy(corr + (size_t)b * n, hard, n);
            } else {
                st |= ST_LSD_RUN;
                st |= (uint32_t)oracle_lsd(code, s, L, mu, omega, 0, corr + (size_t)b * n, NULL);
            }
            status[b] = (uint8_t)st;
            iters[b] = it;
            if (llr_out) memcpy(llr_out + (size_t)b * n, L, sizeof(double) * n);
        }
        free(L); free(hard);
    }
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
