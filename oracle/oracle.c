/*
 * FP64 CPU reference implementation of the BDD Lagrange-decomposition method
 * (FastDOG, Abbas & Swoboda, CVPR 2022).  TEST INFRASTRUCTURE ONLY: the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load this file's
 * library; the solver product never does.  It shares no code with the HIP path.
 *
 * Plain and slow on purpose: every BDD is processed on its own, every quantity
 * recomputed from its definition, all arithmetic in double, compiled with
 * -ffp-contract=off.  The loops over independent BDDs (the "for j in parallel"
 * of Alg. 1) and over variables may run on several host threads (OpenMP,
 * or_set_threads); every sum still runs on one thread in a fixed order, so
 * the thread count never changes a result.
 *
 * Readings of the paper adopted here (each also listed in the design notes):
 *  - BDD of a row (Sec. 5, Def. "BDD" and "Constraint Set Correspondence"):
 *    nodes are the partial sums of the already-assigned variables that are
 *    reachable from the root and can still be completed to a feasible
 *    assignment; no node merging beyond equal partial sums.  Any BDD of the
 *    same set gives the same min-marginals (Sec. 5, remark on reduced BDDs).
 *  - Arc cost: 0 on zero-arcs, lambda of the *source* layer on one-arcs
 *    (Sec. 5, Def. "Weighted BDD"; the forward-pass listing indexes the cost
 *    by the target layer, which only reproduces Fig. 3 when read as the
 *    source layer).
 *  - Min-marginals (Sec. 5, min-marginal-via-shortest-path equation) use
 *    shortest paths that are consistent with the current multipliers: each
 *    sweep recomputes the opposite direction's distances before it starts.
 *  - The deferred differences M-bar are refreshed after *every* sweep, i.e.
 *    the averaging a_i = (omega/|J_i|) sum_k M_ik runs after the forward and
 *    after the backward sweep (Appendix, proof of Prop. 1, feasibility part:
 *    the identity sum_j (lambda_i^j + omega M_ij) = c_i holds only then).
 *    Sums over J_i run in ascending row order.
 *  - Lower bounds (Sec. 3 dual (D), Prop. 1): LB_free = sum_j E^j(lambda^j)
 *    + omega * sum_ij min(M_ij, 0) after each sweep; LB_cert =
 *    sum_j E^j(lambda^j + omega M^j) - sum_i max(r_i, 0) with the multiplier
 *    residual r_i = sum_j (lambda_i^j + omega M_ij) - c_i.
 *  - Termination step of Alg. 1: lambda += omega * M-bar (the algorithm's
 *    last loop); optionally the form the text describes, one more
 *    min-marginal averaging: lambda_i^j += (omega/|J_i|) sum_k M-bar_ik (or_set_termination).  Both
 *    give sum_j lambda_i^j = c_i; the certified bound uses the same form.
 *  - Serial averaging (ablation): the sequential update of Sec. 3 applied
 *    variable by variable in id order, full averaging, no damping, from the
 *    terminated multipliers (see or_run_serial).
 *  - Presolve: a variable that a single row allows only one value for is
 *    fixed and substituted until nothing changes (keeps all min-marginals
 *    finite); variables in no row take x_i = [c_i < 0].
 *  - Alg. 2: r ~ U[-delta, delta] and the perturbations +delta, -delta,
 *    r*delta, sign(sum M)*|r|*delta; "M = 0" means |M| <= tau; the loop runs
 *    while a variable has a zero or disagreeing sign, or belongs to a row the
 *    decoded point violates (those variables get r*delta); sign(0) := sign(r);
 *    re-optimisation = Alg. 1 with M-bar = 0 for `reopt_iters` iterations and
 *    its termination step; r comes from a counter-based SplitMix64 draw.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BOT (-1)
#define OR_TOP (-2)

enum { OR_OK = 0, OR_INVALID = -1, OR_INFEASIBLE = -2, OR_NOMEM = -3, OR_NOT_CONVERGED = -4 };

typedef struct {
    int k;              /* number of layers = number of variables of the row */
    int *var;           /* [k] variable ids, ascending */
    int *coef;          /* [k] coefficients */
    int *lstart;        /* [k+1] node id range of each layer */
    long long *state;   /* [n] partial sum carried by each node */
    int *lo, *hi;       /* [n] child node ids (local), OR_BOT or OR_TOP */
    int n;
} OBdd;

typedef struct {
    int status;
    double omega;
    /* original problem (kept for the final exact check) */
    long long n_vars, n_rows;
    double *cost;
    long long *row_ptr;
    int *col, *coef;
    signed char *sense;
    long long *rhs;
    /* presolve */
    signed char *fixed;      /* -1 free, else fixed value */
    double lb_offset;        /* cost of fixed variables + min(c,0) of unconstrained ones */
    /* subproblems: one per kept row */
    int nb;
    int *brow;               /* original row id */
    OBdd *bdd;
    long long np;            /* number of (variable, subproblem) pairs */
    long long *pstart;       /* [nb+1] pair range of each subproblem */
    int *pvar;               /* [np] */
    int *deg;                /* [n_vars] |J_i| */
    long long *vptr;         /* [n_vars+1] var -> pairs (ascending row order) */
    long long *vpair;        /* [np] */
    /* dual state */
    double *lam, *mm, *avg;
    double *E;               /* [nb] subproblem energy after the last sweep */
    int maxn, maxk;          /* largest node / layer count, for scratch */
    int term_mode;           /* termination step: 0 lambda + omega M-bar, 1 lambda + a_i */
    int nthreads;            /* host threads of the parallel loops (1 = serial) */
} OSolver;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */
static int sense_ok(long long v, int sense, long long b)
{
    if (sense < 0) return v <= b;
    if (sense > 0) return v >= b;
    return v == b;
}

static int cmp_ll(const void *a, const void *b)
{
    long long x = *(const long long *)a, y = *(const long long *)b;
    return (x > y) - (x < y);
}

/* sorted unique in place; returns new length */
static int uniq_ll(long long *v, int n)
{
    if (n == 0) return 0;
    qsort(v, (size_t)n, sizeof(long long), cmp_ll);
    int m = 1;
    for (int i = 1; i < n; ++i)
        if (v[i] != v[m - 1]) v[m++] = v[i];
    return m;
}

static int find_ll(const long long *v, int n, long long x)
{
    int a = 0, b = n - 1;
    while (a <= b) {
        int c = (a + b) / 2;
        if (v[c] == x) return c;
        if (v[c] < x) a = c + 1; else b = c - 1;
    }
    return -1;
}

static void bdd_free(OBdd *d)
{
    free(d->var); free(d->coef); free(d->lstart); free(d->state); free(d->lo); free(d->hi);
    memset(d, 0, sizeof(*d));
}

/*
 * Build the BDD of  sum_h a_h x_{v_h}  (sense)  b  over the given ascending
 * variables (Sec. 5, Def. "BDD").  Returns 0 on success, OR_INFEASIBLE when no
 * assignment satisfies the row.
 */
static int bdd_build(OBdd *d, int k, const int *vars, const int *coefs, int sense, long long b)
{
    memset(d, 0, sizeof(*d));
    d->k = k;
    d->var = malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
    d->coef = malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
    d->lstart = malloc(sizeof(int) * (size_t)(k + 1));
    memcpy(d->var, vars, sizeof(int) * (size_t)k);
    memcpy(d->coef, coefs, sizeof(int) * (size_t)k);

    /* R[h] = all values of sum_{l >= h} a_l x_l (suffix sums), sorted unique */
    long long **R = malloc(sizeof(long long *) * (size_t)(k + 1));
    int *Rn = malloc(sizeof(int) * (size_t)(k + 1));
    R[k] = malloc(sizeof(long long));
    R[k][0] = 0;
    Rn[k] = 1;
    for (int h = k - 1; h >= 0; --h) {
        int n = Rn[h + 1];
        R[h] = malloc(sizeof(long long) * (size_t)(2 * n));
        for (int i = 0; i < n; ++i) {
            R[h][i] = R[h + 1][i];
            R[h][n + i] = R[h + 1][i] + coefs[h];
        }
        Rn[h] = uniq_ll(R[h], 2 * n);
    }
    /* a partial sum s before layer h is alive if some completion satisfies the row */
    long long **S = malloc(sizeof(long long *) * (size_t)(k + 1));
    int *Sn = malloc(sizeof(int) * (size_t)(k + 1));
    int rc = 0;
    {
        int ok0 = 0;
        for (int i = 0; i < Rn[0]; ++i) ok0 |= sense_ok(R[0][i], sense, b);
        if (!ok0) rc = OR_INFEASIBLE;
    }
    if (rc == 0) {
        S[0] = malloc(sizeof(long long));
        S[0][0] = 0;
        Sn[0] = 1;
        for (int h = 0; h < k; ++h) {
            int n = Sn[h];
            long long *cand = malloc(sizeof(long long) * (size_t)(2 * n));
            int m = 0;
            for (int i = 0; i < n; ++i) {
                long long s0 = S[h][i], s1 = S[h][i] + coefs[h];
                for (int t = 0; t < 2; ++t) {
                    long long s = t ? s1 : s0;
                    int alive = 0;
                    for (int r = 0; r < Rn[h + 1]; ++r) alive |= sense_ok(s + R[h + 1][r], sense, b);
                    if (alive) cand[m++] = s;
                }
            }
            Sn[h + 1] = uniq_ll(cand, m);
            S[h + 1] = cand;
        }
        int total = 0;
        for (int h = 0; h < k; ++h) { d->lstart[h] = total; total += Sn[h]; }
        d->lstart[k] = total;
        d->n = total;
        d->state = malloc(sizeof(long long) * (size_t)(total > 0 ? total : 1));
        d->lo = malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
        d->hi = malloc(sizeof(int) * (size_t)(total > 0 ? total : 1));
        for (int h = 0; h < k; ++h) {
            for (int i = 0; i < Sn[h]; ++i) {
                int v = d->lstart[h] + i;
                long long s = S[h][i];
                d->state[v] = s;
                for (int t = 0; t < 2; ++t) {
                    long long c = s + (t ? coefs[h] : 0);
                    int child;
                    if (h == k - 1) {
                        child = sense_ok(c, sense, b) ? OR_TOP : OR_BOT;
                    } else {
                        int idx = find_ll(S[h + 1], Sn[h + 1], c);
                        child = idx < 0 ? OR_BOT : d->lstart[h + 1] + idx;
                    }
                    if (t) d->hi[v] = child; else d->lo[v] = child;
                }
            }
        }
        for (int h = 0; h <= k; ++h) free(S[h]);
    }
    for (int h = 0; h <= k; ++h) free(R[h]);
    free(R); free(Rn); free(S); free(Sn);
    if (rc != 0) bdd_free(d);
    return rc;
}

/* ------------------------------------------------------------------ */
/* shortest paths on one weighted BDD (Sec. 5, Def. "Weighted BDD")    */
/* cost[h] is the one-arc cost of layer h; zero-arcs cost 0.           */
/* ------------------------------------------------------------------ */

/* SP(r, v) for every node; returns SP(r, top) */
static double sp_from_root(const OBdd *d, const double *cost, double *F)
{
    double top = INFINITY;
    for (int v = 0; v < d->n; ++v) F[v] = INFINITY;
    if (d->n > 0) F[0] = 0.0;
    for (int h = 0; h < d->k; ++h) {
        for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
            for (int t = 0; t < 2; ++t) {
                int c = t ? d->hi[v] : d->lo[v];
                double val = t ? F[v] + cost[h] : F[v];
                if (c == OR_BOT) continue;
                if (c == OR_TOP) { if (val < top) top = val; }
                else if (val < F[c]) F[c] = val;
            }
        }
    }
    return top;
}

static double child_val(int c, const double *Bk)
{
    if (c == OR_TOP) return 0.0;
    if (c == OR_BOT) return INFINITY;
    return Bk[c];
}

/* SP(v, top) for every node; returns SP(r, top) */
static double sp_to_top(const OBdd *d, const double *cost, double *Bk)
{
    for (int h = d->k - 1; h >= 0; --h) {
        for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
            double b0 = child_val(d->lo[v], Bk);
            double b1 = child_val(d->hi[v], Bk) + cost[h];
            Bk[v] = b0 < b1 ? b0 : b1;
        }
    }
    return d->n > 0 ? Bk[0] : INFINITY;
}

/* m^0 and m^1 of layer h from SP(r, v) of the layer and SP(s(v), top) of its
 * children (Sec. 5, min-marginal-via-shortest-path equation). */
static void layer_min_marginals(const OBdd *d, int h, double cost_h, const double *F,
                                const double *Bk, double *m0, double *m1)
{
    double a = INFINITY, b = INFINITY;
    for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
        if (d->lo[v] != OR_BOT) {
            double t = F[v] + child_val(d->lo[v], Bk);
            if (t < a) a = t;
        }
        if (d->hi[v] != OR_BOT) {
            double t = (F[v] + cost_h) + child_val(d->hi[v], Bk);
            if (t < b) b = t;
        }
    }
    *m0 = a;
    *m1 = b;
}

/* ------------------------------------------------------------------ */
/* presolve + construction                                             */
/* ------------------------------------------------------------------ */
static int residual_row(const OSolver *s, long long r, int *vars, int *coefs, long long *rhs_out)
{
    int k = 0;
    long long rhs = s->rhs[r];
    for (long long e = s->row_ptr[r]; e < s->row_ptr[r + 1]; ++e) {
        int v = s->col[e], a = s->coef[e];
        if (a == 0) continue;
        if (s->fixed[v] >= 0) { rhs -= (long long)a * s->fixed[v]; continue; }
        vars[k] = v;
        coefs[k] = a;
        ++k;
    }
    /* ascending variable order (insertion sort; rows are short) */
    for (int i = 1; i < k; ++i) {
        int v = vars[i], a = coefs[i], j = i - 1;
        while (j >= 0 && vars[j] > v) { vars[j + 1] = vars[j]; coefs[j + 1] = coefs[j]; --j; }
        vars[j + 1] = v;
        coefs[j + 1] = a;
    }
    *rhs_out = rhs;
    return k;
}

void or_destroy(OSolver *s);

OSolver *or_create(long long n_vars, const double *cost, long long n_rows, const long long *row_ptr,
                   const int *col, const int *coef, const signed char *sense, const long long *rhs,
                   double omega)
{
    OSolver *s = calloc(1, sizeof(OSolver));
    s->omega = omega;
    s->nthreads = 1;
    s->n_vars = n_vars;
    s->n_rows = n_rows;
    long long nnz = row_ptr[n_rows];
    s->cost = malloc(sizeof(double) * (size_t)(n_vars + 1));
    s->row_ptr = malloc(sizeof(long long) * (size_t)(n_rows + 1));
    s->col = malloc(sizeof(int) * (size_t)(nnz + 1));
    s->coef = malloc(sizeof(int) * (size_t)(nnz + 1));
    s->sense = malloc((size_t)(n_rows + 1));
    s->rhs = malloc(sizeof(long long) * (size_t)(n_rows + 1));
    memcpy(s->cost, cost, sizeof(double) * (size_t)n_vars);
    memcpy(s->row_ptr, row_ptr, sizeof(long long) * (size_t)(n_rows + 1));
    memcpy(s->col, col, sizeof(int) * (size_t)nnz);
    memcpy(s->coef, coef, sizeof(int) * (size_t)nnz);
    memcpy(s->sense, sense, (size_t)n_rows);
    memcpy(s->rhs, rhs, sizeof(long long) * (size_t)n_rows);
    s->fixed = malloc((size_t)(n_vars + 1));
    memset(s->fixed, -1, (size_t)(n_vars + 1));

    int maxlen = 1;
    for (long long r = 0; r < n_rows; ++r) {
        if (row_ptr[r + 1] - row_ptr[r] > maxlen) maxlen = (int)(row_ptr[r + 1] - row_ptr[r]);
        for (long long e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
            if (col[e] < 0 || col[e] >= n_vars) { s->status = OR_INVALID; return s; }
    }
    int *vars = malloc(sizeof(int) * (size_t)maxlen);
    int *coefs = malloc(sizeof(int) * (size_t)maxlen);

    /* presolve: fix variables a row allows only one value for, until nothing changes */
    int changed = 1;
    while (changed && s->status == 0) {
        changed = 0;
        for (long long r = 0; r < n_rows && s->status == 0; ++r) {
            long long b;
            int k = residual_row(s, r, vars, coefs, &b);
            if (k == 0) {
                if (!sense_ok(0, s->sense[r], b)) s->status = OR_INFEASIBLE;
                continue;
            }
            OBdd d;
            if (bdd_build(&d, k, vars, coefs, s->sense[r], b) != 0) { s->status = OR_INFEASIBLE; break; }
            for (int h = 0; h < k; ++h) {
                int can0 = 0, can1 = 0;
                for (int v = d.lstart[h]; v < d.lstart[h + 1]; ++v) {
                    can0 |= d.lo[v] != OR_BOT;
                    can1 |= d.hi[v] != OR_BOT;
                }
                if (!can0 || !can1) {
                    s->fixed[vars[h]] = (signed char)(can1 ? 1 : 0);
                    changed = 1;
                }
            }
            bdd_free(&d);
        }
    }
    if (s->status != 0) { free(vars); free(coefs); return s; }

    /* one subproblem per row that still has free variables */
    s->brow = malloc(sizeof(int) * (size_t)(n_rows + 1));
    s->bdd = calloc((size_t)(n_rows + 1), sizeof(OBdd));
    s->pstart = malloc(sizeof(long long) * (size_t)(n_rows + 2));
    s->nb = 0;
    s->np = 0;
    s->pstart[0] = 0;
    for (long long r = 0; r < n_rows; ++r) {
        long long b;
        int k = residual_row(s, r, vars, coefs, &b);
        if (k == 0) continue;
        if (bdd_build(&s->bdd[s->nb], k, vars, coefs, s->sense[r], b) != 0) { s->status = OR_INFEASIBLE; break; }
        s->brow[s->nb] = (int)r;
        s->np += k;
        s->nb++;
        s->pstart[s->nb] = s->np;
    }
    free(vars);
    free(coefs);
    if (s->status != 0) return s;

    s->pvar = malloc(sizeof(int) * (size_t)(s->np + 1));
    s->deg = calloc((size_t)(n_vars + 1), sizeof(int));
    s->maxn = 1;
    s->maxk = 1;
    for (int j = 0; j < s->nb; ++j) {
        OBdd *d = &s->bdd[j];
        for (int h = 0; h < d->k; ++h) {
            s->pvar[s->pstart[j] + h] = d->var[h];
            s->deg[d->var[h]]++;
        }
        if (d->n > s->maxn) s->maxn = d->n;
        if (d->k > s->maxk) s->maxk = d->k;
    }
    s->vptr = calloc((size_t)(n_vars + 2), sizeof(long long));
    for (long long i = 0; i < n_vars; ++i) s->vptr[i + 1] = s->vptr[i] + s->deg[i];
    s->vpair = malloc(sizeof(long long) * (size_t)(s->np + 1));
    long long *fill = malloc(sizeof(long long) * (size_t)(n_vars + 1));
    memcpy(fill, s->vptr, sizeof(long long) * (size_t)n_vars);
    for (long long p = 0; p < s->np; ++p) s->vpair[fill[s->pvar[p]]++] = p;  /* pairs are in row order */
    free(fill);

    s->lb_offset = 0.0;
    for (long long i = 0; i < n_vars; ++i) {
        if (s->fixed[i] >= 0) s->lb_offset += s->fixed[i] ? cost[i] : 0.0;
        else if (s->deg[i] == 0) s->lb_offset += cost[i] < 0.0 ? cost[i] : 0.0;
    }
    s->lam = calloc((size_t)(s->np + 1), sizeof(double));
    s->mm = calloc((size_t)(s->np + 1), sizeof(double));
    s->avg = calloc((size_t)(n_vars + 1), sizeof(double));
    s->E = calloc((size_t)(s->nb + 1), sizeof(double));
    return s;
}

void or_destroy(OSolver *s)
{
    if (!s) return;
    if (s->bdd)
        for (int j = 0; j < s->nb; ++j) bdd_free(&s->bdd[j]);
    free(s->bdd); free(s->brow); free(s->pstart); free(s->pvar); free(s->deg); free(s->vptr);
    free(s->vpair); free(s->lam); free(s->mm); free(s->avg); free(s->E); free(s->fixed);
    free(s->cost); free(s->row_ptr); free(s->col); free(s->coef); free(s->sense); free(s->rhs);
    free(s);
}

/* ------------------------------------------------------------------ */
/* queries                                                             */
/* ------------------------------------------------------------------ */
int or_status(const OSolver *s) { return s->status; }
double or_lb_offset(const OSolver *s) { return s->lb_offset; }

void or_sizes(const OSolver *s, long long *nb, long long *np, long long *nn)
{
    long long n = 0;
    for (int j = 0; j < s->nb; ++j) n += s->bdd[j].n;
    *nb = s->nb;
    *np = s->np;
    *nn = n;
}

void or_pairs(const OSolver *s, int *pair_var, int *pair_row)
{
    for (int j = 0; j < s->nb; ++j)
        for (long long p = s->pstart[j]; p < s->pstart[j + 1]; ++p) {
            pair_var[p] = s->pvar[p];
            pair_row[p] = s->brow[j];
        }
}

void or_fixed(const OSolver *s, signed char *out) { memcpy(out, s->fixed, (size_t)s->n_vars); }

void or_get(const OSolver *s, double *lam, double *mm, double *avg)
{
    if (lam) memcpy(lam, s->lam, sizeof(double) * (size_t)s->np);
    if (mm) memcpy(mm, s->mm, sizeof(double) * (size_t)s->np);
    if (avg) memcpy(avg, s->avg, sizeof(double) * (size_t)s->n_vars);
}

void or_set(OSolver *s, const double *lam, const double *mm, const double *avg)
{
    if (lam) memcpy(s->lam, lam, sizeof(double) * (size_t)s->np);
    if (mm) memcpy(s->mm, mm, sizeof(double) * (size_t)s->np);
    if (avg) memcpy(s->avg, avg, sizeof(double) * (size_t)s->n_vars);
}

void or_energies(const OSolver *s, double *E) { memcpy(E, s->E, sizeof(double) * (size_t)s->nb); }

/* node table of subproblem j: layer, partial sum, children (local ids, -1 bot, -2 top) */
int or_bdd_nodes(const OSolver *s, int j, int *layer, long long *state, int *lo, int *hi)
{
    const OBdd *d = &s->bdd[j];
    for (int h = 0; h < d->k; ++h)
        for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
            if (layer) layer[v] = h;
            if (state) state[v] = d->state[v];
            if (lo) lo[v] = d->lo[v];
            if (hi) hi[v] = d->hi[v];
        }
    return d->n;
}

/* SP(r, .) and SP(., top) of subproblem j under the current multipliers */
void or_bdd_sp(const OSolver *s, int j, double *F, double *Bk, double *top_f, double *top_b)
{
    const OBdd *d = &s->bdd[j];
    const double *cost = s->lam + s->pstart[j];
    *top_f = sp_from_root(d, cost, F);
    *top_b = sp_to_top(d, cost, Bk);
}

/* ------------------------------------------------------------------ */
/* Alg. 1 building blocks                                              */
/* ------------------------------------------------------------------ */

/* lambda_i^j = c_i / |J_i|, M-bar = 0 (Alg. 1 initialisation, Sec. 3) */
void or_init(OSolver *s)
{
    for (long long p = 0; p < s->np; ++p) {
        int i = s->pvar[p];
        s->lam[p] = s->cost[i] / (double)s->deg[i];
        s->mm[p] = 0.0;
    }
    for (long long i = 0; i < s->n_vars; ++i) s->avg[i] = 0.0;
}

/* one sweep of subproblem j; dir 0 = ascending variables, 1 = descending.
 * update != 0 applies the deferred parallel update of Sec. 3; update == 0 only
 * records the min-marginal differences at fixed multipliers. */
static void sweep_one(OSolver *s, int j, int dir, int update, double *F, double *Bk, double *cost)
{
    const OBdd *d = &s->bdd[j];
    long long p0 = s->pstart[j];
    const double w = s->omega;
    for (int h = 0; h < d->k; ++h) cost[h] = s->lam[p0 + h];
    if (dir == 0) {
        sp_to_top(d, cost, Bk);
        double top = INFINITY;
        for (int v = 0; v < d->n; ++v) F[v] = INFINITY;
        F[0] = 0.0;
        for (int h = 0; h < d->k; ++h) {
            long long p = p0 + h;
            double m0, m1;
            layer_min_marginals(d, h, cost[h], F, Bk, &m0, &m1);
            s->mm[p] = m1 - m0;
            if (update) {
                s->lam[p] = (s->lam[p] - w * s->mm[p]) + s->avg[d->var[h]];
                cost[h] = s->lam[p];
            }
            for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
                for (int t = 0; t < 2; ++t) {
                    int c = t ? d->hi[v] : d->lo[v];
                    double val = t ? F[v] + cost[h] : F[v];
                    if (c == OR_BOT) continue;
                    if (c == OR_TOP) { if (val < top) top = val; }
                    else if (val < F[c]) F[c] = val;
                }
            }
        }
        s->E[j] = top;
    } else {
        sp_from_root(d, cost, F);
        for (int h = d->k - 1; h >= 0; --h) {
            long long p = p0 + h;
            double m0, m1;
            layer_min_marginals(d, h, cost[h], F, Bk, &m0, &m1);
            s->mm[p] = m1 - m0;
            if (update) {
                s->lam[p] = (s->lam[p] - w * s->mm[p]) + s->avg[d->var[h]];
                cost[h] = s->lam[p];
            }
            for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
                double b0 = child_val(d->lo[v], Bk);
                double b1 = child_val(d->hi[v], Bk) + cost[h];
                Bk[v] = b0 < b1 ? b0 : b1;
            }
        }
        s->E[j] = Bk[0];
    }
}

static void scratch3(const OSolver *s, double **F, double **Bk, double **cost)
{
    *F = malloc(sizeof(double) * (size_t)s->maxn);
    *Bk = malloc(sizeof(double) * (size_t)s->maxn);
    *cost = malloc(sizeof(double) * (size_t)s->maxk);
}

/* host threads for the parallel loops; subproblems of one sweep touch
 * disjoint pairs, so any thread count gives the same result */
void or_set_threads(OSolver *s, int n) { s->nthreads = n > 0 ? n : 1; }

/* sweep over every subproblem (the "for j in parallel" loop of Alg. 1) */
void or_sweep(OSolver *s, int dir, int update)
{
#pragma omp parallel num_threads(s->nthreads)
    {
        double *F, *Bk, *cost;
        scratch3(s, &F, &Bk, &cost);
#pragma omp for schedule(dynamic, 256)
        for (int j = 0; j < s->nb; ++j) sweep_one(s, j, dir, update, F, Bk, cost);
        free(F); free(Bk); free(cost);
    }
}

/* sweep over a chosen list of distinct subproblems only (they are independent) */
void or_sweep_subset(OSolver *s, int dir, int update, long long nsel, const long long *sel)
{
#pragma omp parallel num_threads(s->nthreads)
    {
        double *F, *Bk, *cost;
        scratch3(s, &F, &Bk, &cost);
#pragma omp for schedule(dynamic, 256)
        for (long long q = 0; q < nsel; ++q) sweep_one(s, (int)sel[q], dir, update, F, Bk, cost);
        free(F); free(Bk); free(cost);
    }
}

/* a_i = (omega / |J_i|) * sum_{k in J_i} M_ik, ascending row order (deferred M-bar <- M) */
void or_average(OSolver *s)
{
#pragma omp parallel for num_threads(s->nthreads) schedule(static)
    for (long long i = 0; i < s->n_vars; ++i) {
        if (s->deg[i] == 0) { s->avg[i] = 0.0; continue; }
        double sum = 0.0;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) sum += s->mm[s->vpair[q]];
        s->avg[i] = (s->omega / (double)s->deg[i]) * sum;
    }
}

/* LB_free = sum_j E^j(lambda^j) + omega * sum min(M, 0)  (+ presolve offset) */
double or_lb_free(const OSolver *s)
{
    double e = 0.0, t = 0.0;
    for (int j = 0; j < s->nb; ++j) e += s->E[j];
    for (long long p = 0; p < s->np; ++p) t += s->mm[p] < 0.0 ? s->mm[p] : 0.0;
    return (e + s->omega * t) + s->lb_offset;
}

void or_set_termination(OSolver *s, int mode) { s->term_mode = mode; }

/* the terminated multipliers of the current state, per pair (into t):
 * lambda + omega M-bar, or lambda_i^j + (omega/|J_i|) sum_k M-bar_ik with the
 * sum in ascending row order */
static void terminated(const OSolver *s, double *t)
{
    if (s->term_mode == 0) {
        for (long long p = 0; p < s->np; ++p) t[p] = s->lam[p] + s->omega * s->mm[p];
        return;
    }
#pragma omp parallel for num_threads(s->nthreads) schedule(static)
    for (long long i = 0; i < s->n_vars; ++i) {
        if (s->deg[i] == 0) continue;
        double sum = 0.0;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) sum += s->mm[s->vpair[q]];
        const double a = (s->omega / (double)s->deg[i]) * sum;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) t[s->vpair[q]] = s->lam[s->vpair[q]] + a;
    }
}

/* LB_cert = sum_j E^j(t'^j) (+ offset): the Lagrange dual (Sec. 3, problem
 * (D)) at t', the terminated multipliers t (lambda + omega M-bar by default)
 * made dual feasible by spreading each variable's residual
 * r_i = sum_j t_i^j - c_i evenly over its subproblems:
 * t'_i^j = t_i^j - r_i / |J_i|, so sum_j t'_i^j = c_i.  *max_residual gets
 * max_i |r_i| of t itself. */
double or_lb_cert(const OSolver *s, double *max_residual)
{
    double *t = malloc(sizeof(double) * (size_t)(s->np > 0 ? s->np : 1));
    double *Ej = malloc(sizeof(double) * (size_t)(s->nb > 0 ? s->nb : 1));
    terminated(s, t);
    double mr = 0.0;
    for (long long i = 0; i < s->n_vars; ++i) {
        if (s->deg[i] == 0) continue;
        double sum = 0.0;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) sum += t[s->vpair[q]];
        const double r = sum - s->cost[i];
        if (fabs(r) > mr) mr = fabs(r);
        const double share = r / (double)s->deg[i];
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) t[s->vpair[q]] = t[s->vpair[q]] - share;
    }
#pragma omp parallel num_threads(s->nthreads)
    {
        double *F = malloc(sizeof(double) * (size_t)s->maxn);
        double *cost = malloc(sizeof(double) * (size_t)s->maxk);
#pragma omp for schedule(dynamic, 256)
        for (int j = 0; j < s->nb; ++j) {
            const OBdd *d = &s->bdd[j];
            for (int h = 0; h < d->k; ++h) cost[h] = t[s->pstart[j] + h];
            Ej[j] = sp_from_root(d, cost, F);
        }
        free(F);
        free(cost);
    }
    double e = 0.0;
    for (int j = 0; j < s->nb; ++j) e += Ej[j];
    free(Ej);
    free(t);
    if (max_residual) *max_residual = mr;
    return e + s->lb_offset;
}

/* termination step of Alg. 1: lambda <- the terminated multipliers */
void or_terminate(OSolver *s)
{
    double *t = malloc(sizeof(double) * (size_t)(s->np > 0 ? s->np : 1));
    terminated(s, t);
    memcpy(s->lam, t, sizeof(double) * (size_t)s->np);
    free(t);
}

/* full Alg. 1 iterations from the current state; lb_hist gets LB_free after
 * every sweep (2 per iteration) when non-NULL */
void or_run_dual(OSolver *s, int n_iter, double *lb_hist)
{
    for (int it = 0; it < n_iter; ++it) {
        or_sweep(s, 0, 1);
        or_average(s);
        if (lb_hist) lb_hist[2 * it] = or_lb_free(s);
        or_sweep(s, 1, 1);
        or_average(s);
        if (lb_hist) lb_hist[2 * it + 1] = or_lb_free(s);
    }
}

/* ------------------------------------------------------------------ */
/* Serial min-marginal averaging (ablation of the deferred scheme)     */
/* ------------------------------------------------------------------ */

/* One sweep of the sequential scheme the paper compares against (Sec. 3,
 * update (dual_update_serial)): variables in ascending (dir 0) or descending
 * (dir 1) id order; for variable i, the min-marginal differences M_ik of
 * every subproblem k in J_i at the current multipliers, then
 *     lambda_i^k <- (lambda_i^k - M_ik) + (1/|J_i|) * sum_{k in J_i} M_ik
 * (sum in ascending row order) before the next variable is visited.  A
 * subproblem's layers come in variable order, so each sweep visits them in
 * order: dir 0 keeps SP(r, .) up to the current layer and uses SP(., top)
 * computed at the start of the sweep for the layers not yet visited (their
 * multipliers are unchanged), dir 1 the mirror image.  The update keeps
 * sum_k lambda_i^k unchanged, so multipliers that start dual feasible stay
 * feasible, and E^j after the sweep is the energy at the final multipliers. */
static void serial_sweep(OSolver *s, int dir, long long *noff, int *pb, double *F, double *Bk, double *cost)
{
    for (int j = 0; j < s->nb; ++j) {
        const OBdd *d = &s->bdd[j];
        for (int h = 0; h < d->k; ++h) cost[h] = s->lam[s->pstart[j] + h];
        if (dir == 0) {
            sp_to_top(d, cost, Bk + noff[j]);
            for (int v = 0; v < d->n; ++v) F[noff[j] + v] = INFINITY;
            if (d->n > 0) F[noff[j]] = 0.0;
            s->E[j] = INFINITY;
        } else {
            sp_from_root(d, cost, F + noff[j]);
        }
    }
    for (long long idx = 0; idx < s->n_vars; ++idx) {
        const long long i = dir == 0 ? idx : s->n_vars - 1 - idx;
        if (s->deg[i] == 0) continue;
        double sum = 0.0;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) {
            const long long p = s->vpair[q];
            const int j = pb[p];
            const int h = (int)(p - s->pstart[j]);
            double m0, m1;
            layer_min_marginals(&s->bdd[j], h, s->lam[p], F + noff[j], Bk + noff[j], &m0, &m1);
            s->mm[p] = m1 - m0;
            sum += s->mm[p];
        }
        const double a = (1.0 / (double)s->deg[i]) * sum;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) {
            const long long p = s->vpair[q];
            const int j = pb[p];
            const OBdd *d = &s->bdd[j];
            const int h = (int)(p - s->pstart[j]);
            s->lam[p] = (s->lam[p] - s->mm[p]) + a;
            double *Fj = F + noff[j], *Bj = Bk + noff[j];
            if (dir == 0) {
                for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v)
                    for (int t = 0; t < 2; ++t) {
                        int c = t ? d->hi[v] : d->lo[v];
                        double val = t ? Fj[v] + s->lam[p] : Fj[v];
                        if (c == OR_BOT) continue;
                        if (c == OR_TOP) { if (val < s->E[j]) s->E[j] = val; }
                        else if (val < Fj[c]) Fj[c] = val;
                    }
            } else {
                for (int v = d->lstart[h]; v < d->lstart[h + 1]; ++v) {
                    double b0 = child_val(d->lo[v], Bj);
                    double b1 = child_val(d->hi[v], Bj) + s->lam[p];
                    Bj[v] = b0 < b1 ? b0 : b1;
                }
                if (h == 0) s->E[j] = Bj[0];
            }
        }
    }
}

/* n_iter iterations (forward + backward sweep) of the serial scheme, starting
 * from the terminated multipliers (termination step of Alg. 1 first, so they
 * are dual feasible); lb_hist gets sum_j E^j + offset after every sweep when
 * non-NULL.  Afterwards M-bar = 0 and a_i = 0: lambda alone is the dual point. */
void or_run_serial(OSolver *s, int n_iter, double *lb_hist)
{
    long long *noff = malloc(sizeof(long long) * (size_t)(s->nb + 1));
    int *pb = malloc(sizeof(int) * (size_t)(s->np > 0 ? s->np : 1));
    double *cost = malloc(sizeof(double) * (size_t)(s->maxk > 0 ? s->maxk : 1));
    noff[0] = 0;
    for (int j = 0; j < s->nb; ++j) {
        noff[j + 1] = noff[j] + s->bdd[j].n;
        for (long long p = s->pstart[j]; p < s->pstart[j + 1]; ++p) pb[p] = j;
    }
    double *F = malloc(sizeof(double) * (size_t)(noff[s->nb] > 0 ? noff[s->nb] : 1));
    double *Bk = malloc(sizeof(double) * (size_t)(noff[s->nb] > 0 ? noff[s->nb] : 1));
    or_terminate(s);
    for (long long p = 0; p < s->np; ++p) s->mm[p] = 0.0;
    for (int it = 0; it < n_iter; ++it)
        for (int dir = 0; dir < 2; ++dir) {
            serial_sweep(s, dir, noff, pb, F, Bk, cost);
            if (lb_hist) {
                double e = 0.0;
                for (int j = 0; j < s->nb; ++j) e += s->E[j];
                lb_hist[2 * it + dir] = e + s->lb_offset;
            }
        }
    for (long long p = 0; p < s->np; ++p) s->mm[p] = 0.0;
    for (long long i = 0; i < s->n_vars; ++i) s->avg[i] = 0.0;
    free(noff); free(pb); free(cost); free(F); free(Bk);
}

/* ------------------------------------------------------------------ */
/* Alg. 2: perturbation primal rounding                                */
/* ------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea & Flood 2014) applied to
 * seed ^ round*K1 ^ i*K2; top 53 bits -> [0, 1) */
double or_rng_u01(unsigned long long seed, unsigned long long round, unsigned long long i)
{
    uint64_t z = (uint64_t)seed ^ ((uint64_t)round * 0xD1B54A32D192ED03ULL) ^ ((uint64_t)i * 0x8CB92BA72F3D8DD7ULL);
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int row_satisfied(const OSolver *s, long long r, const unsigned char *x)
{
    long long lhs = 0;
    for (long long e = s->row_ptr[r]; e < s->row_ptr[r + 1]; ++e) lhs += (long long)s->coef[e] * x[s->col[e]];
    return sense_ok(lhs, s->sense[r], s->rhs[r]);
}

/* count of variables whose min-marginal differences are not all > tau or all < -tau */
static long long count_conflicts(const OSolver *s, double tau, const unsigned char *flag)
{
    long long n = 0;
    for (long long i = 0; i < s->n_vars; ++i) {
        if (s->deg[i] == 0) continue;
        int pos = 1, neg = 1;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) {
            double m = s->mm[s->vpair[q]];
            pos &= m > tau;
            neg &= m < -tau;
        }
        if (flag[i] || !(pos || neg)) ++n;
    }
    return n;
}

/* one perturbation step of Alg. 2 for every variable (the four cases);
 * flag (may be NULL) marks variables of rows the decoded point violated.
 * scale 0: r ~ U[-delta, delta] as the listing samples it, so r*delta reaches
 * delta^2; scale 1: r ~ U[-1, 1], so every step is at most delta. */
void or_perturb(OSolver *s, int round, double delta, double tau, unsigned long long seed,
                const unsigned char *flag, int scale)
{
#pragma omp parallel for num_threads(s->nthreads) schedule(static)
    for (long long i = 0; i < s->n_vars; ++i) {
        if (s->deg[i] == 0) continue;
        double r = 2.0 * or_rng_u01(seed, (unsigned long long)round, (unsigned long long)i) - 1.0;
        if (scale == 0) r = r * delta;
        int pos = 1, neg = 1, zero = 1;
        double sum = 0.0;
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) {
            double m = s->mm[s->vpair[q]];
            pos &= m > tau;
            neg &= m < -tau;
            zero &= fabs(m) <= tau;
            sum += m;
        }
        double pert;
        if (flag && flag[i]) pert = r * delta;
        else if (pos) pert = delta;
        else if (neg) pert = -delta;
        else if (zero) pert = r * delta;
        else {
            double mag = fabs(r) * delta;
            int sg = sum > 0.0 ? 1 : sum < 0.0 ? -1 : (r >= 0.0 ? 1 : -1);
            pert = sg > 0 ? mag : -mag;
        }
        for (long long q = s->vptr[i]; q < s->vptr[i + 1]; ++q) {
            long long p = s->vpair[q];
            s->lam[p] = s->lam[p] + pert;
        }
    }
}

int or_round(OSolver *s, double delta0, double alpha, int reopt_iters, int max_rounds, double tau,
             unsigned long long seed, int scale, unsigned char *x_out, double *ub, int *rounds_out,
             long long *conflict_hist)
{
    size_t np = (size_t)s->np, nv = (size_t)s->n_vars;
    double *lam0 = malloc(sizeof(double) * (np + 1)), *mm0 = malloc(sizeof(double) * (np + 1));
    double *avg0 = malloc(sizeof(double) * (nv + 1));
    memcpy(lam0, s->lam, sizeof(double) * np);
    memcpy(mm0, s->mm, sizeof(double) * np);
    memcpy(avg0, s->avg, sizeof(double) * nv);
    unsigned char *flag = calloc(nv + 1, 1), *x = calloc(nv + 1, 1);

    or_terminate(s);
    or_sweep(s, 0, 0);   /* full min-marginals at fixed multipliers */
    double delta = delta0;
    int rc = OR_NOT_CONVERGED, round;
    for (round = 0;; ++round) {
        long long nconf = count_conflicts(s, tau, flag);
        if (conflict_hist && round <= max_rounds) conflict_hist[round] = nconf;
        if (nconf == 0) {
            for (long long i = 0; i < s->n_vars; ++i) {
                if (s->fixed[i] >= 0) x[i] = (unsigned char)s->fixed[i];
                else if (s->deg[i] == 0) x[i] = s->cost[i] < 0.0;
                else x[i] = s->mm[s->vpair[s->vptr[i]]] < 0.0;
            }
            int bad = 0;
            for (int j = 0; j < s->nb; ++j) {
                if (row_satisfied(s, s->brow[j], x)) continue;
                bad = 1;
                for (int h = 0; h < s->bdd[j].k; ++h) flag[s->bdd[j].var[h]] = 1;
            }
            if (!bad) { rc = OR_OK; break; }
        }
        if (round == max_rounds) break;
        or_perturb(s, round, delta, tau, seed, flag, scale);
        memset(flag, 0, nv);
        delta = delta * alpha;
        for (long long i = 0; i < s->n_vars; ++i) s->avg[i] = 0.0;
        for (long long p = 0; p < s->np; ++p) s->mm[p] = 0.0;
        or_run_dual(s, reopt_iters, NULL);
        or_terminate(s);
        or_sweep(s, 0, 0);
    }
    if (rounds_out) *rounds_out = round;
    if (rc == OR_OK) {
        double u = 0.0;
        for (long long i = 0; i < s->n_vars; ++i) u += x[i] ? s->cost[i] : 0.0;
        if (ub) *ub = u;
        if (x_out) memcpy(x_out, x, nv);
    }
    memcpy(s->lam, lam0, sizeof(double) * np);
    memcpy(s->mm, mm0, sizeof(double) * np);
    memcpy(s->avg, avg0, sizeof(double) * nv);
    free(lam0); free(mm0); free(avg0); free(flag); free(x);
    return rc;
}

/* exact integer check of x against every original row; returns #violated rows */
long long or_count_violated(const OSolver *s, const unsigned char *x)
{
    long long n = 0;
    for (long long r = 0; r < s->n_rows; ++r) n += !row_satisfied(s, r, x);
    return n;
}
