/*
 * CPU oracle for Deep Greedy Switching (DGS) on the Linear Sum Assignment
 * Problem.  TEST INFRASTRUCTURE ONLY: it exists to check the GPU library
 * and is called only from the test suite, the smoke check and the CPU
 * timing leg of the benchmark.  The GPU library never links or calls it,
 * and it shares no code with the GPU library.
 *
 * Plain, slow and obviously correct on purpose.  All arithmetic is int64.
 * The functions follow the paper (Roverso et al., "GPU-Based Heuristic
 * Solver for Linear Sum Assignment Problems Under Real-time Constraints"):
 *
 *   LSAP        Section 3, the maximisation problem over permutations.
 *   sigma/tau   Section 3.3: sigma(j) = agent holding job j, tau(i) = job of
 *               agent i, tau = M(sigma).
 *   switch      Section 3.3: switch(i, j, sigma) gives job j to agent i and
 *               i's old job to the old owner sigma(j) (a 2-exchange).
 *   ADE         Algorithm 2: agent i scans every job j' != tau(i) and keeps
 *               the first strictly better exchange (so the lowest j' wins a
 *               tie); j_i and delta_i of Section 3.3.
 *   JDE         Section 3.2: the job side of Algorithm 2 -- job j scans every
 *               agent i != sigma(j) and keeps the first strictly better one.
 *   Switching   Section 3.3 and Algorithm 1: take the best exchange over all
 *               agents, apply it while it improves f, re-evaluate.
 *   Initial     Section 3.1: a greedy start that takes the benefits into
 *               account.
 *
 * Readings where the paper leaves a choice (the GPU library follows the
 * same readings):
 *   R1  Steepest ascent: after every switch the per-agent bests equal a
 *       fresh ADE of every agent; the switch taken is the global best.
 *   R2  Steepest ascent scans agents only (for a full square assignment JDE
 *       enumerates the same 2-exchanges); JDE is kept for the job side of
 *       Parallel DGS, where its tie-break (lowest agent) picks exchanges
 *       that ADE's (lowest job) does not.
 *   R3  Ties: within an agent the lowest job index; across agents the
 *       lowest agent index.
 *   R4  A switch is applied only if its gain is strictly positive.
 *   R5  Greedy start: agents 0..n-1 in order, each takes its best free job,
 *       lowest job index on ties.
 *   R6  A job with no owner (sigma(j) = -1) is a plain move with gain
 *       a[i][j] - a[i][tau(i)].  It cannot occur for square inputs; it is
 *       kept so the gain definition is complete.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NEG_INF INT64_MIN

/* a_ij, row-major. */
static inline int64_t at(const int32_t *A, int64_t n, int64_t i, int64_t j) {
    return (int64_t)A[i * n + j];
}

/* Threads of the OpenMP loops below (k > 0), for timing the oracle on a
 * given number of cores; returns the count now in effect. */
int32_t orc_set_threads(int32_t k) {
    if (k > 0) omp_set_num_threads(k);
    return (int32_t)omp_get_max_threads();
}

/* f(sigma) = sum_i a[i][tau(i)]  (Section 3, objective). */
int64_t orc_objective(const int32_t *A, int32_t n, const int32_t *tau) {
    int64_t f = 0;
    for (int64_t i = 0; i < n; ++i) f += at(A, n, i, tau[i]);
    return f;
}

/* 1 if tau is a permutation of 0..n-1. */
int32_t orc_is_permutation(const int32_t *tau, int32_t n) {
    char *seen = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int ok = 1;
    for (int32_t i = 0; i < n && ok; ++i) {
        if (tau[i] < 0 || tau[i] >= n || seen[tau[i]]) ok = 0;
        else seen[tau[i]] = 1;
    }
    free(seen);
    return ok;
}

/* Greedy initial assignment (Section 3.1, reading R5). */
void orc_greedy(const int32_t *A, int32_t n, int32_t *tau) {
    char *taken = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t i = 0; i < n; ++i) {
        int64_t best = ORC_NEG_INF;
        int32_t bj = -1;
        for (int64_t j = 0; j < n; ++j) {
            if (taken[j]) continue;
            if (at(A, n, i, j) > best) { best = at(A, n, i, j); bj = (int32_t)j; }
        }
        tau[i] = bj;
        taken[bj] = 1;
    }
    free(taken);
}

/* f(switch(i, j', sigma)) - f(sigma): agent i takes job j', the owner
 * i' = sigma(j') takes i's job j = tau(i).  Only the two changed terms of
 * the objective differ. */
static inline int64_t exchange_gain(const int32_t *A, int64_t n, const int32_t *tau,
                                    const int32_t *sigma, int64_t i, int64_t jp) {
    int64_t j = tau[i];
    int64_t ip = sigma[jp];
    if (ip < 0) return at(A, n, i, jp) - at(A, n, i, j); /* R6 */
    return (at(A, n, i, jp) + at(A, n, ip, j)) - (at(A, n, i, j) + at(A, n, ip, jp));
}

/* ADE for one agent (Algorithm 2): best (gain, job) over j' != tau(i),
 * first strictly better wins.  The best is recorded even when it does not
 * improve (gain <= 0), so the full per-agent result can be compared; the
 * sentinel (ORC_NEG_INF, -1) means agent i has no other job (n = 1). */
static void ade(const int32_t *A, int64_t n, const int32_t *tau, const int32_t *sigma,
                int64_t i, int64_t *g_out, int32_t *j_out) {
    int64_t bg = ORC_NEG_INF;
    int32_t bj = -1;
    for (int64_t jp = 0; jp < n; ++jp) {
        if (jp == tau[i]) continue;
        int64_t g = exchange_gain(A, n, tau, sigma, i, jp);
        if (g > bg) { bg = g; bj = (int32_t)jp; }
    }
    *g_out = bg;
    *j_out = bj;
}

static void invert(const int32_t *tau, int32_t n, int32_t *sigma) {
    for (int32_t j = 0; j < n; ++j) sigma[j] = -1;
    for (int32_t i = 0; i < n; ++i) sigma[tau[i]] = i;
}

/* Difference evaluation of every agent for the assignment tau. */
void orc_scan(const int32_t *A, int32_t n, const int32_t *tau, int64_t *g_out, int32_t *j_out) {
    int32_t *sigma = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    invert(tau, n, sigma);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) ade(A, n, tau, sigma, i, &g_out[i], &j_out[i]);
    free(sigma);
}

/* JDE for one job (Section 3.2, the job side of Algorithm 2): the best
 * agent i != sigma(j) to take job j -- its current owner then takes tau(i),
 * so the gain is exchange_gain(i, j) -- scanning agents in index order and
 * keeping the first strictly better one (lowest agent on ties).  Recorded
 * even when <= 0; (ORC_NEG_INF, -1) when n == 1. */
static void jde(const int32_t *A, int64_t n, const int32_t *tau, const int32_t *sigma,
                int64_t j, int64_t *g_out, int32_t *i_out) {
    int64_t bg = ORC_NEG_INF;
    int32_t bi = -1;
    for (int64_t i = 0; i < n; ++i) {
        if (i == sigma[j]) continue;
        int64_t g = exchange_gain(A, n, tau, sigma, i, j);
        if (g > bg) { bg = g; bi = (int32_t)i; }
    }
    *g_out = bg;
    *i_out = bi;
}

/* Job difference evaluation of every job for the assignment tau. */
void orc_scan_jobs(const int32_t *A, int32_t n, const int32_t *tau, int64_t *g_out, int32_t *i_out) {
    int32_t *sigma = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    invert(tau, n, sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < n; ++j) jde(A, n, tau, sigma, j, &g_out[j], &i_out[j]);
    free(sigma);
}

/* Best switch over all agents: largest gain, lowest agent on ties, and only
 * a strictly positive gain counts (R3, R4).  Returns the agent or -1. */
static int64_t pick(const int64_t *g, int64_t n) {
    int64_t bi = -1, bg = 0;
    for (int64_t i = 0; i < n; ++i)
        if (g[i] > bg) { bg = g[i]; bi = i; }
    return bi;
}

/* switch(i, j, sigma) applied in place to tau and sigma (Section 3.3). */
static void apply_switch(int32_t *tau, int32_t *sigma, int32_t i, int32_t j) {
    int32_t j0 = tau[i];
    int32_t k = sigma[j];
    tau[i] = j;
    sigma[j] = i;
    if (k >= 0) { tau[k] = j0; sigma[j0] = k; }
    else sigma[j0] = -1;
}

/*
 * DGS by definition: after every switch every agent is re-evaluated from
 * scratch (R1).  tau holds the start on entry and the result on exit.
 * max_switches < 0 means no limit (the paper's anytime property, Section 3:
 * stopping early still leaves a full assignment).  Optional trace arrays
 * (capacity trace_cap) receive (agent, job, gain) of every switch taken.
 * Returns the number of switches S; *f_out receives the final objective.
 */
int64_t orc_dgs_full(const int32_t *A, int32_t n, int32_t *tau, int64_t max_switches,
                     int64_t *f_out, int32_t *tr_i, int32_t *tr_j, int64_t *tr_g,
                     int64_t trace_cap) {
    int32_t *sigma = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *jb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t f = orc_objective(A, n, tau);
    int64_t S = 0;
    invert(tau, n, sigma);
    for (;;) {
        if (max_switches >= 0 && S >= max_switches) break;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) ade(A, n, tau, sigma, i, &g[i], &jb[i]);
        int64_t i = pick(g, n);
        if (i < 0) break;
        if (S < trace_cap) { tr_i[S] = (int32_t)i; tr_j[S] = jb[i]; tr_g[S] = g[i]; }
        apply_switch(tau, sigma, (int32_t)i, jb[i]);
        f += g[i];
        ++S;
    }
    *f_out = f;
    free(sigma);
    free(g);
    free(jb);
    return S;
}

/* (g, j) better than (bg, bj): larger gain, lower job on ties. */
static inline int better(int64_t g, int32_t j, int64_t bg, int32_t bj) {
    return g > bg || (g == bg && j < bj);
}

/*
 * DGS with exact incremental re-evaluation (same result as orc_dgs_full,
 * far fewer operations).  After switch(i*, j*) with partner k = old
 * sigma(j*) and j0 = old tau(i*):
 *   - agents i* and k changed jobs, so every exchange they take part in
 *     changed: they are re-evaluated in full (Algorithm 1 re-evaluates the
 *     agents involved in the switch);
 *   - for any other agent r only the exchanges towards jobs j0 and j*
 *     changed (their owners changed); all other gains of r are unchanged.
 *     If r's stored best job is neither j0 nor j*, the new best is the
 *     better of the stored best and the two new candidates.  If it is one
 *     of them, a new candidate strictly above the stored gain is the best
 *     (every other gain is <= the stored one); otherwise r is re-evaluated
 *     in full, since an unchanged job with equal gain and lower index may
 *     exist.
 * Optional counters: *rescans_out = number of full re-evaluations of
 * agents other than i*, k.
 */
int64_t orc_dgs_incr(const int32_t *A, int32_t n, int32_t *tau, int64_t max_switches,
                     int64_t *f_out, int32_t *tr_i, int32_t *tr_j, int64_t *tr_g,
                     int64_t trace_cap, int64_t *rescans_out) {
    int32_t *sigma = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *jb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t f = orc_objective(A, n, tau);
    int64_t S = 0, rescans = 0;
    invert(tau, n, sigma);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) ade(A, n, tau, sigma, i, &g[i], &jb[i]);
    for (;;) {
        if (max_switches >= 0 && S >= max_switches) break;
        int64_t is = pick(g, n);
        if (is < 0) break;
        int32_t js = jb[is];
        int32_t j0 = tau[is];
        int32_t k = sigma[js];
        if (S < trace_cap) { tr_i[S] = (int32_t)is; tr_j[S] = js; tr_g[S] = g[is]; }
        f += g[is];
        apply_switch(tau, sigma, (int32_t)is, js);
        ++S;
        int64_t local_rescans = 0;
#pragma omp parallel for schedule(static) reduction(+ : local_rescans)
        for (int64_t r = 0; r < n; ++r) {
            if (r == is || r == k) {
                ade(A, n, tau, sigma, r, &g[r], &jb[r]);
                continue;
            }
            int64_t ga = ORC_NEG_INF, gb = ORC_NEG_INF;
            int32_t ca = j0, cb = js;
            if (tau[r] != j0) ga = exchange_gain(A, n, tau, sigma, r, j0);
            if (tau[r] != js) gb = exchange_gain(A, n, tau, sigma, r, js);
            /* best of the two new candidates */
            int64_t cg = ga;
            int32_t cj = ca;
            if (better(gb, cb, cg, cj)) { cg = gb; cj = cb; }
            if (jb[r] != j0 && jb[r] != js) {
                if (better(cg, cj, g[r], jb[r])) { g[r] = cg; jb[r] = cj; }
            } else if (cg > g[r]) {
                g[r] = cg;
                jb[r] = cj;
            } else {
                ade(A, n, tau, sigma, r, &g[r], &jb[r]);
                ++local_rescans;
            }
        }
        rescans += local_rescans;
    }
    *f_out = f;
    if (rescans_out) *rescans_out = rescans;
    free(sigma);
    free(g);
    free(jb);
    return S;
}

/* ---- rectangular instances: n agents, m >= n jobs (Section 1: n providers,
 * m receivers).  Row stride m; sigma(j) = -1 for a job nobody holds, and
 * exchange_gain's R6 branch (a move to that job) is live. ---------------- */

/* One entry a_ij of the matrix, for the global greedy start. */
typedef struct {
    int32_t v, i, j;
} orc_entry;

/* Larger entry first; among equal entries the lower agent, then the lower
 * job. */
static int entry_before(const void *x, const void *y) {
    const orc_entry *a = (const orc_entry *)x, *b = (const orc_entry *)y;
    if (a->v != b->v) return a->v > b->v ? -1 : 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    return a->j < b->j ? -1 : (a->j > b->j);
}

/*
 * Global greedy start (the variant of Section 3.1's greedy start that looks
 * at all benefits at once): while an agent is free, the largest entry a_ij
 * whose agent i and job j are both free is taken (the lowest agent, then the
 * lowest job, among equal entries).  Computed by putting every entry in
 * that order once and walking it: the entry the definition takes next is
 * always the first one left whose agent and job are both free, since an
 * entry passed over has a taken agent or job, and taken stays taken.
 * n <= m; tau receives n distinct jobs.
 */
void orc_global_greedy(const int32_t *A, int32_t n, int32_t m, int32_t *tau) {
    const int64_t cnt = (int64_t)n * m;
    orc_entry *e = (orc_entry *)malloc(sizeof(orc_entry) * (size_t)(cnt > 0 ? cnt : 1));
    char *agent_taken = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    char *job_taken = (char *)calloc((size_t)(m > 0 ? m : 1), 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < m; ++j) {
            e[i * m + j].v = A[i * m + j];
            e[i * m + j].i = (int32_t)i;
            e[i * m + j].j = (int32_t)j;
        }
    qsort(e, (size_t)cnt, sizeof(orc_entry), entry_before);
    int32_t left = n;
    for (int64_t x = 0; x < cnt && left > 0; ++x) {
        if (agent_taken[e[x].i] || job_taken[e[x].j]) continue;
        tau[e[x].i] = e[x].j;
        agent_taken[e[x].i] = 1;
        job_taken[e[x].j] = 1;
        --left;
    }
    free(e);
    free(agent_taken);
    free(job_taken);
}

/* ADE of agent i over all m jobs j' != tau(i): exchanges with owned jobs,
 * moves to free ones (R6); first strictly better wins (lowest job on ties). */
static void ade_rect(const int32_t *A, int64_t m, const int32_t *tau, const int32_t *sigma,
                     int64_t i, int64_t *g_out, int32_t *j_out) {
    int64_t bg = ORC_NEG_INF;
    int32_t bj = -1;
    for (int64_t jp = 0; jp < m; ++jp) {
        if (jp == tau[i]) continue;
        int64_t g = exchange_gain(A, m, tau, sigma, i, jp);
        if (g > bg) { bg = g; bj = (int32_t)jp; }
    }
    *g_out = bg;
    *j_out = bj;
}

/*
 * Steepest-ascent DGS on an n x m instance (n <= m) by definition: after
 * every change every agent is re-evaluated from scratch over all m jobs;
 * the best agent (largest gain, lowest agent on ties) is applied while its
 * gain is > 0.  tau: n distinct jobs in [0, m), the start on entry and the
 * result on exit.  Returns S; *f_out receives the final objective.
 */
int64_t orc_rect_dgs(const int32_t *A, int32_t n, int32_t m, int32_t *tau, int64_t max_switches,
                     int64_t *f_out) {
    int32_t *sigma = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *jb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t j = 0; j < m; ++j) sigma[j] = -1;
    for (int32_t i = 0; i < n; ++i) sigma[tau[i]] = i;
    int64_t f = 0, S = 0;
    for (int64_t i = 0; i < n; ++i) f += at(A, m, i, tau[i]);
    for (;;) {
        if (max_switches >= 0 && S >= max_switches) break;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) ade_rect(A, m, tau, sigma, i, &g[i], &jb[i]);
        int64_t i = pick(g, n);
        if (i < 0) break;
        apply_switch(tau, sigma, (int32_t)i, jb[i]);
        f += g[i];
        ++S;
    }
    *f_out = f;
    free(sigma);
    free(g);
    free(jb);
    return S;
}

/*
 * Exact LSAP optimum (maximisation), for the optimality gap.  Shortest
 * augmenting paths with dual potentials (the O(n^3) Hungarian method of
 * Kuhn as refined by Jonker and Volgenant), on costs c_ij = -a_ij.
 * Writes an optimal assignment to tau_out and returns its benefit.
 */
int64_t orc_hungarian(const int32_t *A, int32_t n, int32_t *tau_out) {
    if (n <= 0) return 0;
    const int64_t INF = INT64_MAX / 4;
    int64_t N = n;
    /* 1-based arrays: u (rows), v (cols), p[j] = row matched to col j, way */
    int64_t *u = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *v = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *p = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *way = (int64_t *)calloc((size_t)N + 1, sizeof(int64_t));
    int64_t *minv = (int64_t *)malloc(sizeof(int64_t) * ((size_t)N + 1));
    char *used = (char *)malloc((size_t)N + 1);
    for (int64_t i = 1; i <= N; ++i) {
        p[0] = i;
        int64_t j0 = 0;
        for (int64_t j = 0; j <= N; ++j) { minv[j] = INF; used[j] = 0; }
        do {
            used[j0] = 1;
            int64_t i0 = p[j0], delta = INF, j1 = 0;
            for (int64_t j = 1; j <= N; ++j) {
                if (used[j]) continue;
                int64_t cur = -at(A, N, i0 - 1, j - 1) - u[i0] - v[j];
                if (cur < minv[j]) { minv[j] = cur; way[j] = j0; }
                if (minv[j] < delta) { delta = minv[j]; j1 = j; }
            }
            for (int64_t j = 0; j <= N; ++j) {
                if (used[j]) { u[p[j]] += delta; v[j] -= delta; }
                else minv[j] -= delta;
            }
            j0 = j1;
        } while (p[j0] != 0);
        do {
            int64_t j1 = way[j0];
            p[j0] = p[j1];
            j0 = j1;
        } while (j0);
    }
    for (int64_t j = 1; j <= N; ++j) tau_out[p[j] - 1] = (int32_t)(j - 1);
    int64_t f = orc_objective(A, n, tau_out);
    free(u); free(v); free(p); free(way); free(minv); free(used);
    return f;
}
