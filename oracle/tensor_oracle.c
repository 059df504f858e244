/*
 * Plain FP64 tensor-propagator recursion for the memory-truncated,
 * discretized Feynman-Vernon path sum.
 *
 * TEST INFRASTRUCTURE ONLY (oracle).  Not part of the product path; shares
 * no code with the HIP library.
 *
 * What it computes (Sec. II, exact path-sum equation with the discretized
 * influence functional and the eta definitions; tensor-propagator scheme of
 * Makri and Makarov named in the Introduction):
 *
 *   rho(t_n)[o_n] = sum_{o_0..o_{n-1}} rho0[o_0] prod_{k<n} K_{k+1}[o_{k+1}, o_k]
 *                   prod_{k<=n} prod_{max(0,k-L) <= k' <= k} F_{eta(k,k';n)}(o_k, o_k')
 *
 * K_{k+1} is the bare propagator over (t_k, t_{k+1}]: the same matrix for
 * every interval when H is constant, one matrix per interval for a driven H(t)
 * (the Hamiltonian of the paper's model carries a time-dependent Rabi
 * frequency, Sec. III); step n uses K_n.
 *
 * Because each influence factor couples points at most L apart, the partial
 * sum over all points older than n-L+1 can be carried as a tensor A over the
 * last min(n, L) points (oldest point's index varies fastest in memory).  Step
 * n multiplies A by every factor that involves the new point n, treating n as
 * an interior point, and, once the window is full (n >= L), sums out the oldest
 * point, which no later factor touches.  rho(t_n) is the same product with the
 * final-point classes, summed over every point but n.
 *
 * Eta classes (see oracle/eta.py):
 *   self_int  interior self pair            self_end  initial or final self pair
 *   lag[D]    interior pair, lag D          init[k]   interior point k with point 0
 *   fin[D]    final with interior, lag D    fin_init[n] final point n with point 0
 * Each array has L+1 complex entries (entry 0 unused), interleaved (re, im).
 *
 * Liouville index o = a*M + b for (s^+ = s[a], s^- = s[b]); K holds n_K
 * matrices of N x N, row-major (K[o' * N + o]), and step n uses matrix
 * min(n, n_K) - 1; rho0 and every output rho are N complex values.
 *
 * Path filtering (oracle_propagate_filtered): see propagate_impl.
 *
 * Reductions: rho sums are accumulated with Neumaier compensation over fixed
 * chunks of output entries and the chunk partials are combined in order, so
 * the result does not depend on the number of threads.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define CHUNK 4096

static cplx ld(const double *ri, size_t k) { return ri[2 * k] + I * ri[2 * k + 1]; }

/* F_eta(o, p) = exp(-(s_a - s_b)(eta s_c - conj(eta) s_d)) */
static cplx influence(const double *s, int M, int o, int p, cplx eta) {
    int a = o / M, b = o % M, c = p / M, d = p % M;
    return cexp(-(s[a] - s[b]) * (eta * s[c] - conj(eta) * s[d]));
}

static void fill_table(const double *s, int M, cplx eta, cplx *T) {
    int N = M * M;
    for (int o = 0; o < N; ++o)
        for (int p = 0; p < N; ++p) T[o * N + p] = influence(s, M, o, p, eta);
}

typedef struct { double sr, cr, si, ci; } nsum;

static void nadd1(double *s, double *c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}
static void nadd(nsum *a, cplx x) { nadd1(&a->sr, &a->cr, creal(x)); nadd1(&a->si, &a->ci, cimag(x)); }
static cplx nval(const nsum *a) { return (a->sr + a->cr) + I * (a->si + a->ci); }

static size_t ipow(size_t b, int e) { size_t r = 1; while (e-- > 0) r *= b; return r; }

static double now_s(void) {
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

/*
 * Path filtering (Sim's on-the-fly filtering, as read here): with theta >= 0,
 * every entry of the augmented tensor whose magnitude is not above theta is
 * dropped (set to zero) as soon as it is formed -- the initial tensor and the
 * tensor after every step -- so the paths it stands for take no further part
 * in the sum.  theta < 0 keeps everything (the plain recursion).  kept
 * (optional): the entries left after step n at index n (n = 0 .. n_steps);
 * margin (optional): the smallest | |A_x| - theta | / theta over every entry
 * formed, i.e. how close any decision came to the threshold.
 */
static int propagate_impl(int M, const double *s, const double *K_ri, int n_K, const double *rho0_ri,
                          int L, int n_steps,
                          const double *eta_self_int, const double *eta_self_end,
                          const double *eta_lag, const double *eta_init,
                          const double *eta_fin, const double *eta_fin_init,
                          double *rho_out, double *step_seconds, int n_threads,
                          double theta, long long *kept, double *margin);

static long long filter_entries(cplx *A, size_t count, double theta, double *margin) {
    long long k = 0;
    for (size_t x = 0; x < count; ++x) {
        const double a = cabs(A[x]);
        if (margin && theta > 0.0) {
            const double d = fabs(a - theta) / theta;
            if (d < *margin) *margin = d;
        }
        if (a <= theta) A[x] = 0;
        else ++k;
    }
    return k;
}

/*
 * Returns 0 on success, 1 on bad arguments, 2 on allocation failure.
 * rho_out: (n_steps + 1) * N complex (interleaved); rho_out[0] = rho0.
 * step_seconds (optional, may be NULL): wall time of each step n = 1..n_steps
 * at index n-1.
 */
int oracle_propagate(int M, const double *s, const double *K_ri, int n_K, const double *rho0_ri,
                     int L, int n_steps,
                     const double *eta_self_int, const double *eta_self_end,
                     const double *eta_lag, const double *eta_init,
                     const double *eta_fin, const double *eta_fin_init,
                     double *rho_out, double *step_seconds, int n_threads) {
    return propagate_impl(M, s, K_ri, n_K, rho0_ri, L, n_steps, eta_self_int, eta_self_end, eta_lag, eta_init,
                          eta_fin, eta_fin_init, rho_out, step_seconds, n_threads, -1.0, NULL, NULL);
}

/* The same recursion with the path filtering above (theta >= 0). */
int oracle_propagate_filtered(int M, const double *s, const double *K_ri, int n_K, const double *rho0_ri,
                              int L, int n_steps,
                              const double *eta_self_int, const double *eta_self_end,
                              const double *eta_lag, const double *eta_init,
                              const double *eta_fin, const double *eta_fin_init,
                              double *rho_out, int n_threads, double theta, long long *kept, double *margin) {
    if (!(theta >= 0.0)) return 1;
    return propagate_impl(M, s, K_ri, n_K, rho0_ri, L, n_steps, eta_self_int, eta_self_end, eta_lag, eta_init,
                          eta_fin, eta_fin_init, rho_out, NULL, n_threads, theta, kept, margin);
}

static int propagate_impl(int M, const double *s, const double *K_ri, int n_K, const double *rho0_ri,
                          int L, int n_steps,
                          const double *eta_self_int, const double *eta_self_end,
                          const double *eta_lag, const double *eta_init,
                          const double *eta_fin, const double *eta_fin_init,
                          double *rho_out, double *step_seconds, int n_threads,
                          double theta, long long *kept, double *margin) {
    if (M < 1 || M > 8 || L < 1 || n_steps < 0 || n_K < 1) return 1;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
    const int N = M * M;
    const size_t NN = (size_t)N * N;

    cplx *K = malloc(sizeof(cplx) * NN * n_K);
    cplx *self_int = malloc(sizeof(cplx) * N), *self_end = malloc(sizeof(cplx) * N);
    cplx *T_lag = malloc(sizeof(cplx) * NN * (L + 1));
    cplx *T_init = malloc(sizeof(cplx) * NN * (L + 1));
    cplx *T_fin = malloc(sizeof(cplx) * NN * (L + 1));
    cplx *T_fin_init = malloc(sizeof(cplx) * NN * (L + 1));
    /* the tensor never holds more than min(L, n_steps + 1) axes */
    const size_t cap = ipow(N, L < n_steps + 1 ? L : n_steps + 1);
    cplx *A = malloc(sizeof(cplx) * cap), *B = malloc(sizeof(cplx) * cap);
    const size_t n_chunks_max = cap / CHUNK + 2;
    nsum *part = malloc(sizeof(nsum) * n_chunks_max * N);
    if (!K || !self_int || !self_end || !T_lag || !T_init || !T_fin || !T_fin_init || !A || !B || !part) {
        free(K); free(self_int); free(self_end); free(T_lag); free(T_init); free(T_fin);
        free(T_fin_init); free(A); free(B); free(part);
        return 2;
    }
    for (size_t k = 0; k < NN * n_K; ++k) K[k] = ld(K_ri, k);
    const cplx e_si = ld(eta_self_int, 0), e_se = ld(eta_self_end, 0);
    for (int o = 0; o < N; ++o) {
        self_int[o] = influence(s, M, o, o, e_si);
        self_end[o] = influence(s, M, o, o, e_se);
    }
    for (int D = 1; D <= L; ++D) {
        fill_table(s, M, ld(eta_lag, D), T_lag + NN * D);
        fill_table(s, M, ld(eta_init, D), T_init + NN * D);
        fill_table(s, M, ld(eta_fin, D), T_fin + NN * D);
        fill_table(s, M, ld(eta_fin_init, D), T_fin_init + NN * D);
    }

    /* rho(t_0) = rho0; A holds point 0 with its initial self factor. */
    for (int o = 0; o < N; ++o) {
        rho_out[2 * o] = rho0_ri[2 * o];
        rho_out[2 * o + 1] = rho0_ri[2 * o + 1];
        A[o] = ld(rho0_ri, o) * self_end[o];
    }
    if (margin) *margin = INFINITY;
    if (theta >= 0.0) {
        const long long k0 = filter_entries(A, (size_t)N, theta, margin);
        if (kept) kept[0] = k0;
    }

    for (int n = 1; n <= n_steps; ++n) {
        double t0 = now_s();
        const int p_lo = n - L > 0 ? n - L : 0;   /* oldest point held in A */
        const int ax = n - p_lo;                   /* axes of A = min(n, L) */
        const int sum_out = (ax == L);             /* oldest leaves the window after this step */
        const size_t in_count = ipow(N, ax);
        const size_t upper_count = in_count / N;   /* points p_lo+1 .. n-1 */
        const size_t out_count = sum_out ? in_count : in_count * N;
        const cplx *Kn = K + NN * (size_t)(n < n_K ? n - 1 : n_K - 1);   /* propagator of step n */
        /* class tables of predecessor point k' for the new point n */
#define T_INT(kp) ((kp) == 0 ? T_init + NN * n : T_lag + NN * (n - (kp)))
#define T_FIN(kp) ((kp) == 0 ? T_fin_init + NN * n : T_fin + NN * (n - (kp)))
        /* Loop over (upper, o_n); the digit-0 point p_lo is handled innermost. */
        const size_t n_outer = upper_count * N;
        const size_t n_chunks = (n_outer + CHUNK - 1) / CHUNK;
        memset(part, 0, sizeof(nsum) * n_chunks * N);
        const cplx *F0 = T_INT(p_lo), *F0f = T_FIN(p_lo);
        #pragma omp parallel for schedule(static)
        for (size_t ch = 0; ch < n_chunks; ++ch) {
            const size_t lo = ch * CHUNK;
            const size_t hi = lo + CHUNK < n_outer ? lo + CHUNK : n_outer;
            for (size_t idx = lo; idx < hi; ++idx) {
                const int on = (int)(idx / upper_count);
                const size_t up = idx % upper_count;
                /* upper points p_lo+1+j, j = 0..ax-2; o_{n-1} is the newest of A */
                cplx P = self_int[on], Pf = self_end[on];
                size_t rem = up;
                int newest = -1;
                for (int j = 0; j < ax - 1; ++j) {
                    const int d = (int)(rem % N);
                    rem /= N;
                    const int kp = p_lo + 1 + j;
                    P *= T_INT(kp)[on * N + d];
                    Pf *= T_FIN(kp)[on * N + d];
                    newest = d;
                }
                if (ax >= 2) {          /* bare propagator from o_{n-1} (an upper point) */
                    P *= Kn[on * N + newest];
                    Pf *= Kn[on * N + newest];
                }
                cplx acc = 0, accf = 0;
                for (int i = 0; i < N; ++i) {
                    const cplx a = A[(size_t)i + (size_t)N * up];
                    cplx f = F0[on * N + i], ff = F0f[on * N + i];
                    if (ax == 1) {      /* o_{n-1} is the digit-0 point itself */
                        f *= Kn[on * N + i];
                        ff *= Kn[on * N + i];
                    }
                    accf += ff * a;
                    if (sum_out) acc += f * a;
                    else B[(size_t)i + (size_t)N * up + in_count * (size_t)on] = P * f * a;
                }
                if (sum_out) B[up + upper_count * (size_t)on] = P * acc;
                nadd(&part[ch * N + on], Pf * accf);
            }
        }
#undef T_INT
#undef T_FIN
        nsum rs[64];
        memset(rs, 0, sizeof(rs));
        for (size_t ch = 0; ch < n_chunks; ++ch)
            for (int o = 0; o < N; ++o) {
                cplx v = nval(&part[ch * N + o]);
                nadd(&rs[o], v);
            }
        for (int o = 0; o < N; ++o) {
            cplx v = nval(&rs[o]);
            rho_out[(size_t)2 * N * n + 2 * o] = creal(v);
            rho_out[(size_t)2 * N * n + 2 * o + 1] = cimag(v);
        }
        if (theta >= 0.0) {
            const long long k = filter_entries(B, out_count, theta, margin);
            if (kept) kept[n] = k;
        }
        cplx *tmp = A; A = B; B = tmp;
        if (step_seconds) step_seconds[n - 1] = now_s() - t0;
    }
    free(K); free(self_int); free(self_end); free(T_lag); free(T_init); free(T_fin);
    free(T_fin_init); free(A); free(B); free(part);
    return 0;
}
