/*
 * lddmm_oracle.c -- plain FP64 CPU oracle for landmark geodesic shooting.
 *
 * TEST INFRASTRUCTURE.  This file is the checker of the GPU library, not part
 * of it.  Only the test-suite, the smoke check and the benchmark's CPU-baseline
 * leg load it; the GPU library never calls, links or includes it, and it
 * shares no code, header, table or constant with the HIP sources.
 *
 * What it computes (paper Sec. 2.1, eqs. 1-3, and Algs. 1-2):
 *
 *   kernel      g_ij = exp(-|q_i - q_j|^2 / (2 sigma^2))         (Sec. 2.1, Alg. 2)
 *   Hamiltonian H(q,p) = 1/2 sum_i sum_j g_ij p_i . p_j          (eq. 1)
 *   flow        dq/dt = dH/dp,  dp/dt = -dH/dq                    (eq. 2)
 *                 Hp_i = dH/dp_i = sum_j g_ij p_j
 *                 Hq_i = dH/dq_i = -c sum_j g_ij (p_i.p_j)(q_i - q_j),  c = 1/sigma^2
 *   integrator  explicit Euler, dt = 1/T, q and p updated simultaneously
 *               from the step-t values (Alg. 1, forward loop); optionally
 *               (an extension: the paper takes Euler steps) the classical
 *               fourth-order Runge-Kutta step of the same field f = (Hp, -Hq):
 *                 k1 = f(y), k2 = f(y + h/2 k1), k3 = f(y + h/2 k2),
 *                 k4 = f(y + h k3),  y' = y + h/6 (k1 + 2 k2 + 2 k3 + k4)
 *   objective   L(p0) = H(q0,p0) + lambda sum_i |q_i(1) - x_i|^2   (eq. 3)
 *   gradient    exact adjoint of the discrete Euler map, run backwards in
 *               time (Alg. 1, backward loop); dL/dp0 = b(0) + Hp(q0,p0),
 *               and also dL/dq0 = a(0) + Hq(q0,p0), dL/dx = -2 lambda (q(1)-x).
 *               For the Runge-Kutta step, the exact adjoint of its four
 *               stage equations (reverse-mode differentiation, see below)
 *   optimiser   L-BFGS on p0 (Sec. 2.1 and Alg. 1, steps (e)-(f)), own
 *               implementation: two-loop recursion + strong-Wolfe search
 *   velocity    v(x,t) = sum_l g(|q_l(t) - x|) p_l(t) at any point x (eq. 4),
 *               with the Hamiltonian's Gaussian; the flow of points moves
 *               them by the same explicit Euler steps as the landmarks,
 *               x(t+1) = x(t) + dt v(x(t), t) with the step-t landmark state
 *
 * Readings of passages that the extracted text garbles (eq. 1 loses the 1/2
 * and a bracket, the kernel loses its sign and the 2 sigma^2, eq. 3 says
 * argmax, Alg. 1 starts from q0/T and returns the adjoint without the
 * energy term) follow the definitions above; the build's design notes list
 * each one.
 *
 * The adjoint.  With Delta_ij = q_i - q_j, s_ij = p_i.p_j, adjoint variables
 * a = dL/dq(t+1), b = dL/dp(t+1), db_ij = b_i - b_j, e_ij = Delta_ij . db_ij
 * and pi_ij = a_i.p_j + p_i.a_j, the transpose of the Jacobian of one Euler
 * step gives a(t) = a + dt A, b(t) = b + dt B with
 *     A_i = c sum_j g_ij [ s_ij db_ij - (pi_ij + c s_ij e_ij) Delta_ij ]
 *     B_i =   sum_j g_ij [ a_j + c e_ij p_j ]
 * (A = H_qp a - H_qq b and B = H_pp a - H_pq b, the Hessian blocks of H).
 * This is derived, not printed: the paper names StepBackward but gives no
 * formula for it.  (A, B) = J(y)^T (a, b), J the Jacobian of f at y = (q, p).
 *
 * The Runge-Kutta adjoint.  With stage states Y1 = y, Y2 = y + h/2 k1,
 * Y3 = y + h/2 k2, Y4 = y + h k3 and lambda' = dL/dy', differentiating the
 * stage equations in reverse gives
 *     w4 = J(Y4)^T (h/6 lambda')
 *     w3 = J(Y3)^T (h/3 lambda' + h w4)
 *     w2 = J(Y2)^T (h/3 lambda' + h/2 w3)
 *     w1 = J(Y1)^T (h/6 lambda' + h/2 w2)
 *     lambda = dL/dy = lambda' + w1 + w2 + w3 + w4.
 * The oracle recomputes the stage states from the stored state of the step.
 *
 * Every sum over j runs in index order 0..N-1 including j = i; rows are
 * split over threads, which does not change any row's order of summation,
 * so results do not depend on the thread count.  With compensated = 1 each
 * sum uses Neumaier's compensated summation instead of a plain running sum.
 *
 * Layout: every point set is [N,3] row-major FP64.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* threads over rows                                                        */
/* ------------------------------------------------------------------------ */

static int g_threads = 1;

void oracle_set_threads(int k) { g_threads = k < 1 ? 1 : (k > 512 ? 512 : k); }
int oracle_get_threads(void) { return g_threads; }

typedef void (*row_fn)(void *ctx, int i0, int i1);
typedef struct { row_fn fn; void *ctx; int i0, i1; } row_job;

static void *row_thread(void *v) {
    row_job *j = (row_job *)v;
    j->fn(j->ctx, j->i0, j->i1);
    return NULL;
}

static void for_rows(int n, row_fn fn, void *ctx) {
    int k = g_threads < n ? g_threads : n;
    if (k <= 1) { fn(ctx, 0, n); return; }
    pthread_t th[512];
    row_job jobs[512];
    for (int t = 0; t < k; ++t) {
        jobs[t].fn = fn; jobs[t].ctx = ctx;
        jobs[t].i0 = (int)((int64_t)n * t / k);
        jobs[t].i1 = (int)((int64_t)n * (t + 1) / k);
        if (t == 0) continue;
        if (pthread_create(&th[t], NULL, row_thread, &jobs[t]) != 0) {
            row_thread(&jobs[t]);          /* no thread available: run inline */
            jobs[t].fn = NULL;
        }
    }
    row_thread(&jobs[0]);
    for (int t = 1; t < k; ++t)
        if (jobs[t].fn) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------ */
/* sums                                                                     */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } acc_t;   /* running sum (+ Neumaier term) */

static inline void acc_add(acc_t *a, double x, int comp) {
    if (!comp) { a->s += x; return; }
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static inline double acc_get(const acc_t *a) { return a->s + a->c; }

static inline double gauss(const double *qi, const double *qj, double sigma) {
    double dx = qi[0] - qj[0], dy = qi[1] - qj[1], dz = qi[2] - qj[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    return exp(-r2 / (2.0 * sigma * sigma));
}

/* ------------------------------------------------------------------------ */
/* one step's pair sums: the forward field (Hq, Hp)                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, comp; double sigma;
    const double *q, *p;
    double *Hq, *Hp;
} fwd_ctx;

/* row i of the forward sums, written to hq[0..2], hp[0..2] */
static void fwd_row(const fwd_ctx *k, int i, double *hq_out, double *hp_out) {
    const double c = 1.0 / (k->sigma * k->sigma);
    const double *qi = k->q + 3 * i, *pi = k->p + 3 * i;
    acc_t hp[3] = {{0, 0}, {0, 0}, {0, 0}}, hq[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int j = 0; j < k->n; ++j) {
        const double *qj = k->q + 3 * j, *pj = k->p + 3 * j;
        double g = gauss(qi, qj, k->sigma);
        double s = pi[0] * pj[0] + pi[1] * pj[1] + pi[2] * pj[2];
        for (int d = 0; d < 3; ++d) {
            acc_add(&hp[d], g * pj[d], k->comp);
            acc_add(&hq[d], g * s * (qi[d] - qj[d]), k->comp);
        }
    }
    for (int d = 0; d < 3; ++d) {
        hp_out[d] = acc_get(&hp[d]);
        hq_out[d] = -c * acc_get(&hq[d]);
    }
}

static void fwd_rows(void *v, int i0, int i1) {
    fwd_ctx *k = (fwd_ctx *)v;
    for (int i = i0; i < i1; ++i) fwd_row(k, i, k->Hq + 3 * i, k->Hp + 3 * i);
}

void oracle_pair_forward(int n, double sigma, const double *q, const double *p,
                         double *Hq, double *Hp, int compensated) {
    fwd_ctx k = {n, compensated, sigma, q, p, Hq, Hp};
    for_rows(n, fwd_rows, &k);
}

/* The same sums for a listed subset of rows only (all j), for checking
 * sampled outputs of problems too large for the full O(N^2) oracle.
 * Outputs are [nrows][3]. */
void oracle_pair_forward_rows(int n, double sigma, const double *q, const double *p,
                              const int *rows, int nrows, double *Hq, double *Hp) {
    fwd_ctx k = {n, 0, sigma, q, p, NULL, NULL};
    for (int r = 0; r < nrows; ++r) fwd_row(&k, rows[r], Hq + 3 * r, Hp + 3 * r);
}

/* H(q,p) = 1/2 sum_ij g_ij p_i.p_j  (eq. 1), summed row by row */
typedef struct { int n, comp; double sigma; const double *q, *p; double *row; } ham_ctx;

static void ham_rows(void *v, int i0, int i1) {
    ham_ctx *k = (ham_ctx *)v;
    for (int i = i0; i < i1; ++i) {
        const double *qi = k->q + 3 * i, *pi = k->p + 3 * i;
        acc_t r = {0, 0};
        for (int j = 0; j < k->n; ++j) {
            const double *pj = k->p + 3 * j;
            acc_add(&r, gauss(qi, k->q + 3 * j, k->sigma) *
                            (pi[0] * pj[0] + pi[1] * pj[1] + pi[2] * pj[2]), k->comp);
        }
        k->row[i] = acc_get(&r);
    }
}

double oracle_hamiltonian(int n, double sigma, const double *q, const double *p, int compensated) {
    double *row = (double *)malloc(sizeof(double) * (size_t)n);
    if (!row) return NAN;
    ham_ctx k = {n, compensated, sigma, q, p, row};
    for_rows(n, ham_rows, &k);
    acc_t h = {0, 0};
    for (int i = 0; i < n; ++i) acc_add(&h, row[i], compensated);
    free(row);
    return 0.5 * acc_get(&h);
}

/* ------------------------------------------------------------------------ */
/* one step's adjoint pair sums (A, B)                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, comp; double sigma;
    const double *q, *p, *a, *b;
    double *A, *B;
} adj_ctx;

/* row i of the adjoint sums, written to A_out[0..2], B_out[0..2] */
static void adj_row(const adj_ctx *k, int i, double *A_out, double *B_out) {
    const double c = 1.0 / (k->sigma * k->sigma);
    const double *qi = k->q + 3 * i, *pi = k->p + 3 * i;
    const double *ai = k->a + 3 * i, *bi = k->b + 3 * i;
    acc_t sa[3] = {{0, 0}, {0, 0}, {0, 0}}, sb[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int j = 0; j < k->n; ++j) {
        const double *qj = k->q + 3 * j, *pj = k->p + 3 * j;
        const double *aj = k->a + 3 * j, *bj = k->b + 3 * j;
        double g = gauss(qi, qj, k->sigma);
        double D[3], db[3];
        for (int d = 0; d < 3; ++d) { D[d] = qi[d] - qj[d]; db[d] = bi[d] - bj[d]; }
        double s = pi[0] * pj[0] + pi[1] * pj[1] + pi[2] * pj[2];
        double e = D[0] * db[0] + D[1] * db[1] + D[2] * db[2];
        double pij = ai[0] * pj[0] + ai[1] * pj[1] + ai[2] * pj[2]
                   + pi[0] * aj[0] + pi[1] * aj[1] + pi[2] * aj[2];
        for (int d = 0; d < 3; ++d) {
            acc_add(&sa[d], g * (s * db[d] - (pij + c * s * e) * D[d]), k->comp);
            acc_add(&sb[d], g * (aj[d] + c * e * pj[d]), k->comp);
        }
    }
    for (int d = 0; d < 3; ++d) {
        A_out[d] = c * acc_get(&sa[d]);
        B_out[d] = acc_get(&sb[d]);
    }
}

static void adj_rows(void *v, int i0, int i1) {
    adj_ctx *k = (adj_ctx *)v;
    for (int i = i0; i < i1; ++i) adj_row(k, i, k->A + 3 * i, k->B + 3 * i);
}

void oracle_pair_adjoint(int n, double sigma, const double *q, const double *p,
                         const double *a, const double *b, double *A, double *B, int compensated) {
    adj_ctx k = {n, compensated, sigma, q, p, a, b, A, B};
    for_rows(n, adj_rows, &k);
}

void oracle_pair_adjoint_rows(int n, double sigma, const double *q, const double *p,
                              const double *a, const double *b, const int *rows, int nrows,
                              double *A, double *B) {
    adj_ctx k = {n, 0, sigma, q, p, a, b, NULL, NULL};
    for (int r = 0; r < nrows; ++r) adj_row(&k, rows[r], A + 3 * r, B + 3 * r);
}

/* ------------------------------------------------------------------------ */
/* forward shooting (Alg. 1, forward loop)                                  */
/* ------------------------------------------------------------------------ */

/* The four stages of one Runge-Kutta step from (q, p): stage states
 * Ys[s] = [q (3N), p (3N)] and their fields (Hq, Hp) in Hqs[s], Hps[s]
 * (k_s = (Hp, -Hq) at Ys[s]).  Buffers are 3N (states 6N) each. */
static void rk4_stages(int n, double sigma, double h, const double *q, const double *p,
                       double *Ys[4], double *Hqs[4], double *Hps[4], int compensated) {
    size_t m = 3 * (size_t)n;
    const double c[4] = {0.0, 0.5 * h, 0.5 * h, h};   /* Y_s = y + c_s k_{s-1} */
    for (int st = 0; st < 4; ++st) {
        double *Yq = Ys[st], *Yp = Ys[st] + m;
        for (size_t k = 0; k < m; ++k) {
            if (st == 0) { Yq[k] = q[k]; Yp[k] = p[k]; }
            else {
                Yq[k] = q[k] + c[st] * Hps[st - 1][k];
                Yp[k] = p[k] - c[st] * Hqs[st - 1][k];
            }
        }
        oracle_pair_forward(n, sigma, Yq, Yp, Hqs[st], Hps[st], compensated);
    }
}

/* Scratch of 4 stage states and 4 fields for the Runge-Kutta step. */
typedef struct { double *Y[4], *Hq[4], *Hp[4]; } rk4_buf;

static int rk4_alloc(rk4_buf *b, int n) {
    size_t m = 3 * (size_t)n;
    int ok = 1;
    for (int st = 0; st < 4; ++st) {
        b->Y[st] = (double *)malloc(sizeof(double) * 2 * m);
        b->Hq[st] = (double *)malloc(sizeof(double) * m);
        b->Hp[st] = (double *)malloc(sizeof(double) * m);
        ok = ok && b->Y[st] && b->Hq[st] && b->Hp[st];
    }
    return ok;
}

static void rk4_free(rk4_buf *b) {
    for (int st = 0; st < 4; ++st) { free(b->Y[st]); free(b->Hq[st]); free(b->Hp[st]); }
}

/* traj (optional): (T+1) slots of [q (3N), p (3N)]; slot t = state at step t.
 * Hp0 (optional): Hp(q0,p0), 3N.  Returns 0, or -2 when memory runs out. */
static int shoot_forward_impl(int n, int T, double sigma, const double *q0, const double *p0,
                              double *q1, double *p1, double *H0, double *traj, double *Hp0,
                              double *Hq0, int compensated, int rk4) {
    size_t m = 3 * (size_t)n;
    double *q = (double *)malloc(sizeof(double) * m), *p = (double *)malloc(sizeof(double) * m);
    double *Hq = (double *)malloc(sizeof(double) * m), *Hp = (double *)malloc(sizeof(double) * m);
    rk4_buf rb;
    memset(&rb, 0, sizeof rb);
    if (!q || !p || !Hq || !Hp || (rk4 && !rk4_alloc(&rb, n))) {
        free(q); free(p); free(Hq); free(Hp); rk4_free(&rb);
        return -2;
    }
    memcpy(q, q0, sizeof(double) * m);
    memcpy(p, p0, sizeof(double) * m);
    const double dt = 1.0 / T;
    for (int t = 0; t < T; ++t) {
        if (traj) {
            memcpy(traj + (size_t)t * 2 * m, q, sizeof(double) * m);
            memcpy(traj + (size_t)t * 2 * m + m, p, sizeof(double) * m);
        }
        if (rk4) {
            rk4_stages(n, sigma, dt, q, p, rb.Y, rb.Hq, rb.Hp, compensated);
            memcpy(Hq, rb.Hq[0], sizeof(double) * m);   /* the field at the step's state */
            memcpy(Hp, rb.Hp[0], sizeof(double) * m);
        } else {
            oracle_pair_forward(n, sigma, q, p, Hq, Hp, compensated);
        }
        if (t == 0) {
            if (Hp0) memcpy(Hp0, Hp, sizeof(double) * m);
            if (Hq0) memcpy(Hq0, Hq, sizeof(double) * m);
            if (H0) {   /* H(q0,p0) = 1/2 sum_i p0_i . Hp_i(q0,p0) */
                acc_t h = {0, 0};
                for (size_t k = 0; k < m; ++k) acc_add(&h, p[k] * Hp[k], compensated);
                *H0 = 0.5 * acc_get(&h);
            }
        }
        if (rk4) {
            for (size_t k = 0; k < m; ++k) {   /* y' = y + h/6 (k1 + 2 k2 + 2 k3 + k4) */
                q[k] = q[k] + dt / 6.0 * (rb.Hp[0][k] + 2.0 * rb.Hp[1][k] + 2.0 * rb.Hp[2][k]
                                          + rb.Hp[3][k]);
                p[k] = p[k] - dt / 6.0 * (rb.Hq[0][k] + 2.0 * rb.Hq[1][k] + 2.0 * rb.Hq[2][k]
                                          + rb.Hq[3][k]);
            }
        } else {
            for (size_t k = 0; k < m; ++k) {   /* simultaneous Euler update */
                q[k] = q[k] + dt * Hp[k];
                p[k] = p[k] - dt * Hq[k];
            }
        }
    }
    rk4_free(&rb);
    if (traj) {
        memcpy(traj + (size_t)T * 2 * m, q, sizeof(double) * m);
        memcpy(traj + (size_t)T * 2 * m + m, p, sizeof(double) * m);
    }
    if (q1) memcpy(q1, q, sizeof(double) * m);
    if (p1) memcpy(p1, p, sizeof(double) * m);
    free(q); free(p); free(Hq); free(Hp);
    return 0;
}

/* integrator: 0 explicit Euler, 1 classical Runge-Kutta (fourth order) */
int oracle_shoot_forward(int n, int T, double sigma, const double *q0, const double *p0,
                         double *q1, double *p1, double *H0, double *traj, double *Hp0,
                         int compensated, int integrator) {
    return shoot_forward_impl(n, T, sigma, q0, p0, q1, p1, H0, traj, Hp0, NULL, compensated,
                              integrator == 1);
}

/* ------------------------------------------------------------------------ */
/* the velocity field at arbitrary points and their flow (eq. 4)            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n, comp; double sigma;
    const double *q, *p, *x;
    double *v;
} vel_ctx;

/* v(x_i) = sum_l g(|q_l - x_i|) p_l, landmarks in index order */
static void vel_rows(void *v, int i0, int i1) {
    vel_ctx *k = (vel_ctx *)v;
    for (int i = i0; i < i1; ++i) {
        const double *xi = k->x + 3 * i;
        acc_t s[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int l = 0; l < k->n; ++l) {
            const double *pl = k->p + 3 * l;
            double g = gauss(k->q + 3 * l, xi, k->sigma);
            for (int d = 0; d < 3; ++d) acc_add(&s[d], g * pl[d], k->comp);
        }
        for (int d = 0; d < 3; ++d) k->v[3 * i + d] = acc_get(&s[d]);
    }
}

/* Velocity of eq. 4 at m points x [m,3] for the landmark state (q, p) [n,3]. */
void oracle_velocity(int n, int m, double sigma, const double *q, const double *p,
                     const double *x, double *v, int compensated) {
    vel_ctx k = {n, compensated, sigma, q, p, x, v};
    for_rows(m, vel_rows, &k);
}

/* Flow of m points x0 [m,3] along the landmark motion from (q0, p0): at each
 * of the T steps the points take the velocity of the landmark state at step
 * t, and landmarks and points are then updated together.  x1 [m,3] receives
 * the points at t = 1; q1 (optional) the landmarks.  Returns 0 or -2.
 * integrator 1: the Runge-Kutta step of the joint system (landmarks and
 * points), each point stage taking the velocity of the landmark stage state. */
int oracle_flow(int n, int T, double sigma, const double *q0, const double *p0, int m,
                const double *x0, double *x1, double *q1, int compensated, int integrator) {
    if (integrator == 1) {
        size_t nn = 3 * (size_t)n, mm = 3 * (size_t)m;
        double *q = (double *)malloc(sizeof(double) * nn), *p = (double *)malloc(sizeof(double) * nn);
        double *x = (double *)malloc(sizeof(double) * (mm ? mm : 1));
        double *X = (double *)malloc(sizeof(double) * (mm ? mm : 1));
        double *v[4];
        rk4_buf rb;
        memset(&rb, 0, sizeof rb);
        int ok = q && p && x && X && rk4_alloc(&rb, n);
        for (int st = 0; st < 4; ++st) {
            v[st] = (double *)malloc(sizeof(double) * (mm ? mm : 1));
            ok = ok && v[st];
        }
        if (!ok) {
            free(q); free(p); free(x); free(X); rk4_free(&rb);
            for (int st = 0; st < 4; ++st) free(v[st]);
            return -2;
        }
        memcpy(q, q0, sizeof(double) * nn);
        memcpy(p, p0, sizeof(double) * nn);
        if (mm) memcpy(x, x0, sizeof(double) * mm);
        const double h = 1.0 / T, c[4] = {0.0, 0.5 / T, 0.5 / T, 1.0 / T};
        for (int t = 0; t < T; ++t) {
            rk4_stages(n, sigma, h, q, p, rb.Y, rb.Hq, rb.Hp, compensated);
            for (int st = 0; st < 4; ++st) {   /* X_s = x + c_s v_{s-1} */
                for (size_t k = 0; k < mm; ++k) X[k] = st == 0 ? x[k] : x[k] + c[st] * v[st - 1][k];
                oracle_velocity(n, m, sigma, rb.Y[st], rb.Y[st] + nn, X, v[st], compensated);
            }
            for (size_t k = 0; k < nn; ++k) {
                q[k] = q[k] + h / 6.0 * (rb.Hp[0][k] + 2.0 * rb.Hp[1][k] + 2.0 * rb.Hp[2][k]
                                         + rb.Hp[3][k]);
                p[k] = p[k] - h / 6.0 * (rb.Hq[0][k] + 2.0 * rb.Hq[1][k] + 2.0 * rb.Hq[2][k]
                                         + rb.Hq[3][k]);
            }
            for (size_t k = 0; k < mm; ++k)
                x[k] = x[k] + h / 6.0 * (v[0][k] + 2.0 * v[1][k] + 2.0 * v[2][k] + v[3][k]);
        }
        if (mm) memcpy(x1, x, sizeof(double) * mm);
        if (q1) memcpy(q1, q, sizeof(double) * nn);
        free(q); free(p); free(x); free(X); rk4_free(&rb);
        for (int st = 0; st < 4; ++st) free(v[st]);
        return 0;
    }
    size_t nn = 3 * (size_t)n, mm = 3 * (size_t)m;
    double *q = (double *)malloc(sizeof(double) * nn), *p = (double *)malloc(sizeof(double) * nn);
    double *Hq = (double *)malloc(sizeof(double) * nn), *Hp = (double *)malloc(sizeof(double) * nn);
    double *x = (double *)malloc(sizeof(double) * (mm ? mm : 1));
    double *v = (double *)malloc(sizeof(double) * (mm ? mm : 1));
    if (!q || !p || !Hq || !Hp || !x || !v) {
        free(q); free(p); free(Hq); free(Hp); free(x); free(v);
        return -2;
    }
    memcpy(q, q0, sizeof(double) * nn);
    memcpy(p, p0, sizeof(double) * nn);
    if (mm) memcpy(x, x0, sizeof(double) * mm);
    const double dt = 1.0 / T;
    for (int t = 0; t < T; ++t) {
        oracle_pair_forward(n, sigma, q, p, Hq, Hp, compensated);
        oracle_velocity(n, m, sigma, q, p, x, v, compensated);
        for (size_t k = 0; k < nn; ++k) {
            q[k] = q[k] + dt * Hp[k];
            p[k] = p[k] - dt * Hq[k];
        }
        for (size_t k = 0; k < mm; ++k) x[k] = x[k] + dt * v[k];
    }
    if (mm) memcpy(x1, x, sizeof(double) * mm);
    if (q1) memcpy(q1, q, sizeof(double) * nn);
    free(q); free(p); free(Hq); free(Hp); free(x); free(v);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* loss and gradient (Alg. 1 ComputeGradient, eq. 3)                        */
/* ------------------------------------------------------------------------ */

/* Loss and its gradients.  terms (optional): [energy term, mismatch sum
 * |q1-x|^2]; q1 (optional): q(1).  grad_q0, grad_x (optional): dL/dq0 =
 * a(0) + Hq(q0,p0) (the adjoint of q at t = 0 plus the energy term's own
 * dependence on q0) and dL/dx = -2 lambda (q(1) - x).
 *
 * energy_final = 0: the energy term is H(q0,p0) (eq. 3).  energy_final = 1:
 * it is H(q(1),p(1)), the energy as Alg. 1 evaluates it after the forward
 * loop (equal to H(q0,p0) in continuous time, where H is conserved).  Then
 * the terminal adjoint picks up dH/dq(1) = Hq(q(1),p(1)) and dH/dp(1) =
 * Hp(q(1),p(1)), and the gradients are the adjoint at t = 0 alone. */
int oracle_shoot_grad_all(int n, int T, double sigma, double lambda, const double *q0,
                          const double *p0, const double *x, double *loss, double *grad,
                          double *grad_q0, double *grad_x, double *q1, double *terms,
                          int compensated, int energy_final, int integrator) {
    const int rk4 = integrator == 1;
    size_t m = 3 * (size_t)n;
    double *traj = (double *)malloc(sizeof(double) * (size_t)(T + 1) * 2 * m);
    double *Hp0 = (double *)malloc(sizeof(double) * m), *Hq0 = (double *)malloc(sizeof(double) * m);
    double *a = (double *)malloc(sizeof(double) * m), *b = (double *)malloc(sizeof(double) * m);
    double *A = (double *)malloc(sizeof(double) * m), *B = (double *)malloc(sizeof(double) * m);
    double *HqT = (double *)malloc(sizeof(double) * m), *HpT = (double *)malloc(sizeof(double) * m);
    double *ua = (double *)malloc(sizeof(double) * m), *ub = (double *)malloc(sizeof(double) * m);
    double *la = (double *)malloc(sizeof(double) * m), *lb = (double *)malloc(sizeof(double) * m);
    rk4_buf rb;
    memset(&rb, 0, sizeof rb);
    if (!traj || !Hp0 || !Hq0 || !a || !b || !A || !B || !HqT || !HpT || !ua || !ub || !la ||
        !lb || (rk4 && !rk4_alloc(&rb, n))) {
        free(traj); free(Hp0); free(Hq0); free(a); free(b); free(A); free(B);
        free(HqT); free(HpT); free(ua); free(ub); free(la); free(lb); rk4_free(&rb);
        return -2;
    }
    double E = 0.0;
    shoot_forward_impl(n, T, sigma, q0, p0, NULL, NULL, &E, traj, Hp0, Hq0, compensated, rk4);
    const double *qT = traj + (size_t)T * 2 * m, *pT = qT + m;
    if (energy_final) {   /* H(q(1),p(1)) = 1/2 sum_i p_i(1) . Hp_i(q(1),p(1)) */
        oracle_pair_forward(n, sigma, qT, pT, HqT, HpT, compensated);
        acc_t h = {0, 0};
        for (size_t k = 0; k < m; ++k) acc_add(&h, pT[k] * HpT[k], compensated);
        E = 0.5 * acc_get(&h);
    }
    acc_t mis = {0, 0};
    for (size_t k = 0; k < m; ++k) {
        double r = qT[k] - x[k];
        acc_add(&mis, r * r, compensated);
        a[k] = 2.0 * lambda * r;    /* dL/dq(1) */
        b[k] = 0.0;                 /* dL/dp(1) */
        if (energy_final) { a[k] += HqT[k]; b[k] = HpT[k]; }
        if (grad_x) grad_x[k] = -2.0 * lambda * r;
    }
    double mismatch = acc_get(&mis);
    if (loss) *loss = E + lambda * mismatch;
    if (terms) { terms[0] = E; terms[1] = mismatch; }
    if (q1) memcpy(q1, qT, sizeof(double) * m);
    const double dt = 1.0 / T;
    for (int t = T - 1; t >= 0; --t) {
        const double *qt = traj + (size_t)t * 2 * m, *pt = qt + m;
        if (!rk4) {
            oracle_pair_adjoint(n, sigma, qt, pt, a, b, A, B, compensated);
            for (size_t k = 0; k < m; ++k) {   /* simultaneous update */
                a[k] = a[k] + dt * A[k];
                b[k] = b[k] + dt * B[k];
            }
            continue;
        }
        /* Runge-Kutta step: (a, b) = lambda' on entry; stage adjoints from the
         * last stage to the first, accumulated into (la, lb) */
        rk4_stages(n, sigma, dt, qt, pt, rb.Y, rb.Hq, rb.Hp, compensated);
        const double wl[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};   /* weight of lambda' */
        const double wn[4] = {0.5 * dt, 0.5 * dt, dt, 0.0};             /* of w_{s+1} */
        memcpy(la, a, sizeof(double) * m);
        memcpy(lb, b, sizeof(double) * m);
        for (int st = 3; st >= 0; --st) {
            for (size_t k = 0; k < m; ++k) {   /* u_s = wl_s lambda' + wn_s w_{s+1} */
                ua[k] = wl[st] * a[k] + (st < 3 ? wn[st] * A[k] : 0.0);
                ub[k] = wl[st] * b[k] + (st < 3 ? wn[st] * B[k] : 0.0);
            }
            oracle_pair_adjoint(n, sigma, rb.Y[st], rb.Y[st] + m, ua, ub, A, B, compensated);
            for (size_t k = 0; k < m; ++k) { la[k] += A[k]; lb[k] += B[k]; }   /* w_s */
        }
        memcpy(a, la, sizeof(double) * m);
        memcpy(b, lb, sizeof(double) * m);
    }
    rk4_free(&rb);
    free(ua); free(ub); free(la); free(lb);
    if (grad)
        for (size_t k = 0; k < m; ++k) grad[k] = b[k] + (energy_final ? 0.0 : Hp0[k]);
    if (grad_q0)
        for (size_t k = 0; k < m; ++k) grad_q0[k] = a[k] + (energy_final ? 0.0 : Hq0[k]);
    free(traj); free(Hp0); free(Hq0); free(a); free(b); free(A); free(B); free(HqT); free(HpT);
    return 0;
}

int oracle_shoot_grad(int n, int T, double sigma, double lambda, const double *q0,
                      const double *p0, const double *x, double *loss, double *grad,
                      double *q1, double *terms, int compensated) {
    return oracle_shoot_grad_all(n, T, sigma, lambda, q0, p0, x, loss, grad, NULL, NULL, q1,
                                 terms, compensated, 0, 0);
}

/* ------------------------------------------------------------------------ */
/* L-BFGS with a strong-Wolfe line search (Alg. 1, steps (e)-(f))           */
/* ------------------------------------------------------------------------ */

typedef struct {
    int max_iter, m, max_fev;
    double gtol, ftol_rel, c1, c2;
    int init;           /* 0: p0 = 0, 1: p0 = (x - q0)/T, 2: caller's p0 */
} oracle_opts;

typedef struct {
    double loss, H0, mismatch, grad_norm, avg_dist, max_dist;
    int iters, fevals, status;   /* status: 0 converged, 1 not converged, -4 non-finite */
} oracle_result;

typedef struct {
    int n, T, comp; double sigma, lambda;
    const double *q0, *x;
    int fevals;
} objective;

static double dot(size_t m, const double *u, const double *v) {
    double s = 0.0;
    for (size_t k = 0; k < m; ++k) s += u[k] * v[k];
    return s;
}

static double eval_obj(objective *o, const double *p, double *g) {
    double f = 0.0;
    o->fevals++;
    if (oracle_shoot_grad(o->n, o->T, o->sigma, o->lambda, o->q0, p, o->x, &f, g, NULL, NULL,
                          o->comp) != 0)
        return NAN;
    return f;
}

/* Minimiser of the cubic through (a0,f0,d0), (a1,f1,d1) (Nocedal & Wright,
 * Numerical Optimization, eq. 3.59), kept inside the middle 80 % of the
 * bracket; midpoint when the cubic has no usable minimiser. */
static double cubic_step(double a0, double f0, double d0, double a1, double f1, double d1) {
    double lo = a0 < a1 ? a0 : a1, hi = a0 < a1 ? a1 : a0, w = hi - lo;
    double mid = 0.5 * (a0 + a1);
    double t1 = d0 + d1 - 3.0 * (f0 - f1) / (a0 - a1);
    double disc = t1 * t1 - d0 * d1;
    if (!(disc >= 0.0)) return mid;
    double t2 = sqrt(disc);
    if (a1 < a0) t2 = -t2;
    double den = d1 - d0 + 2.0 * t2;
    double a = a1 - (a1 - a0) * ((d1 + t2 - t1) / den);
    if (!isfinite(a) || a < lo + 0.1 * w || a > hi - 0.1 * w) return mid;
    return a;
}

/* The same step, exported for the tests that pin it against closed-form
 * minimisers of cubics and its fallback branches. */
double oracle_cubic_step(double a0, double f0, double d0, double a1, double f1, double d1) {
    return cubic_step(a0, f0, d0, a1, f1, d1);
}

/* Strong-Wolfe line search along d from x (f, g given), N&W Algs. 3.5/3.6.
 * On success writes the accepted point to xn, fn, gn and returns 1. */
static int line_search(objective *o, size_t m, const double *x, double f, const double *g,
                       const double *d, double a_init, const oracle_opts *op,
                       double *xn, double *fn, double *gn) {
    const double d0 = dot(m, g, d);
    int fev = 0;
    double a_prev = 0.0, f_prev = f, dp_prev = d0;
    double a = a_init;
    double a_lo = 0, f_lo = 0, dp_lo = 0, a_hi = 0, f_hi = 0, dp_hi = 0;
    for (int i = 1;; ++i) {
        if (fev >= op->max_fev) return 0;
        for (size_t k = 0; k < m; ++k) xn[k] = x[k] + a * d[k];
        double fa = eval_obj(o, xn, gn); ++fev;
        double da = dot(m, gn, d);
        if (!isfinite(fa) || !isfinite(da) || fa > f + op->c1 * a * d0 || (i > 1 && fa >= f_prev)) {
            a_lo = a_prev; f_lo = f_prev; dp_lo = dp_prev;
            a_hi = a; f_hi = fa; dp_hi = da;
            break;
        }
        if (fabs(da) <= -op->c2 * d0) { *fn = fa; return 1; }
        if (da >= 0.0) {
            a_lo = a; f_lo = fa; dp_lo = da;
            a_hi = a_prev; f_hi = f_prev; dp_hi = dp_prev;
            break;
        }
        a_prev = a; f_prev = fa; dp_prev = da;
        a = 2.0 * a;                       /* expand the step */
    }
    /* zoom between a_lo (best point satisfying sufficient decrease) and a_hi */
    for (;;) {
        if (fev >= op->max_fev) return 0;
        if (fabs(a_hi - a_lo) <= 1e-14 * fabs(a_lo) + 1e-300) return 0;
        double aj;
        if (isfinite(f_hi) && isfinite(dp_hi))
            aj = cubic_step(a_lo, f_lo, dp_lo, a_hi, f_hi, dp_hi);
        else
            aj = 0.5 * (a_lo + a_hi);
        for (size_t k = 0; k < m; ++k) xn[k] = x[k] + aj * d[k];
        double fj = eval_obj(o, xn, gn); ++fev;
        double dj = dot(m, gn, d);
        if (!isfinite(fj) || !isfinite(dj) || fj > f + op->c1 * aj * d0 || fj >= f_lo) {
            a_hi = aj; f_hi = fj; dp_hi = dj;
        } else {
            if (fabs(dj) <= -op->c2 * d0) { *fn = fj; return 1; }
            if (dj * (a_hi - a_lo) >= 0.0) { a_hi = a_lo; f_hi = f_lo; dp_hi = dp_lo; }
            a_lo = aj; f_lo = fj; dp_lo = dj;
        }
    }
}

/* trace (optional): per accepted iteration k (0 = start), loss and |g|,
 * 2*(max_iter+1) doubles. */
int oracle_solve(int n, int T, double sigma, double lambda, const double *q0, const double *x,
                 double *p0, const oracle_opts *op, oracle_result *res, double *trace,
                 int compensated) {
    size_t m = 3 * (size_t)n;
    int M = op->m < 1 ? 1 : op->m;
    double *buf = (double *)calloc((size_t)(6 + 2 * M) * m + 2 * (size_t)M, sizeof(double));
    if (!buf) return -2;
    double *xk = buf, *g = xk + m, *d = g + m, *xn = d + m, *gn = xn + m, *tmp = gn + m;
    double *S = tmp + m, *Y = S + (size_t)M * m, *rho = Y + (size_t)M * m, *alpha = rho + M;
    objective o = {n, T, compensated, sigma, lambda, q0, x, 0};

    if (op->init == 0) memset(xk, 0, sizeof(double) * m);
    else if (op->init == 1) for (size_t k = 0; k < m; ++k) xk[k] = (x[k] - q0[k]) / T;
    else memcpy(xk, p0, sizeof(double) * m);

    double f = eval_obj(&o, xk, g);
    int status = 1, iters = 0, used = 0, newest = -1;
    double gnorm = sqrt(dot(m, g, g));
    if (trace) { trace[0] = f; trace[1] = gnorm; }
    if (!isfinite(f) || !isfinite(gnorm)) status = -4;
    else if (gnorm <= op->gtol * fmax(1.0, sqrt(dot(m, xk, xk)))) status = 0;

    while (status == 1 && iters < op->max_iter) {
        /* search direction: d = -H g by the two-loop recursion */
        memcpy(d, g, sizeof(double) * m);
        for (int h = 0; h < used; ++h) {           /* newest to oldest */
            int s = (newest - h + M) % M;
            alpha[s] = rho[s] * dot(m, S + (size_t)s * m, d);
            for (size_t k = 0; k < m; ++k) d[k] -= alpha[s] * Y[(size_t)s * m + k];
        }
        if (used > 0) {
            const double *sn = S + (size_t)newest * m, *yn = Y + (size_t)newest * m;
            double gamma = dot(m, sn, yn) / dot(m, yn, yn);
            for (size_t k = 0; k < m; ++k) d[k] *= gamma;
        }
        for (int h = used - 1; h >= 0; --h) {      /* oldest to newest */
            int s = (newest - h + M) % M;
            double beta = rho[s] * dot(m, Y + (size_t)s * m, d);
            for (size_t k = 0; k < m; ++k) d[k] += (alpha[s] - beta) * S[(size_t)s * m + k];
        }
        for (size_t k = 0; k < m; ++k) d[k] = -d[k];
        if (!(dot(m, g, d) < 0.0)) {                /* not a descent direction: restart */
            used = 0; newest = -1;
            for (size_t k = 0; k < m; ++k) d[k] = -g[k];
        }
        double a0 = used == 0 ? 1.0 / sqrt(dot(m, d, d)) : 1.0;
        double fn = 0.0;
        if (!line_search(&o, m, xk, f, g, d, a0, op, xn, &fn, gn)) { status = 1; break; }
        /* curvature pair */
        int slot = (newest + 1) % M;
        double sy = 0.0, yy = 0.0;
        for (size_t k = 0; k < m; ++k) {
            double sk = xn[k] - xk[k], yk = gn[k] - g[k];
            S[(size_t)slot * m + k] = sk;
            Y[(size_t)slot * m + k] = yk;
            sy += sk * yk; yy += yk * yk;
        }
        if (sy > 1e-16 * yy && sy > 0.0) {
            rho[slot] = 1.0 / sy;
            newest = slot;
            if (used < M) ++used;
        }
        double f_old = f;
        memcpy(xk, xn, sizeof(double) * m);
        memcpy(g, gn, sizeof(double) * m);
        f = fn;
        ++iters;
        gnorm = sqrt(dot(m, g, g));
        if (trace) { trace[2 * iters] = f; trace[2 * iters + 1] = gnorm; }
        if (gnorm <= op->gtol * fmax(1.0, sqrt(dot(m, xk, xk)))) { status = 0; break; }
        if (op->ftol_rel > 0.0 &&
            f_old - f <= op->ftol_rel * fmax(fmax(fabs(f_old), fabs(f)), 1.0)) { status = 0; break; }
    }
    memcpy(p0, xk, sizeof(double) * m);
    if (res) {
        double terms[2] = {0, 0};
        double *q1 = tmp;
        oracle_shoot_grad(n, T, sigma, lambda, q0, xk, x, &res->loss, gn, q1, terms, compensated);
        res->H0 = terms[0];
        res->mismatch = terms[1];
        res->grad_norm = gnorm;
        double sum = 0.0, mx = 0.0;
        for (int i = 0; i < n; ++i) {      /* AverageDist / MaxDist (Sec. 3.1) */
            double dx = q1[3 * i] - x[3 * i], dy = q1[3 * i + 1] - x[3 * i + 1],
                   dz = q1[3 * i + 2] - x[3 * i + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            sum += r;
            if (r > mx) mx = r;
        }
        res->avg_dist = sum / n;
        res->max_dist = mx;
        res->iters = iters;
        res->fevals = o.fevals;
        res->status = status;
    }
    free(buf);
    return status;
}
