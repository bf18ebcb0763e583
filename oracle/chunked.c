/*
 * Sequential chunked Hessian / Hessian-vector product on the CPU (float64).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the CPU oracle's rendering of the
 * paper's method; nothing in the HIP library includes or links it.
 *
 * An hDual<csize> is an array of 2*csize+2 doubles (Sec. III.B, Sec. IV):
 *   v[0]                value
 *   v[1]                d/dx_i                 (i = the Hessian row)
 *   v[2 .. csize+1]     d/dx_{cs+l}            (cs = first column of the chunk)
 *   v[csize+2 .. 2csize+1]  d2/dx_i dx_{cs+l}
 * The operator rules are those of Sec. III.A written out per component
 * (the product rule as in Fig. 1); unary functions follow the chain rule
 * g(u) = <g, g' u_1, g' u_{2+l}, g' u_{c+2+l} + g'' u_1 u_{2+l}>.
 *
 * chunk_init  : CHUNK-INIT (Sec. III.B) - one-hot seeds for row i, chunk cs.
 * chunk_hess  : CHUNK-HESS (Sec. III.B) - n * ceil(n/csize) calls of f.
 * chess_vec   : CHESS-VEC (Sec. VI) - the same calls, each chunk dotted with
 *               the input vector and summed per row; H is never stored.
 * schunk_hess : SCHUNK-HESS (Sec. III.B) - only the chunks that reach the
 *               diagonal or lie right of it are evaluated; the entries left
 *               of a row's own chunk are copied from their mirror images.
 * sc_hess_vec : SC-HESS-VEC (Sec. VI) - the same calls; a computed entry
 *               H(i, s) right of row i's own chunk also adds H(i, s) in[i] to
 *               r(s), in place of the call that would have computed H(s, i).
 * When n is not a multiple of csize the last chunk seeds only columns < n
 * and its surplus components are ignored.
 *
 * Built twice from this source: once plain (timed as the CPU baseline, with
 * OpenMP over independent points) and once with -DCHESSFAD_COUNT_OPS, where
 * every scalar addition and multiplication increments a counter so the
 * operation counts of Sec. V can be checked against the code that runs.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef CHESSFAD_COUNT_OPS
static long g_adds, g_muls;
#define ADD(a, b) (g_adds++, (a) + (b))
#define SUB(a, b) (g_adds++, (a) - (b))
#define MUL(a, b) (g_muls++, (a) * (b))
#else
#define ADD(a, b) ((a) + (b))
#define SUB(a, b) ((a) - (b))
#define MUL(a, b) ((a) * (b))
#endif

enum { ROSENBROCK = 0, ACKLEY = 1, FLETCHER_POWELL = 2 };

typedef struct {
    int n, cs;          /* number of variables, chunk size csize */
    int len;            /* 2*cs + 2 components per hDual */
    const double *A, *B, *E;
} ctx_t;

/* ------------------------------------------------------------ operators */
static void hd_copy(const ctx_t *c, double *r, const double *u) { memcpy(r, u, sizeof(double) * c->len); }

static void hd_add(const ctx_t *c, double *r, const double *u, const double *w) {
    for (int k = 0; k < c->len; k++) r[k] = ADD(u[k], w[k]);
}

static void hd_sub(const ctx_t *c, double *r, const double *u, const double *w) {
    for (int k = 0; k < c->len; k++) r[k] = SUB(u[k], w[k]);
}

/* product rule: value, the csize+1 first derivatives, then the chunk of
 * second derivatives u0 w_h + u1 w_c + w1 u_c + w0 u_h */
static void hd_mul(const ctx_t *c, double *r, const double *u, const double *w) {
    const int cs = c->cs;
    double t[2 * cs + 2];
    t[0] = MUL(u[0], w[0]);
    for (int k = 1; k <= cs + 1; k++) t[k] = ADD(MUL(u[0], w[k]), MUL(w[0], u[k]));
    for (int j = 2; j <= cs + 1; j++)
        t[cs + j] = ADD(ADD(ADD(MUL(u[0], w[cs + j]), MUL(u[1], w[j])), MUL(w[1], u[j])), MUL(w[0], u[cs + j]));
    hd_copy(c, r, t);
}

static void hd_scale(const ctx_t *c, double *r, double s, const double *u) {
    for (int k = 0; k < c->len; k++) r[k] = MUL(s, u[k]);
}

/* s + u touches only the value */
static void hd_add_scalar(const ctx_t *c, double *r, double s, const double *u) {
    hd_copy(c, r, u);
    r[0] = ADD(s, u[0]);
}

/* s - u: the value is a subtraction, the other components change sign */
static void hd_rsub_scalar(const ctx_t *c, double *r, double s, const double *u) {
    r[0] = SUB(s, u[0]);
    for (int k = 1; k < c->len; k++) r[k] = -u[k];
}

/* chain rule with g = g(u0), g1 = g'(u0), g2 = g''(u0) */
static void hd_unary(const ctx_t *c, double *r, const double *u, double g, double g1, double g2) {
    const int cs = c->cs;
    double t[2 * cs + 2];
    t[0] = g;
    for (int k = 1; k <= cs + 1; k++) t[k] = MUL(g1, u[k]);
    double g2u1 = MUL(g2, u[1]);
    for (int l = 0; l < cs; l++) t[cs + 2 + l] = ADD(MUL(g1, u[cs + 2 + l]), MUL(g2u1, u[2 + l]));
    hd_copy(c, r, t);
}

static void hd_sin(const ctx_t *c, double *r, const double *u) { hd_unary(c, r, u, sin(u[0]), cos(u[0]), -sin(u[0])); }
static void hd_cos(const ctx_t *c, double *r, const double *u) { hd_unary(c, r, u, cos(u[0]), -sin(u[0]), -cos(u[0])); }
static void hd_exp(const ctx_t *c, double *r, const double *u) { double e = exp(u[0]); hd_unary(c, r, u, e, e, e); }
static void hd_sqrt(const ctx_t *c, double *r, const double *u) {
    double s = sqrt(u[0]);
    hd_unary(c, r, u, s, 0.5 / s, -0.25 / (s * u[0]));
}

/* ------------------------------------------------------------ functions */
/* sum_{k<n-1} 100 (y_{k+1} - y_k^2)^2 + (1 - y_k)^2 */
static void f_rosenbrock(const ctx_t *c, double *res, double *const *y) {
    const int L = c->len;
    double a[L], b[L], t[L];
    for (int k = 0; k + 1 < c->n; k++) {
        hd_mul(c, a, y[k], y[k]);            /* y_k^2              */
        hd_sub(c, b, y[k + 1], a);           /* y_{k+1} - y_k^2    */
        hd_mul(c, b, b, b);                  /* (.)^2              */
        hd_scale(c, b, 100.0, b);            /* 100 (.)^2          */
        hd_rsub_scalar(c, a, 1.0, y[k]);     /* 1 - y_k            */
        hd_mul(c, a, a, a);                  /* (1 - y_k)^2        */
        hd_add(c, t, b, a);
        if (k == 0) hd_copy(c, res, t); else hd_add(c, res, res, t);
    }
}

/* -20 exp(-0.2 sqrt(sum y^2 / n)) - exp(sum cos(2 pi y) / n) + 20 + e */
static void f_ackley(const ctx_t *c, double *res, double *const *y) {
    const int L = c->len, n = c->n;
    double ss[L], cs[L], t[L], u[L];
    for (int k = 0; k < n; k++) {
        hd_mul(c, t, y[k], y[k]);
        if (k == 0) hd_copy(c, ss, t); else hd_add(c, ss, ss, t);
        hd_scale(c, u, 2.0 * M_PI, y[k]);
        hd_cos(c, u, u);
        if (k == 0) hd_copy(c, cs, u); else hd_add(c, cs, cs, u);
    }
    hd_scale(c, t, 1.0 / n, ss);
    hd_sqrt(c, t, t);                        /* rho               */
    hd_scale(c, t, -0.2, t);
    hd_exp(c, t, t);
    hd_scale(c, t, -20.0, t);                /* -20 exp(-0.2 rho) */
    hd_scale(c, u, 1.0 / n, cs);
    hd_exp(c, u, u);                         /* exp(q)            */
    hd_sub(c, t, t, u);
    hd_add_scalar(c, res, 20.0 + M_E, t);
}

/* sum_m (E_m - sum_j A_mj sin y_j + B_mj cos y_j)^2 */
static void f_fletcher_powell(const ctx_t *c, double *res, double *const *y) {
    const int L = c->len, n = c->n;
    double *sy = malloc(sizeof(double) * (size_t)L * n);
    double *cy = malloc(sizeof(double) * (size_t)L * n);
    double inner[L], t[L];
    for (int j = 0; j < n; j++) {
        hd_sin(c, sy + (size_t)j * L, y[j]);
        hd_cos(c, cy + (size_t)j * L, y[j]);
    }
    for (int m = 0; m < n; m++) {
        for (int j = 0; j < n; j++) {
            hd_scale(c, t, c->A[(size_t)m * n + j], sy + (size_t)j * L);
            if (j == 0) hd_copy(c, inner, t); else hd_add(c, inner, inner, t);
            hd_scale(c, t, c->B[(size_t)m * n + j], cy + (size_t)j * L);
            hd_add(c, inner, inner, t);
        }
        hd_rsub_scalar(c, t, c->E[m], inner);    /* residual r_m */
        hd_mul(c, t, t, t);
        if (m == 0) hd_copy(c, res, t); else hd_add(c, res, res, t);
    }
    free(sy);
    free(cy);
}

#ifdef CHESSFAD_COUNT_OPS
static long g_calls;
#define COUNT_CALL() (g_calls++)
#else
#define COUNT_CALL() ((void)0)
#endif

static void eval_f(int func, const ctx_t *c, double *res, double *const *y) {
    COUNT_CALL();
    if (func == ROSENBROCK) f_rosenbrock(c, res, y);
    else if (func == ACKLEY) f_ackley(c, res, y);
    else f_fletcher_powell(c, res, y);
}

/* ------------------------------------------------------------ the method */
/* CHUNK-INIT: y_k = <a_k, [k = i], [k = cstart + l] (l < csize), 0...> */
static void chunk_init(const ctx_t *c, double *const *y, const double *a, int i, int cstart) {
    for (int k = 0; k < c->n; k++) {
        double *yk = y[k];
        memset(yk, 0, sizeof(double) * c->len);
        yk[0] = a[k];
        if (k == i) yk[1] = 1.0;
        if (k >= cstart && k < cstart + c->cs) yk[k - cstart + 2] = 1.0;
    }
}

typedef struct {
    double *store;
    double **y;
    double *temp;
} scratch_t;

static int scratch_init(scratch_t *s, const ctx_t *c) {
    s->store = malloc(sizeof(double) * (size_t)c->len * (c->n + 1));
    s->y = malloc(sizeof(double *) * c->n);
    if (!s->store || !s->y) return -1;
    for (int k = 0; k < c->n; k++) s->y[k] = s->store + (size_t)k * c->len;
    s->temp = s->store + (size_t)c->n * c->len;
    return 0;
}

static void scratch_free(scratch_t *s) { free(s->store); free(s->y); }

/* CHESS-VEC for one point: out[i] = sum over chunks of sum_l H[i][cs+l] in[cs+l] */
static void chess_vec(int func, const ctx_t *c, scratch_t *s, const double *a, const double *in, double *out) {
    const int n = c->n, cs = c->cs, nchunk = (n + cs - 1) / cs;
    for (int i = 0; i < n; i++) {
        double res = 0.0;
        for (int j = 0; j < nchunk; j++) {
            int cstart = j * cs;
            chunk_init(c, s->y, a, i, cstart);
            eval_f(func, c, s->temp, s->y);
            for (int l = 0; l < cs && cstart + l < n; l++)
                res = ADD(res, MUL(s->temp[cs + 2 + l], in[cstart + l]));
        }
        out[i] = res;
    }
}

/* CHUNK-HESS for one point: H[i][cstart + l] = temp.v[csize + 2 + l] */
static void chunk_hess(int func, const ctx_t *c, scratch_t *s, const double *a, double *H) {
    const int n = c->n, cs = c->cs, nchunk = (n + cs - 1) / cs;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < nchunk; j++) {
            int cstart = j * cs;
            chunk_init(c, s->y, a, i, cstart);
            eval_f(func, c, s->temp, s->y);
            for (int l = 0; l < cs && cstart + l < n; l++) H[(size_t)i * n + cstart + l] = s->temp[cs + 2 + l];
        }
}

/* SC-HESS-VEC for one point.  Row i evaluates its own chunk scn = i / csize
 * and every chunk after it; an entry in a later chunk updates both r(i) and
 * its mirror r(s).  Inside the own chunk every row computes its entries
 * itself, so nothing is added twice.  All csize components of each call are
 * used (the last chunk: those below n). */
static void sc_hess_vec(int func, const ctx_t *c, scratch_t *s, const double *a, const double *in, double *out) {
    const int n = c->n, cs = c->cs, nchunk = (n + cs - 1) / cs;
    for (int k = 0; k < n; k++) out[k] = 0.0;
    for (int i = 0; i < n; i++) {
        const int scn = i / cs;
        for (int cn = scn; cn < nchunk; cn++) {
            const int cstart = cn * cs;
            chunk_init(c, s->y, a, i, cstart);
            eval_f(func, c, s->temp, s->y);
            for (int l = 0; l < cs && cstart + l < n; l++) {
                const int col = cstart + l;
                const double h = s->temp[cs + 2 + l];
                out[i] = ADD(out[i], MUL(h, in[col]));
                if (cn > scn) out[col] = ADD(out[col], MUL(h, in[i]));
            }
        }
    }
}

/* SCHUNK-HESS for one point: the evaluated chunks as in CHUNK-HESS, then for
 * every row i the columns left of its own chunk, j < (i / csize) csize, are
 * copied from H[j][i] (which row j evaluated, since i lies in a later chunk
 * than j). */
static void schunk_hess(int func, const ctx_t *c, scratch_t *s, const double *a, double *H) {
    const int n = c->n, cs = c->cs, nchunk = (n + cs - 1) / cs;
    for (int i = 0; i < n; i++)
        for (int j = i / cs; j < nchunk; j++) {
            int cstart = j * cs;
            chunk_init(c, s->y, a, i, cstart);
            eval_f(func, c, s->temp, s->y);
            for (int l = 0; l < cs && cstart + l < n; l++) H[(size_t)i * n + cstart + l] = s->temp[cs + 2 + l];
        }
    for (int i = cs; i < n; i++) {
        const int endindex = (i / cs) * cs;
        for (int j = 0; j < endindex; j++) H[(size_t)i * n + j] = H[(size_t)j * n + i];
    }
}

static int check(int func, int n, int csize, const double *A, const double *B, const double *E) {
    if (func < 0 || func > 2) return -1;
    if (n < 1 || (func == ROSENBROCK && n < 2)) return -2;
    if (csize < 1) return -3;
    if (func == FLETCHER_POWELL && (!A || !B || !E)) return -5;
    return 0;
}

static int run_hvp(int func, int n, long npts, const double *x, const double *v, double *out, int csize,
                   const double *A, const double *B, const double *E, int nthreads, int sym) {
    int rc = check(func, n, csize, A, B, E);
    if (rc) return rc;
    ctx_t c = {n, csize, 2 * csize + 2, A, B, E};
    int err = 0;
#ifndef CHESSFAD_COUNT_OPS
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : err)
#endif
    {
        scratch_t s;
        if (scratch_init(&s, &c)) err = 1;
        else {
#ifndef CHESSFAD_COUNT_OPS
#pragma omp for schedule(static)
#endif
            for (long p = 0; p < npts; p++)
                (sym ? sc_hess_vec : chess_vec)(func, &c, &s, x + (size_t)p * n, v + (size_t)p * n,
                                                out + (size_t)p * n);
        }
        scratch_free(&s);
    }
    return err ? -8 : 0;
}

static int run_hessian(int func, int n, long npts, const double *x, double *H, int csize,
                       const double *A, const double *B, const double *E, int nthreads, int sym) {
    int rc = check(func, n, csize, A, B, E);
    if (rc) return rc;
    ctx_t c = {n, csize, 2 * csize + 2, A, B, E};
    int err = 0;
#ifndef CHESSFAD_COUNT_OPS
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1) reduction(| : err)
#endif
    {
        scratch_t s;
        if (scratch_init(&s, &c)) err = 1;
        else {
#ifndef CHESSFAD_COUNT_OPS
#pragma omp for schedule(static)
#endif
            for (long p = 0; p < npts; p++)
                (sym ? schunk_hess : chunk_hess)(func, &c, &s, x + (size_t)p * n, H + (size_t)p * n * n);
        }
        scratch_free(&s);
    }
    return err ? -8 : 0;
}

int oracle_hvp(int func, int n, long npts, const double *x, const double *v, double *out, int csize,
               const double *A, const double *B, const double *E, int nthreads) {
    return run_hvp(func, n, npts, x, v, out, csize, A, B, E, nthreads, 0);
}

int oracle_hvp_sym(int func, int n, long npts, const double *x, const double *v, double *out, int csize,
                   const double *A, const double *B, const double *E, int nthreads) {
    return run_hvp(func, n, npts, x, v, out, csize, A, B, E, nthreads, 1);
}

int oracle_hessian(int func, int n, long npts, const double *x, double *H, int csize,
                   const double *A, const double *B, const double *E, int nthreads) {
    return run_hessian(func, n, npts, x, H, csize, A, B, E, nthreads, 0);
}

int oracle_hessian_sym(int func, int n, long npts, const double *x, double *H, int csize,
                       const double *A, const double *B, const double *E, int nthreads) {
    return run_hessian(func, n, npts, x, H, csize, A, B, E, nthreads, 1);
}

/* Gradient and value from the first-order components of row i's calls. */
int oracle_value_grad(int func, int n, const double *x, double *fval, double *grad, int csize,
                      const double *A, const double *B, const double *E) {
    int rc = check(func, n, csize, A, B, E);
    if (rc) return rc;
    ctx_t c = {n, csize, 2 * csize + 2, A, B, E};
    scratch_t s;
    if (scratch_init(&s, &c)) return -8;
    for (int i = 0; i < n; i++) {
        chunk_init(&c, s.y, x, i, 0);
        eval_f(func, &c, s.temp, s.y);
        grad[i] = s.temp[1];
        *fval = s.temp[0];
    }
    scratch_free(&s);
    return 0;
}

#ifdef CHESSFAD_COUNT_OPS
/* Scalar operation counts of one CHESS-VEC (sym = 0) or SC-HESS-VEC (sym = 1)
 * on one point, and the number of f calls it makes; also the counts for
 * single operator applications. */
int oracle_count_hvp(int func, int n, const double *x, const double *v, double *out, int csize,
                     const double *A, const double *B, const double *E, long *adds, long *muls, long *calls,
                     int sym) {
    int rc = check(func, n, csize, A, B, E);
    if (rc) return rc;
    ctx_t c = {n, csize, 2 * csize + 2, A, B, E};
    scratch_t s;
    if (scratch_init(&s, &c)) return -8;
    g_adds = g_muls = g_calls = 0;
    (sym ? sc_hess_vec : chess_vec)(func, &c, &s, x, v, out);
    *adds = g_adds;
    *muls = g_muls;
    *calls = g_calls;
    scratch_free(&s);
    return 0;
}

/* op: 0 = hDual + hDual, 1 = hDual x hDual, 2 = double x hDual, 3 = unary */
int oracle_count_op(int op, int csize, long *adds, long *muls) {
    ctx_t c = {1, csize, 2 * csize + 2, 0, 0, 0};
    double u[2 * csize + 2], w[2 * csize + 2], r[2 * csize + 2];
    for (int k = 0; k < c.len; k++) { u[k] = 1.0 + k; w[k] = 2.0 - k; }
    g_adds = g_muls = 0;
    if (op == 0) hd_add(&c, r, u, w);
    else if (op == 1) hd_mul(&c, r, u, w);
    else if (op == 2) hd_scale(&c, r, 3.0, u);
    else if (op == 3) hd_unary(&c, r, u, 0.5, 0.25, 0.125);
    else return -1;
    *adds = g_adds;
    *muls = g_muls;
    return 0;
}
#endif
