/*
 * isnmf_oracle.c -- FP64 CPU oracle for online Itakura-Saito NMF
 * (Lefevre, Bach, Fevotte, "Online algorithms for Nonnegative Matrix
 * Factorization with the Itakura-Saito divergence", arXiv:1106.4198).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only through
 * the seeded synthetic inputs.
 *
 * Plain loops in double precision, index order, no blocking or reordering.
 * The only parallelism is an optional OpenMP split over independent frames
 * (inner loop) and over independent rows f (statistics); every sum is taken
 * in index order inside one thread, so results do not depend on the thread
 * count.
 *
 * Layout: column-major everywhere.  V is F x n (frame n at V + n*ldv),
 * W, A, B are F x K (element (f,k) at f + k*ld), H is K x n.
 *
 * Readings of points the paper leaves open (all stated once more in the
 * design notes of the repository):
 *  - h update: the majorize-minimize multiplicative update with exponent 1/2
 *    (section 2.1 asks for "similar updates" that keep descent; 1/2 is the
 *    IS exponent of that update);
 *  - fresh restart starts from h = 1 (section 2.3, fresh or warm restarts);
 *  - forgetting multiplies the PAST statistics: A <- rho*A + sum a
 *    (section 2.3, scaling past data; identical to Algorithm 1 at rho = 1);
 *  - column rescaling uses the L1 sum s_k = sum_f W_fk (Algorithm 1);
 *  - 0/0 guards: when a denominator is zero the old value is kept and the
 *    event is counted in the returned flag count;
 *  - penalty on H (section 2.2, Extensions): psi(s) = lambda log(a + s) of
 *    the column sum, entering the h update through its tangent.
 *
 * Parity pins: see tests/test_oracle_pins.py.  Every function below is
 * pinned there by a closed form, an invariant or a stated property of the
 * paper; none is marked "parity unpinned".
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

static int g_threads = 1;

/* Number of OpenMP threads used by the frame/row parallel loops (>= 1). */
void isnmf_ref_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

int isnmf_ref_get_threads(void) { return g_threads; }

/*
 * One Itakura-Saito term  y/x - log(y/x) - 1  (section 2.1, definition of
 * d_IS).  Written as u - 1 - log u with u = y/x.  Near u = 1 the difference
 * cancels, so for |u - 1| < 0.1 the Taylor series of  d - log(1 + d)
 * (d = u - 1) is summed instead: d^2/2 - d^3/3 + d^4/4 - ... up to d^24
 * (truncation below 1e-22 relative).
 */
double isnmf_ref_dis_term(double y, double x)
{
    double u = y / x;
    double d = u - 1.0;
    if (fabs(d) < 0.1) {
        /* sum_{j=2}^{24} (-1)^j d^j / j, Horner form */
        double s = 0.0;
        for (int j = 24; j >= 2; --j) {
            double c = ((j & 1) ? -1.0 : 1.0) / (double)j;
            s = s * d + c;
        }
        return s * d * d;
    }
    return d - log(u);
}

/* d_IS(eps + y, eps + x) summed over n entries (section 2.1 and the
 * small-amplitude remedy of section 2.3). */
double isnmf_ref_dis(const double *y, const double *x, long n, double eps)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i)
        s += isnmf_ref_dis_term(eps + y[i], eps + x[i]);
    return s;
}

/*
 * Objective of eq. (1) with the eps shift of section 2.3:
 *   (1/N) sum_n sum_f d_IS(eps + V_fn, eps + (W H)_fn).
 */
double isnmf_ref_objective(int F, int K, int N,
                           const double *V, long ldv,
                           const double *W, long ldw,
                           const double *H, long ldh, double eps)
{
    double total = 0.0;
    for (int n = 0; n < N; ++n) {
        for (int f = 0; f < F; ++f) {
            double wh = 0.0;
            for (int k = 0; k < K; ++k)
                wh += W[IX(f, k, ldw)] * H[IX(k, n, ldh)];
            total += isnmf_ref_dis_term(eps + V[IX(f, n, ldv)], eps + wh);
        }
    }
    return N > 0 ? total / (double)N : 0.0;
}

/*
 * Fit one activation vector h (length K) to one frame v (length F) against a
 * fixed dictionary W: the inner argmin of Algorithm 1, truncated to `iters`
 * multiplicative updates (section 2.3, fresh or warm restarts).  One update:
 *   x_f   = eps + sum_k W_fk h_k
 *   num_k = sum_f W_fk (eps + v_f) / x_f^2
 *   den_k = sum_f W_fk / x_f
 *   h_k  <- h_k * sqrt(num_k / den_k)
 * h holds the starting point on entry and the result on exit.  x (length
 * F + K) is scratch.  Returns the number of guarded 0/0 events.
 */
int isnmf_ref_fit_h(int F, int K, const double *v, const double *W, long ldw,
                    double *h, int iters, double eps, double *x)
{
    int flags = 0;
    for (int it = 0; it < iters; ++it) {
        for (int f = 0; f < F; ++f) {
            double s = eps;
            for (int k = 0; k < K; ++k)
                s += W[IX(f, k, ldw)] * h[k];
            x[f] = s;
        }
        /* all num/den use the same h (simultaneous update) */
        for (int k = 0; k < K; ++k) {
            double num = 0.0, den = 0.0;
            for (int f = 0; f < F; ++f) {
                double wf = W[IX(f, k, ldw)];
                num += wf * (eps + v[f]) / (x[f] * x[f]);
                den += wf / x[f];
            }
            /* store the factor; apply after all k are computed */
            if (den > 0.0 && num >= 0.0)
                x[F + k] = sqrt(num / den);
            else {
                x[F + k] = 1.0;
                ++flags;
            }
        }
        for (int k = 0; k < K; ++k)
            h[k] *= x[F + k];
    }
    return flags;
}

/*
 * One online step on a minibatch of b frames (Algorithm 1 with beta = b;
 * the recursion of eq. (4) in the mini-batch form of section 2.3):
 *
 *  1. for every frame n: h_n <- inner fit (fresh: from 1; warm: from H[:,n])
 *  2. with x = eps + W h_n:
 *        a_fk = (eps + v_f) / x_f^2 * h_k * W_fk^2
 *        b_fk = h_k / x_f
 *     summed over the minibatch into dA, dB; the frame losses
 *     sum_f d_IS(eps + v_f, x_f) are added to *loss_sum (eq. (5) numerator)
 *  3. A <- rho*A + dA,  B <- rho*B + dB      (scaling past data)
 *  4. if update_w:  W_fk <- sqrt(A_fk / B_fk)
 *  5. if normalize: s_k = sum_f W_fk; W /= s, A /= s, B *= s, and for warm
 *     restarts H[k,:] *= s so that W H is unchanged (rescaling W)
 *  6. *dw_norm = || W_new - W_old ||_F       (stopping test of Algorithm 1)
 *
 * W is overwritten in place.  H (K x b, ldh) receives the fitted
 * activations; with warm != 0 it also supplies the starting point.
 * Returns the number of guarded 0/0 events (0 in normal operation).
 */
int isnmf_ref_online_step(int F, int K, int b,
                          const double *V, long ldv,
                          double *W, long ldw,
                          double *A, double *B,
                          double *H, long ldh,
                          int iters, double eps, double rho,
                          int normalize, int warm, int update_w,
                          double *loss_sum, double *dw_norm)
{
    int flags = 0;
    double *Wold = (double *)malloc(sizeof(double) * (size_t)F * K);
    double *dA = (double *)calloc((size_t)F * K, sizeof(double));
    double *dB = (double *)calloc((size_t)F * K, sizeof(double));
    double *X = (double *)malloc(sizeof(double) * (size_t)F * (b > 0 ? b : 1));
    double *floss = (double *)calloc((size_t)(b > 0 ? b : 1), sizeof(double));
    int *fflags = (int *)calloc((size_t)(b > 0 ? b : 1), sizeof(int));
    if (!Wold || !dA || !dB || !X || !floss || !fflags) {
        free(Wold); free(dA); free(dB); free(X); free(floss); free(fflags);
        return -1;
    }
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < F; ++f)
            Wold[IX(f, k, F)] = W[IX(f, k, ldw)];

    /* 1-2a: frames are independent given W */
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int n = 0; n < b; ++n) {
        double *h = H + (size_t)n * ldh;
        double *scratch = (double *)malloc(sizeof(double) * (size_t)(F + K));
        const double *v = V + (size_t)n * ldv;
        if (!warm)
            for (int k = 0; k < K; ++k)
                h[k] = 1.0;
        fflags[n] = isnmf_ref_fit_h(F, K, v, W, ldw, h, iters, eps, scratch);
        double l = 0.0;
        for (int f = 0; f < F; ++f) {
            double s = eps;
            for (int k = 0; k < K; ++k)
                s += W[IX(f, k, ldw)] * h[k];
            X[IX(f, n, F)] = s;
            l += isnmf_ref_dis_term(eps + v[f], s);
        }
        floss[n] = l;
        free(scratch);
    }
    for (int n = 0; n < b; ++n) {
        flags += fflags[n];
        if (loss_sum)
            *loss_sum += floss[n];
    }

    /* 2b: a and b summed over the minibatch, in frame order per entry */
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int f = 0; f < F; ++f) {
        for (int n = 0; n < b; ++n) {
            double x = X[IX(f, n, F)];
            double r2 = (eps + V[IX(f, n, ldv)]) / (x * x);
            double r1 = 1.0 / x;
            for (int k = 0; k < K; ++k) {
                double hk = H[IX(k, n, ldh)];
                double w = W[IX(f, k, ldw)];
                dA[IX(f, k, F)] += r2 * hk * w * w;
                dB[IX(f, k, F)] += hk * r1;
            }
        }
    }

    /* 3: fold with the past scaled by rho */
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < F; ++f) {
            A[IX(f, k, F)] = rho * A[IX(f, k, F)] + dA[IX(f, k, F)];
            B[IX(f, k, F)] = rho * B[IX(f, k, F)] + dB[IX(f, k, F)];
        }

    if (update_w) {
        /* 4: dictionary update */
        for (int k = 0; k < K; ++k)
            for (int f = 0; f < F; ++f) {
                double a = A[IX(f, k, F)], bb = B[IX(f, k, F)];
                if (bb > 0.0 && a >= 0.0)
                    W[IX(f, k, ldw)] = sqrt(a / bb);
                else
                    ++flags;
            }
        /* 5: L1 column rescaling */
        if (normalize) {
            for (int k = 0; k < K; ++k) {
                double s = 0.0;
                for (int f = 0; f < F; ++f)
                    s += W[IX(f, k, ldw)];
                if (!(s > 0.0)) {
                    ++flags;
                    continue;
                }
                for (int f = 0; f < F; ++f) {
                    W[IX(f, k, ldw)] /= s;
                    A[IX(f, k, F)] /= s;
                    B[IX(f, k, F)] *= s;
                }
                if (warm)
                    for (int n = 0; n < b; ++n)
                        H[IX(k, n, ldh)] *= s;
            }
        }
    }

    /* 6: change of the dictionary */
    if (dw_norm) {
        double s = 0.0;
        for (int k = 0; k < K; ++k)
            for (int f = 0; f < F; ++f) {
                double d = W[IX(f, k, ldw)] - Wold[IX(f, k, F)];
                s += d * d;
            }
        *dw_norm = sqrt(s);
    }
    free(Wold); free(dA); free(dB); free(X); free(floss); free(fflags);
    return flags;
}

/*
 * Closed-form statistics of eq. (3) at a fixed (W, H), with the eps shift:
 *   X    = eps + W H
 *   A_fk = sum_n H_kn (eps + V_fn) X_fn^-2 W_fk^2
 *   B_fk = sum_n H_kn X_fn^-1
 * A, B are F x K with leading dimension F.
 */
void isnmf_ref_batch_stats(int F, int K, int N,
                           const double *V, long ldv,
                           const double *W, long ldw,
                           const double *H, long ldh, double eps,
                           double *A, double *B)
{
#pragma omp parallel for schedule(static) num_threads(g_threads)
    for (int f = 0; f < F; ++f) {
        for (int k = 0; k < K; ++k) {
            A[IX(f, k, F)] = 0.0;
            B[IX(f, k, F)] = 0.0;
        }
        for (int n = 0; n < N; ++n) {
            double x = eps;
            for (int k = 0; k < K; ++k)
                x += W[IX(f, k, ldw)] * H[IX(k, n, ldh)];
            double v = eps + V[IX(f, n, ldv)];
            for (int k = 0; k < K; ++k) {
                double w = W[IX(f, k, ldw)];
                A[IX(f, k, F)] += H[IX(k, n, ldh)] * v / (x * x) * w * w;
                B[IX(f, k, F)] += H[IX(k, n, ldh)] / x;
            }
        }
    }
}

/*
 * One cycle of batch IS-NMF by multiplicative updates (section 2.1: all of
 * H is updated, the auxiliary function of eq. (2) is recomputed, then W):
 *   1. H_kn <- H_kn sqrt( sum_f W_fk (eps+V_fn) X_fn^-2 / sum_f W_fk X_fn^-1 )
 *      with X = eps + W H from the current H (all columns at once)
 *   2. A, B by eq. (3) at (W, H_new);  W <- sqrt(A / B)
 *   3. if normalize: s_k = sum_f W_fk; W /= s; H[k,:] *= s
 *   4. *obj = objective of eq. (1) at (W_new, H_new)
 * Written independently of the online step (matrix form over all N
 * columns), so that the equivalence of section 2.3 (beta = N, r = 0) can
 * be tested between the two.  Returns the guarded 0/0 count.
 */
int isnmf_ref_batch_cycle(int F, int K, int N,
                          const double *V, long ldv,
                          double *W, long ldw,
                          double *H, long ldh,
                          double eps, int normalize, double *obj)
{
    int flags = 0;
    double *X = (double *)malloc(sizeof(double) * (size_t)F * (N > 0 ? N : 1));
    double *A = (double *)malloc(sizeof(double) * (size_t)F * K);
    double *B = (double *)malloc(sizeof(double) * (size_t)F * K);
    double *G = (double *)malloc(sizeof(double) * (size_t)K * (N > 0 ? N : 1));
    if (!X || !A || !B || !G) {
        free(X); free(A); free(B); free(G);
        return -1;
    }
    /* X = eps + W H */
    for (int n = 0; n < N; ++n)
        for (int f = 0; f < F; ++f) {
            double s = eps;
            for (int k = 0; k < K; ++k)
                s += W[IX(f, k, ldw)] * H[IX(k, n, ldh)];
            X[IX(f, n, F)] = s;
        }
    /* multiplicative factors for all of H, from the same X */
    for (int n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k) {
            double num = 0.0, den = 0.0;
            for (int f = 0; f < F; ++f) {
                double x = X[IX(f, n, F)];
                num += W[IX(f, k, ldw)] * (eps + V[IX(f, n, ldv)]) / (x * x);
                den += W[IX(f, k, ldw)] / x;
            }
            if (den > 0.0 && num >= 0.0)
                G[IX(k, n, K)] = sqrt(num / den);
            else {
                G[IX(k, n, K)] = 1.0;
                ++flags;
            }
        }
    for (int n = 0; n < N; ++n)
        for (int k = 0; k < K; ++k)
            H[IX(k, n, ldh)] *= G[IX(k, n, K)];

    isnmf_ref_batch_stats(F, K, N, V, ldv, W, ldw, H, ldh, eps, A, B);
    for (int k = 0; k < K; ++k)
        for (int f = 0; f < F; ++f) {
            double a = A[IX(f, k, F)], bb = B[IX(f, k, F)];
            if (bb > 0.0 && a >= 0.0)
                W[IX(f, k, ldw)] = sqrt(a / bb);
            else
                ++flags;
        }
    if (normalize)
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int f = 0; f < F; ++f)
                s += W[IX(f, k, ldw)];
            if (!(s > 0.0)) {
                ++flags;
                continue;
            }
            for (int f = 0; f < F; ++f)
                W[IX(f, k, ldw)] /= s;
            for (int n = 0; n < N; ++n)
                H[IX(k, n, ldh)] *= s;
        }
    if (obj)
        *obj = isnmf_ref_objective(F, K, N, V, ldv, W, ldw, H, ldh, eps);
    free(X); free(A); free(B); free(G);
    return flags;
}

/* ------------------------------------------------------------------------
 * Penalty on H (section 2.2, Extensions): a decomposable penalty
 * Psi(H) = sum_n psi(sum_k H_kn) with psi concave and increasing.  The paper
 * names the family, not a psi; the reading here is the log penalty
 *   psi(s) = lambda * log(a + s),   lambda >= 0, a > 0
 * (lambda = 0 is the plain method).  The inner problem of a frame becomes
 *   min_h  d_IS(eps + v, eps + W h) + psi(sum_k h_k).
 * A concave psi lies below its tangent, so at the current h (s = sum_k h_k)
 *   psi(sum_k h'_k) <= psi(s) + psi'(s) (sum_k h'_k - s),
 * a term linear in h'.  Added to the IS auxiliary function of h (the
 * majorizer behind the update of section 2.1), whose h'_k-part is
 * num_k h_k^2 / h'_k + den_k h'_k, it moves psi'(s) into den_k:
 *   h_k <- h_k * sqrt(num_k / (den_k + psi'(s))),  psi'(s) = lambda / (a + s),
 * still a descent step of the penalized inner objective.
 * ------------------------------------------------------------------------ */

/* The penalized inner objective of one frame:
 *   sum_f d_IS(eps + v_f, eps + (W h)_f) + lambda * log(a + sum_k h_k).  */
double isnmf_ref_pen_objective_h(int F, int K, const double *v, const double *W, long ldw,
                                 const double *h, double eps, double lambda, double a)
{
    double total = 0.0, s = 0.0;
    for (int f = 0; f < F; ++f) {
        double x = eps;
        for (int k = 0; k < K; ++k)
            x += W[IX(f, k, ldw)] * h[k];
        total += isnmf_ref_dis_term(eps + v[f], x);
    }
    for (int k = 0; k < K; ++k)
        s += h[k];
    return total + lambda * log(a + s);
}

/* The penalized inner fit: as isnmf_ref_fit_h with psi'(s) added to every
 * den_k, s the sum of h at the start of the update.  Returns the number of
 * guarded 0/0 events. */
int isnmf_ref_fit_h_pen(int F, int K, const double *v, const double *W, long ldw,
                        double *h, int iters, double eps, double lambda, double a, double *x)
{
    int flags = 0;
    for (int it = 0; it < iters; ++it) {
        double s = 0.0;
        for (int k = 0; k < K; ++k)
            s += h[k];
        const double dpsi = lambda / (a + s);
        for (int f = 0; f < F; ++f) {
            double t = eps;
            for (int k = 0; k < K; ++k)
                t += W[IX(f, k, ldw)] * h[k];
            x[f] = t;
        }
        for (int k = 0; k < K; ++k) {
            double num = 0.0, den = 0.0;
            for (int f = 0; f < F; ++f) {
                double wf = W[IX(f, k, ldw)];
                num += wf * (eps + v[f]) / (x[f] * x[f]);
                den += wf / x[f];
            }
            den += dpsi;
            if (den > 0.0 && num >= 0.0)
                x[F + k] = sqrt(num / den);
            else {
                x[F + k] = 1.0;
                ++flags;
            }
        }
        for (int k = 0; k < K; ++k)
            h[k] *= x[F + k];
    }
    return flags;
}

/*
 * One online step with the penalty on H: isnmf_ref_online_step with the
 * penalized inner fit.  The statistics a, b of eq. (4), the fold, the
 * dictionary update and the rescale are those of Algorithm 1 (the penalty
 * involves H only, so the auxiliary function of W is unchanged); the frame
 * losses added to *loss_sum are the d_IS terms alone.
 */
int isnmf_ref_online_step_pen(int F, int K, int b,
                              const double *V, long ldv,
                              double *W, long ldw,
                              double *A, double *B,
                              double *H, long ldh,
                              int iters, double eps, double rho,
                              int normalize, int warm, int update_w,
                              double lambda, double a_psi,
                              double *loss_sum, double *dw_norm)
{
    /* the fit of every frame first, then the unpenalized step from those h
     * with no further updates (iters = 0, warm) */
    int flags = 0;
    double *Hfit = (double *)malloc(sizeof(double) * (size_t)K * (b > 0 ? b : 1));
    if (!Hfit)
        return -1;
#pragma omp parallel for schedule(static) num_threads(g_threads) reduction(+ : flags)
    for (int n = 0; n < b; ++n) {
        double *h = Hfit + (size_t)n * K;
        double *scratch = (double *)malloc(sizeof(double) * (size_t)(F + K));
        for (int k = 0; k < K; ++k)
            h[k] = warm ? H[IX(k, n, ldh)] : 1.0;
        flags += isnmf_ref_fit_h_pen(F, K, V + (size_t)n * ldv, W, ldw, h, iters, eps, lambda,
                                     a_psi, scratch);
        free(scratch);
    }
    for (int n = 0; n < b; ++n)
        for (int k = 0; k < K; ++k)
            H[IX(k, n, ldh)] = Hfit[IX(k, n, K)];
    /* warm = 1 keeps the fitted h as the starting point of zero updates; the
     * rescale then compensates H, which only warm restarts ask for */
    const int f2 = isnmf_ref_online_step(F, K, b, V, ldv, W, ldw, A, B, H, ldh, 0, eps, rho,
                                         normalize, 1, update_w, loss_sum, dw_norm);
    if (!warm)
        for (int n = 0; n < b; ++n)
            for (int k = 0; k < K; ++k)
                H[IX(k, n, ldh)] = Hfit[IX(k, n, K)];
    free(Hfit);
    if (f2 < 0)
        return f2;
    return flags + f2;
}
