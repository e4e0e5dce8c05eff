/*
 * isnmf.h -- C ABI of the MI355X (gfx950) online Itakura-Saito NMF library.
 *
 * Method: Lefevre, Bach, Fevotte, "Online algorithms for Nonnegative Matrix
 * Factorization with the Itakura-Saito divergence" (arXiv:1106.4198).
 * Problem statement (section 2.1, eq. 1): given V in R+^{F x N}, find
 * W in R+^{F x K} and H in R+^{K x N} minimizing
 *     (1/N) sum_n d_IS(v_n, W h_n),   d_IS(y,x) = sum_i y_i/x_i - log(y_i/x_i) - 1,
 * with the eps shift d_IS(eps + y, eps + x) of section 2.3.
 *
 * Conventions shared by every entry point
 *  - Layout: column-major.  V is F x N with frame n at V + n*ldv (ldv >= F);
 *    W is F x K with column k at W + k*ldw (ldw >= F); H is K x N with
 *    column n at H + n*ldh (ldh >= K); A and B are F x K with leading
 *    dimension exactly F.
 *  - Pointers named d_* (and every matrix argument unless stated otherwise)
 *    are DEVICE pointers on the current HIP device; pointers named host_* are
 *    host pointers.  The caller allocates and owns every buffer, workspaces
 *    included; the library never frees caller memory.  Handles are host
 *    objects created and freed by the library.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    Unless stated otherwise a call only enqueues work on that stream and
 *    returns before it completes.
 *  - Errors: every call returns an isnmf_status.  ISNMF_EINVAL is detected
 *    on the host before any device work is enqueued, and leaves all state
 *    untouched.  Non-finite inputs or state met on the device set a sticky
 *    flag word that isnmf_online_status() reads.  No exception crosses the
 *    ABI.
 *  - Threads: a handle is not thread-safe; use one handle per host thread.
 */
#ifndef ISNMF_H
#define ISNMF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ISNMF_OK = 0,
    ISNMF_EINVAL = -1,       /* bad argument; nothing was enqueued          */
    ISNMF_ENOMEM = -2,       /* workspace too small / host allocation failed */
    ISNMF_EDEVICE = -3,      /* a HIP runtime call failed                   */
    ISNMF_ENONFINITE = -4,   /* device flag: non-finite value met           */
    ISNMF_ESTATE = -5,       /* handle in an unusable state                 */
    ISNMF_EUNSUPPORTED = -6  /* shape/precision combination not built       */
} isnmf_status;

/* Arithmetic of the W.H products (the MFMA contractions).  The IS ratios and
 * sqrt(A/B) stay FP32 (FP64 in ISNMF_FP64), A, B and the objective's log-sum
 * are FP64 in every mode. */
typedef enum {
    ISNMF_FP32 = 0,
    ISNMF_BF16 = 1,
    ISNMF_FP16 = 2,
    ISNMF_FP64 = 3   /* whole fit in FP64 (logic check against the oracle) */
} isnmf_precision;

/* Starting point of the inner fit of h (section 2.3, fresh or warm restarts). */
typedef enum {
    ISNMF_H_ONES = 0,  /* fresh restart from h = 1                         */
    ISNMF_H_WARM = 1   /* warm restart from the caller's H (in/out)        */
} isnmf_hinit;

/* Kernel family.  PLAIN: unfused one-op-per-launch kernels (the comparison
 * point); FUSED: one MFMA kernel for the whole inner fit; AUTO: FUSED where
 * the shape is supported, else PLAIN. */
typedef enum {
    ISNMF_KERNEL_AUTO = 0,
    ISNMF_KERNEL_PLAIN = 1,
    ISNMF_KERNEL_FUSED = 2
} isnmf_kernel;

/* Parameters of Algorithm 1.  Defaults (isnmf_params_default):
 * eps 1e-12, inner_iters 20, rho 1, normalize 1, h_init ONES, precision
 * FP32, kernel AUTO, update_w 1, psi_lambda 0, psi_a 1.
 *
 * Penalty on H (section 2.2, Extensions: a concave increasing psi of each
 * column sum).  With psi_lambda > 0 every inner fit minimizes
 *   d_IS(eps + v, eps + W h) + psi_lambda * log(psi_a + sum_k h_k)
 * by the majorize-minimize update with the penalty's tangent:
 *   h_k <- h_k * sqrt(num_k / (den_k + psi_lambda / (psi_a + sum_j h_j))),
 * the sum taken at the start of the update.  The statistics, the fold and
 * the W update are unchanged (the penalty involves H only), and the frame
 * losses stay the d_IS terms.  Supported by FP64 and FP32 handles (FP32 runs
 * the 8-wave VALU fit variant when the shape has one, F <= 1088 and K <= 64,
 * else the plain path); BF16/FP16 handles, isnmf_batch_mu, the batched and the
 * served forms return ISNMF_EUNSUPPORTED for psi_lambda > 0. */
typedef struct {
    double eps;        /* eps >= 0: shift of the small-amplitude remedy (section 2.3)     */
    int inner_iters;   /* >= 0: multiplicative updates of h per frame                     */
    double rho;        /* in [0,1]: weight of past statistics, A <- rho*A + sum a          */
    int normalize;     /* 1: rescale W columns to unit L1 norm after each update (Alg. 1) */
    int h_init;        /* isnmf_hinit                                                     */
    int precision;     /* isnmf_precision                                                 */
    int kernel;        /* isnmf_kernel                                                    */
    int update_w;      /* 1: W <- sqrt(A/B); 0: W frozen, statistics still accumulate     */
    double psi_lambda; /* >= 0: weight of the penalty on H above; 0: none                 */
    double psi_a;      /* > 0: offset a of psi(s) = psi_lambda * log(a + s)               */
} isnmf_params;

typedef struct isnmf_online isnmf_online;   /* opaque handle */

/* Fill *p with the defaults above: Algorithm 1's inputs with eps of section
 * 2.3, rho = 1 (no forgetting) and unit-norm columns.  Host only. */
void isnmf_params_default(isnmf_params *p);

/* Message for a status code (static string, never NULL).  Not part of the
 * method: error reporting of the interface.  Host only. */
const char *isnmf_strerror(int status);

/*
 * Weight of the past statistics for a forgetting factor r (section 2.3,
 * scaling past data): rho = r^(beta / N), with beta frames per update of W
 * and N frames in the data set, so that the past is discounted by r per pass
 * over the N frames whatever beta is; rho -> 1 as N grows, and r = 0 with
 * beta = N gives rho = 0, the batch algorithm.  The result is the
 * isnmf_params.rho of a handle (A <- rho*A + sum a, B <- rho*B + sum b).
 * Host only (no device work).  ISNMF_EINVAL unless 0 <= r <= 1, beta >= 1,
 * n_frames >= 1 and host_rho != NULL.
 */
int isnmf_forgetting_rho(double r, long long beta, long long n_frames, double *host_rho);

/* ------------------------------------------------------------------ online */

/* Bytes of device workspace an online handle (Algorithm 1's state W, A, B of
 * eq. (4), O(FK), plus the minibatch buffers) needs for frames of length F,
 * K components and minibatches of at most b_max frames.  0 on bad sizes. */
size_t isnmf_online_workspace_size(int F, int K, int b_max, const isnmf_params *p);

/*
 * Create an online handle (Algorithm 1, inputs W(0), A(0), B(0), rho, beta,
 * eps).  W0: device F x K FP32 (ldw).  A0, B0: device F x K FP64 or NULL for
 * zero (A(0) = B(0) = 0).  workspace: device memory of at least
 * isnmf_online_workspace_size() bytes, 256-byte aligned, owned by the caller
 * and used by the handle until isnmf_online_destroy.  p == NULL means the
 * defaults.  On error *out is NULL.
 */
int isnmf_online_init(isnmf_online **out, int F, int K, int b_max, const isnmf_params *p,
                      const float *W0, int ldw, const double *A0, const double *B0,
                      void *workspace, size_t ws_bytes, void *stream);

/*
 * One minibatch step (the body of Algorithm 1 at t = 0 mod beta, beta = b;
 * eq. (4) summed over the minibatch):
 *   for each frame n < b: h_n <- inner_iters MU updates of argmin_h
 *        d_IS(eps + v_n, eps + W h)  from h = 1 (ONES) or Hb[:,n] (WARM);
 *   A <- rho*A + sum_n ((eps+v_n)/(eps+W h_n)^2 h_n^T) o W^2,
 *   B <- rho*B + sum_n (1/(eps+W h_n)) h_n^T;
 *   W <- sqrt(A/B); columns rescaled to unit L1 norm (A/s, B*s, warm H*s).
 * Vb: device F x b FP32 (ldv >= F), values >= 0.  1 <= b <= b_max.
 * Hb: NULL, or device K x b FP32 (ldh >= K) receiving the fitted h (also the
 *     starting point under ISNMF_H_WARM, where it is required).
 * d_loss_sum: NULL or device double; sum_n sum_f d_IS(eps+v, eps+W h) of this
 *     minibatch (W before the update) is ADDED to it.
 * d_dw: NULL or device double; receives ||W_new - W_old||_F.
 * The handle's frame counter t advances by b.
 */
int isnmf_online_step(isnmf_online *h, const float *Vb, int ldv, int b,
                      float *Hb, int ldh, double *d_loss_sum, double *d_dw, void *stream);

/*
 * A pass of Algorithm 1 over n_frames frames already resident on the device:
 * consecutive minibatches of b frames (the last one shorter when b does not
 * divide n_frames), each exactly one isnmf_online_step.  V: device F x
 * n_frames FP32 (ldv >= F).  H: NULL or device K x n_frames (ldh >= K)
 * receiving every fitted h (required under ISNMF_H_WARM, where it is also
 * the starting point).  d_loss_sum as in isnmf_online_step (the pass total is
 * added).  1 <= b <= b_max.
 */
int isnmf_online_pass(isnmf_online *h, const float *V, int ldv, long long n_frames, int b,
                      float *H, int ldh, double *d_loss_sum, void *stream);

/*
 * Several passes over a finite set of N frames with warm restarts (section
 * 2.3, finite data sets): the activations of all N frames stay resident in H,
 * and pass p visits the frames in the order perm[p N .. p N + N), in
 * minibatches of b (the last one shorter when b does not divide N).  Each
 * minibatch is one isnmf_online_step on the visited frames whose inner fit
 * starts from their h of the previous visit (H as given on the first), and
 * whose fitted, rescale-compensated h is written back to H.
 * The handle must use ISNMF_H_WARM.  V: device F x N FP32 (ldv >= F).
 * perm: device int, passes x N entries, each pass a permutation of 0..N-1;
 *   an index outside [0, N) reads zero frames, writes nothing and sets the
 *   status bit 8.  A pass that repeats a frame in adjacent minibatches leaves
 *   unspecified which of its h values the later visit starts from.
 *   H: device K x N FP32 (ldh >= K), in/out.
 * d_loss_sum as in isnmf_online_step (the total of every visit is added).
 * 1 <= b <= b_max, passes >= 1.  The frames and activations of a minibatch
 * are gathered into workspace buffers the handle reserves under H_WARM; the
 * gather of one minibatch and the write-back of the one before share a launch.
 */
int isnmf_online_passes(isnmf_online *h, const float *V, int ldv, long long N, const int *perm,
                        int passes, int b, float *H, int ldh, double *d_loss_sum, void *stream);

/*
 * Fit activations only (the inner argmin of Algorithm 1 at the current W, no
 * change to A, B or W): e.g. held-out evaluation, or timing of the fit.
 * Vb, b, Hb, ldh as in isnmf_online_step (Hb may be NULL); d_loss_sum
 * receives += sum_n sum_f d_IS(eps + v_n, eps + W h_n).
 */
int isnmf_online_fit(isnmf_online *h, const float *Vb, int ldv, int b, float *Hb, int ldh,
                     double *d_loss_sum, void *stream);

/*
 * Not part of the method: measurement hooks.
 * Per-launch timing of the fit kernel with HIP events on the launch stream.
 * enable != 0 starts timing every fit launch of this handle (up to
 * `capacity` launches; later launches are not timed); enable == 0 stops.
 * The VALU fit variants are launched with the event pair attached to the
 * dispatch itself (hipExtLaunchKernel), so their time is the kernel's own;
 * the other variants record the pair around the launch.  isnmf_online_timing synchronizes, returns the number
 * of timed launches and their total duration in milliseconds, and clears
 * the record.
 */
int isnmf_online_set_timing(isnmf_online *h, int enable, int capacity);
int isnmf_online_timing(isnmf_online *h, long long *host_launches, double *host_total_ms);

/* Copy the state of Algorithm 1 out: the dictionary W and the statistics A
 * and B of eq. (4) (the sums of the a and b terms over the frames seen, past
 * ones weighted by rho), and the frame counter t.  W: device F x K FP32
 * (ld F) or NULL; A, B: device F x K FP64 (ld F) or NULL; host_t: host or
 * NULL.  A and B come out with the last column rescale applied (A/s, B*s).
 * Enqueued on `stream`. */
int isnmf_online_get(const isnmf_online *h, float *W, double *A, double *B,
                     long long *host_t, void *stream);

/* FP64 master copy of Algorithm 1's W = sqrt(A/B) after the column rescale
 * (device F x K, ld F).  W is kept in FP64 between steps in every mode; the
 * FP32 (or BF16/FP16) copy is rounded from it.  Enqueued on `stream`. */
int isnmf_online_get_w64(const isnmf_online *h, double *W, void *stream);

/* Replace the state of Algorithm 1 (checkpoint restore, or the inputs W(0),
 * A(0), B(0) of a restart): W device FP32 F x K (ld F) or NULL to keep, the
 * eq. (4) statistics A, B device FP64 F x K (ld F) or NULL to keep, t the
 * frame counter (>= 0).  The next step reads them as Algorithm 1 reads its
 * state at t.  Enqueued on `stream`. */
int isnmf_online_set(isnmf_online *h, const float *W, const double *A, const double *B,
                     long long t, void *stream);

/* As isnmf_online_set for Algorithm 1's W given in FP64 (device F x K,
 * ld F). */
int isnmf_online_set_w64(isnmf_online *h, const double *W, void *stream);

/* Not part of the method: error reporting (the 0/0 guards of the h update,
 * section 2.1, and of W = sqrt(A/B), Algorithm 1).
 * Synchronize the handle's last stream and read the sticky device flags:
 * bit 0 a non-finite value in V, bit 1 a guarded 0/0 in the h update, bit 2
 * a guarded 0/0 in W = sqrt(A/B) or the rescale.  Returns ISNMF_ENONFINITE
 * when bit 0 is set, ISNMF_OK otherwise.  Clears the flags. */
int isnmf_online_status(isnmf_online *h, int *host_flags);

/* Not part of the method: shape / mode queries of a handle (host only). */
int isnmf_online_info(const isnmf_online *h, int *F, int *K, int *b_max, int *kernel_used);

/* Not part of the method: free the handle (not the workspace).  Waits for
 * the handle's last stream. */
int isnmf_online_destroy(isnmf_online *h);

/* ------------------------------------------------------------ batched form */

/*
 * Many independent online streams of Algorithm 1 advanced together (one
 * minibatch each per step, eq. (4) summed over it): each step fits one
 * minibatch of every stream that has frames left (fresh restarts), folds it
 * into that stream's A and B and updates its W -- exactly
 * isnmf_online_step on each handle, with one fit launch per kernel variant
 * in use, on up to four lanes, each followed by one fold and one rescale
 * launch for its streams (none where the fits fold and rescale themselves,
 * see isnmf_multi_launches).  The frame
 * cursors live on the device, so a step can be captured into a hipGraph and
 * replayed (isnmf_multi_run with use_graph).
 *
 * handles: S distinct online handles (FUSED kernel, ISNMF_H_ONES), owned by
 *   the caller and not stepped otherwise while the plan is in use.
 * V[s]: device F_s x n_frames[s] FP32 (ldv[s] >= F_s) -- stream s's frames,
 *   consumed in order, b[s] per step (1 <= b[s] <= min(b_max_s, 512)).
 * d_loss: NULL or device double[S]; stream s's minibatch losses are added.
 * workspace: device memory of isnmf_multi_workspace_size() bytes, 256-byte
 *   aligned, caller-owned.  The per-stream descriptors are copied in at
 *   creation (the call synchronizes `stream`).
 */
typedef struct isnmf_multi isnmf_multi;

/* Not part of the method: bytes of device workspace of a plan over these
 * handles and minibatch sizes (descriptor tables, work lists, cursors).
 * 0 on bad arguments. */
size_t isnmf_multi_workspace_size(isnmf_online *const *handles, int S, const int *b);

/* Create the plan (see above): one stream of Algorithm 1 per handle. */
int isnmf_multi_create(isnmf_multi **out, isnmf_online *const *handles, int S,
                       const float *const *V, const int *ldv, const long long *n_frames,
                       const int *b, double *d_loss, void *workspace, size_t ws_bytes,
                       void *stream);

/* One step of Algorithm 1 (one minibatch) for every stream with frames
 * left.  The handles' frame counters advance on the host. */
int isnmf_multi_step(isnmf_multi *m, void *stream);

/* `steps` steps of Algorithm 1 as isnmf_multi_step; use_graph != 0 captures
 * one step into a hipGraph on first use (on a private stream) and replays it
 * on `stream`. */
int isnmf_multi_run(isnmf_multi *m, int steps, int use_graph, void *stream);

/* Not part of the method: largest number of frames any stream has left
 * (host bookkeeping). */
int isnmf_multi_frames_left(const isnmf_multi *m, long long *host_max_left);

/* Not part of the method: the launches of one step of the plan.
 * *fit_launches: one per group of streams on one kernel variant;
 * *fold_launches and *rescale_launches: one each per lane of fit launches
 * (up to four).  There is no fold launch when every stream is on a 16-frame
 * tile variant (BF16 or FP32; tune_set cpw -1 or -3) with b[s] <= 128 and
 * its LDS holds the fold's staging (F <= 608 for BF16 at K <= 64; F = 513 at
 * K <= 52, F <= 400 at K = 64 for FP32): each fit workgroup then folds its
 * stream's minibatch itself, and in the BF16 variant also rescales W (the
 * same bits as the fold and rescale launches), so such a plan of BF16
 * streams has no rescale launch either.  ISNMF_EINVAL for a null argument. */
int isnmf_multi_launches(const isnmf_multi *m, int *fit_launches, int *fold_launches,
                         int *rescale_launches);

/* Not part of the method: wait for the plan's streams and free it (not the
 * handles, not the workspace). */
int isnmf_multi_destroy(isnmf_multi *m);

/* ------------------------------------------------------------- served form */

/*
 * Continuous-batching engine over many online sessions (fresh restarts):
 * each session follows Algorithm 1 with one minibatch per chunk (beta = the
 * chunk length, eq. (4) summed over it), its W, A, B resident on the device.
 * Clients submit chunks of frames already on the device; each engine step
 * takes at most one pending chunk per resident session (oldest first, at
 * most max_per_step chunks and max_frames frames), runs one minibatch step
 * (b = chunk length) for all of them in shared launches, and keeps up to
 * `inflight` steps enqueued while new arrivals join the next one.  Per
 * session, chunks are applied in submission order, exactly as
 * isnmf_online_step would, so a session's result does not depend on what
 * else shares the steps.
 *
 * Admission by HBM footprint.  A session is RESIDENT (it holds one of
 * max_sessions rows of the device descriptor tables and its `footprint` --
 * its workspace bytes, or any figure the caller charges -- counts against
 * hbm_budget) or WAITING in a first-in first-out queue.  The head of the
 * queue is admitted as soon as a row is free and its footprint fits the
 * budget the resident sessions leave; the queue keeps its order (a large
 * head is not overtaken).  isnmf_server_close returns a session's row and
 * footprint once its last submitted chunk has completed, and the next
 * isnmf_server_pump (or the close itself) admits waiting sessions into them.
 * Chunks submitted to a waiting session queue up and are served once it is
 * admitted.  Session states: */
typedef enum {
    ISNMF_SESSION_WAITING = 0,   /* opened, not yet admitted              */
    ISNMF_SESSION_RESIDENT = 1,  /* admitted; its chunks are served       */
    ISNMF_SESSION_CLOSING = 2,   /* closed by the caller, chunks left     */
    ISNMF_SESSION_CLOSED = 3     /* row and footprint returned; the server
                                    no longer touches the handle          */
} isnmf_session_state;

/*
 * workspace: device memory of isnmf_server_workspace_size() bytes (descriptor
 *   tables and work lists), 256-byte aligned, caller-owned.  The server also
 *   allocates `inflight` small pinned host buffers and events.
 * Sessions must use the fused kernel: an MFMA tile variant with one 64-row
 * chunk per wave and K <= 64 (F <= 516), or the BF16 16-frame tile variant
 * (cpw = -1, F <= 640, K <= 64); chunks hold 1..min(b_max, 512, max_frames)
 * frames.
 * Calls are not thread-safe.
 */
typedef struct isnmf_server isnmf_server;

/* Not part of the method: bytes of device workspace of a server with
 * max_sessions resident sessions
 * (the rows of its descriptor tables), max_per_step chunks per engine step and
 * `inflight` steps in flight.  0 on bad sizes. */
size_t isnmf_server_workspace_size(int max_sessions, int max_per_step, int inflight);

/* Create the engine (see above; each session one stream of Algorithm 1).
 * hbm_budget: bytes of session footprint the resident sessions may hold
 * together.  The server's steps run on `stream`. */
int isnmf_server_create(isnmf_server **out, int max_sessions, int max_per_step, int max_frames,
                        int inflight, size_t hbm_budget, void *workspace, size_t ws_bytes,
                        void *stream);

/*
 * Open a session on handle h (one stream of Algorithm 1): *session receives
 * its id (ids are never reused).  The session is admitted at once when the
 * waiting queue is empty, a row is free and the footprint fits; otherwise it
 * waits (isnmf_server_session_state).  ISNMF_ENOMEM when footprint alone
 * exceeds hbm_budget (it could never be admitted); ISNMF_EINVAL when h is
 * already open on this server and not closed; ISNMF_EUNSUPPORTED for a handle
 * whose fit variant the engine does not run (an MFMA tile variant with wg =
 * 1, cpw = 2, nw other than 4 or 8, or K > 64), for a penalty on H or the
 * plain kernel (ISNMF_EINVAL for warm restarts).  Admission enqueues the
 * session's descriptors on the server's stream.
 */
int isnmf_server_open(isnmf_server *s, isnmf_online *h, size_t footprint, int *session);

/*
 * Close a session (Algorithm 1's stream ends): no further chunks are
 * accepted (isnmf_server_submit returns ISNMF_ESTATE), chunks already
 * submitted are still served in order, and once the last of them has
 * completed the session's row and footprint return to the engine and it
 * becomes CLOSED; the caller may then destroy the handle and free its
 * workspace.  Closing twice is not an error.  Never blocks.
 */
int isnmf_server_close(isnmf_server *s, int session);

/* Not part of the method: admission bookkeeping.  *state receives the
 * session's isnmf_session_state (host only, never blocks). */
int isnmf_server_session_state(const isnmf_server *s, int session, int *state);

/* Not part of the method: footprint charged by the resident sessions, and the
 * numbers of resident and waiting sessions (host pointers, any may be NULL). */
int isnmf_server_admission(const isnmf_server *s, size_t *host_used, int *host_resident,
                           int *host_waiting);

/*
 * Running loss of a session (the diagnostic of Algorithm 1's online
 * objective, eq. 1 with eps inside, section 2.3): from the next step on,
 * each served chunk adds its sum of d_IS(eps + v, eps + W h) over the chunk's
 * frames and rows, in FP64, to *d_loss_sum (a device scalar the caller owns
 * and zeroes; NULL turns it off again).  The sum of one chunk is formed in the
 * same order as isnmf_online_step's loss_sum for that chunk, so a session
 * served in a mix accumulates the same bits as stepped alone chunk by chunk.
 * For a resident session, synchronizes the server's stream; for a waiting
 * one, takes effect at admission.  ISNMF_EINVAL for a session id not
 * returned by isnmf_server_open, ISNMF_ESTATE for a closed session.
 */
int isnmf_server_set_loss(isnmf_server *s, int session, double *d_loss_sum);

/* Queue a chunk, the next minibatch of the session's stream (Algorithm 1,
 * beta = n_frames): device F x n_frames FP32, ldv >= F.  arrival: the
 * client's timestamp on isnmf_server_clock() (negative: now).  The frames
 * must stay valid until the chunk completes.  ISNMF_ESTATE once the session
 * is closed or closing. */
int isnmf_server_submit(isnmf_server *s, int session, const float *V, int ldv, int n_frames,
                        double arrival, long long *request);

/* Retire finished steps, release sessions closed meanwhile, admit waiting
 * sessions, and enqueue new steps (the minibatch steps of Algorithm 1 for
 * the chunks taken).  Never blocks on the device. */
int isnmf_server_pump(isnmf_server *s, int *launched_frames);

/* Not part of the method: chunks queued (resident and waiting sessions) and
 * chunks in flight. */
int isnmf_server_pending(const isnmf_server *s, long long *queued, long long *inflight);

/* Pump until every submitted chunk has completed (synchronizes): every
 * queued minibatch step of Algorithm 1 is taken.
 * ISNMF_ESTATE when chunks remain that only waiting sessions hold and nothing
 * is in flight: no release can admit them until the caller closes sessions. */
int isnmf_server_drain(isnmf_server *s);

/* Not part of the method: completed chunks since the last call (host arrays
 * of max_out entries, any may be NULL): request id, session, frames, arrival,
 * launch and completion times in seconds on isnmf_server_clock(). */
int isnmf_server_results(isnmf_server *s, int max_out, long long *req, int *session,
                         int *n_frames, double *arrival, double *start, double *done, int *count);

/* Not part of the method: engine steps and frames served so far. */
int isnmf_server_stats(const isnmf_server *s, long long *steps, long long *frames);

/* Not part of the method: monotonic host clock in seconds used for arrival
 * and completion times. */
double isnmf_server_clock(void);

/* Not part of the method: wait for the engine's streams and free the server
 * (not the handles, not the workspace). */
int isnmf_server_destroy(isnmf_server *s);

/* ------------------------------------------------------------- autotuner */

/* Not part of the method: bytes of device workspace isnmf_autotune needs for
 * (F, K, b) -- a scratch online state, b synthetic frames and a W(0).  0 on
 * bad sizes. */
size_t isnmf_autotune_workspace_size(int F, int K, int b, const isnmf_params *p);

/*
 * Not part of the method: kernel selection for the inner fit of Algorithm 1
 * (the h updates of section 2.1 and the final ratios).
 * Time every fused-fit kernel variant valid for (F, K, precision) on
 * synthetic frames (b per launch, `trials` launches each) and record the
 * fastest in the process-wide tuning table; handles created afterwards with
 * that shape use it.  workspace: device memory of at least
 * isnmf_autotune_workspace_size() bytes, 256-byte aligned, caller-owned (the
 * call allocates no device memory).  Synchronizes `stream`.  out_variant:
 * index of the chosen variant (0 is the default); out_us: its average launch
 * time in microseconds.
 */
int isnmf_autotune(int F, int K, int b, const isnmf_params *p, int trials, int *out_variant,
                   double *out_us, void *workspace, size_t ws_bytes, void *stream);

/* Not part of the method: read / set / clear the tuning table (for
 * persisting it between processes):
 * nw = waves per workgroup, cpw = 64-row chunks per wave, wg = W read from
 * its 16-bit copies in memory instead of registers.  Non-positive cpw name
 * the other variants: cpw = 0 the FP32 VALU variant (one frame per workgroup
 * of nw = 8 waves, or of nw = 16 waves for 1088 < F <= 1152, where it is the
 * FP32 default and the only VALU form), cpw = -4 its BF16 form (nw = 8),
 * cpw = -1 the BF16 16-frame tile variant (16 frames per wave, nw = 8 waves
 * per workgroup, on 16x16x32 MFMA), cpw = -2 its streamed form and cpw = -3
 * the FP32 16-frame tile variant (16x16x4 FP32 MFMA).  The batched form runs
 * all of them; the served form all but the MFMA tile variants with wg = 1,
 * cpw = 2, nw other than 4 or 8, or K > 64.  The autotuner times the variants at the b
 * it is given: a single stream's minibatch for latency, or the frames of all
 * streams of a batched step for throughput. */
int isnmf_tune_get(int F, int K, int precision, int *nw, int *cpw, int *wg);
int isnmf_tune_set(int F, int K, int precision, int nw, int cpw, int wg);
void isnmf_tune_clear(void);

/* ------------------------------------------------------------------- batch */

/* Bytes of device workspace isnmf_batch_mu (section 2.1) needs. */
size_t isnmf_batch_workspace_size(int F, int K, int N, const isnmf_params *p);

/*
 * `cycles` cycles of batch IS-NMF by multiplicative updates (section 2.1):
 * each cycle updates all of H once from the current (W, H), recomputes the
 * statistics A, B of eq. (3) at the new H, sets W = sqrt(A/B) and, if
 * p->normalize, rescales W's columns to unit L1 norm with H compensated.
 * V: device F x N FP32.  W (F x K, ldw) and H (K x N, ldh): device FP32,
 * in/out (H is the starting point; use ones for a fresh start).
 * d_obj_trace: NULL or device double[cycles], objective of eq. (1) after
 * each cycle.  p->inner_iters, rho, h_init and update_w are ignored.  The
 * fused fit runs the tuning table's variant for (F, K, precision), as an
 * online handle does (isnmf_autotune with b = N tunes it for this use).
 */
int isnmf_batch_mu(const float *V, int ldv, int F, int N, float *W, int ldw,
                   float *H, int ldh, int K, int cycles, const isnmf_params *p,
                   double *d_obj_trace, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of device workspace isnmf_objective (eq. (1)) needs. */
size_t isnmf_objective_workspace_size(int F, int K, int N);

/*
 * Objective of eq. (1) with the eps shift:
 *   *d_out = (1/N) sum_n sum_f d_IS(eps + V_fn, eps + (W H)_fn),
 * summed in FP64 in a fixed order (deterministic).  V, W, H: device FP32.
 * d_out: device double.
 */
int isnmf_objective(const float *V, int ldv, const float *W, int ldw, const float *H, int ldh,
                    int F, int K, int N, double eps, double *d_out,
                    void *workspace, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * objective of isnmf_objective, same kernels, same bits, with no workspace
 * argument.  Its per-frame partial sums live in a fixed array of
 * ISNMF_OBJECTIVE_NOALLOC_MAX_FRAMES doubles (8 MiB) inside the library, one
 * copy per GPU, held until the process ends; the call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine).  N above the
 * maximum returns ISNMF_EINVAL before any device work.  Every call on a GPU
 * shares that GPU's array, and each call writes every partial it reads, so
 * calls that follow one another on a stream need nothing cleared; calls that
 * overlap on one GPU (different streams or threads, not ordered) race and
 * must not be issued.  Other arguments as isnmf_objective.
 */
#define ISNMF_OBJECTIVE_NOALLOC_MAX_FRAMES (1 << 20)
int isnmf_objective_noalloc(const float *V, int ldv, const float *W, int ldw, const float *H,
                            int ldh, int F, int K, int N, double eps, double *d_out,
                            void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ISNMF_H */
