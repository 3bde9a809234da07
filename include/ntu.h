/*
 * ntu.h -- C ABI of libntu: the MI355X (gfx950) hot path of the neighbourhood
 * tensor update (NTU) for iPEPS time evolution.
 *
 * Method: J. Dziarmaga, "Time evolution of an infinite projected entangled
 * pair state: a neighborhood tensor update", arXiv:2107.06635, Sec. II
 * (Figs. 2, 4, 5 and Eqs. (1)-(5)).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every call
 * ---------------------------------------------------------------------------
 * Tensors.  Every array argument is an ntu_tensor descriptor: a DEVICE
 *   pointer to memory the caller allocated, its element type, and its shape
 *   and strides (in elements).  The library never frees or reallocates caller
 *   memory.  Batched operands carry the batch as their leading dimension;
 *   uneven bond dimensions are handled by one call per dimension.  Only
 *   dense row-major layouts are accepted (stride of the last dimension 1,
 *   each other stride the product of the later extents; extents of 1 may
 *   have any stride).  Each call checks every descriptor against the shape
 *   it needs (named below) before anything is launched: a NULL descriptor or
 *   data pointer gives NTU_ERR_ARG, memory that is not device memory
 *   NTU_ERR_ARG, a wrong element type NTU_ERR_DTYPE, a wrong rank, extent or
 *   stride NTU_ERR_SHAPE.
 * Storage.  Row-major, last index fastest.  NTU_C128 is interleaved
 *   (re, im) double pairs (the layout of a complex128 array), NTU_F64 plain
 *   doubles, NTU_C64 interleaved float pairs (accepted for site tensors
 *   only: read with an upcast, and in ntu_trotter_step also written back
 *   rounded).  All other results are written in the context's compute type
 *   (NTU_F64 or NTU_C128).
 * Canonical bond.  The updated bond joins X.r to Y.l.  r_g is the rank of the
 *   gate split (Fig. 2(a)), R = D * r_g the dimension of the enlarged bond.
 * Streams.  Work is enqueued on the context's stream (ntu_set_stream) and is
 *   asynchronous; results are valid after that stream is synchronised.  No
 *   call allocates device memory or synchronises: all scratch space comes from
 *   the workspace allocated by ntu_ctx_create, so call sequences can be
 *   captured into a HIP graph.
 * Errors.  Argument, shape and dtype errors are detected on the host before
 *   anything is launched; the call then returns a negative status and
 *   ntu_last_error() describes it.  Numerical conditions (non-finite values)
 *   are reported in the caller's device stats buffers.
 * Concurrency.  One context serves one stream; calls on one context must not
 *   overlap.  Distinct contexts are independent.
 */
#ifndef NTU_H
#define NTU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ntu_ctx ntu_ctx;
typedef int32_t ntu_status;

enum {
  NTU_OK = 0,
  NTU_ERR_ARG = -1,         /* null pointer, bad enum, batch < 0 ...        */
  NTU_ERR_SHAPE = -2,       /* D, p, r_g outside what the context supports   */
  NTU_ERR_DTYPE = -3,       /* dtype not accepted for this operand           */
  NTU_ERR_HIP = -4,         /* a HIP runtime call failed                     */
  NTU_ERR_NONFINITE = -5,   /* reserved: non-finite values are flagged in stats */
  NTU_ERR_WORKSPACE = -6,   /* request exceeds the context's workspace       */
  NTU_ERR_UNSUPPORTED = -7  /* valid request the library does not implement  */
};

/* element types */
enum { NTU_F64 = 0, NTU_C128 = 1, NTU_C64 = 2 };

#define NTU_MAX_DIMS 8
/* A dense row-major device array (see "Tensors" above). */
typedef struct ntu_tensor {
  void* data;                     /* device pointer to the first element      */
  int32_t dtype;                  /* NTU_F64, NTU_C128 or NTU_C64             */
  int32_t ndim;                   /* 1 .. NTU_MAX_DIMS                        */
  int64_t shape[NTU_MAX_DIMS];    /* extents                                  */
  int64_t stride[NTU_MAX_DIMS];   /* in elements                              */
} ntu_tensor;

/* arithmetic of the environment contraction (ntu_env_contract) */
enum {
  NTU_PREC_F64 = 0,    /* FP64 throughout                                      */
  NTU_PREC_BF16X3 = 1, /* operands split hi+lo in bfloat16, 3 MFMA products,
                          FP32 accumulation, FP32 intermediates               */
  NTU_PREC_FP16X3 = 2, /* same with float16 and the low part scaled by 2^11    */
  NTU_PREC_BF16X6 = 3  /* three-way bfloat16 split, 6 products                 */
};

/* metric repair modes (ntu_metric_fix) */
enum { NTU_FIX_HERM = 0, NTU_FIX_HERM_CLIP = 1 };
/* Bond-update scheme of a Trotter step: the full NTU update, or the SVDU
 * update of Fig. 2 (reduction, truncated SVD of R_X R_Y^T, recombination; no
 * environment), with the singular values normalised by the largest as at the
 * end of the NTU update (Fig. 5(d)). */
enum { NTU_SCHEME_NTU = 0, NTU_SCHEME_SVDU = 1 };

/* the four inequivalent bonds of the two-site checkerboard */
enum { NTU_BOND_H1 = 0, NTU_BOND_H2 = 1, NTU_BOND_V1 = 2, NTU_BOND_V2 = 3 };

/*
 * Context.  Allocates the workspace for items up to bond dimension max_D,
 * physical dimension d, ancilla dimension d_anc (1 = none), gate rank r_g and
 * max_batch items per call, in compute type dtype (NTU_F64 or NTU_C128).
 * device: HIP device ordinal.  The stream is the null stream until
 * ntu_set_stream is called.  Returns NTU_ERR_HIP if the workspace cannot be
 * allocated.
 */
ntu_status ntu_ctx_create(ntu_ctx** out, int device, int dtype, int d, int d_anc,
                          int r_g, int max_D, int max_batch);
ntu_status ntu_ctx_destroy(ntu_ctx* ctx);
/* stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream). */
ntu_status ntu_set_stream(ntu_ctx* ctx, void* stream);
/*
 * Side stream of ntu_trotter_step.  Each bond's SVDU initial guess (Fig.
 * 2(c,d)) needs only the reduction, so the step computes it on a second
 * stream while the environment is contracted, ordered by events recorded on
 * the context's stream (so the pair can be captured into a HIP graph).  By
 * default the context owns that stream; stream != NULL makes the step use
 * the caller's (hipStream_t, for instance one shared by several contexts, so
 * that fewer streams compete for hardware queues); NULL restores the
 * context's own.  The caller keeps the stream alive while the context uses it.
 */
ntu_status ntu_set_aux_stream(ntu_ctx* ctx, void* stream);
/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char* ntu_last_error(const ntu_ctx* ctx);
/* Bytes of device workspace held by ctx. */
size_t ntu_workspace_bytes(const ntu_ctx* ctx);
/* Library version string (static). */
const char* ntu_version(void);

/*
 * Gate split, Fig. 2(a).  For each item, the two-site gate
 * G[(s1' s2'), (s1 s2)] (d^2 x d^2, compute type) is regrouped as
 * [(s1' s1), (s2' s2)] and SV-decomposed; the r_g leading terms give
 * GA[s1', s1, k] = sqrt(sigma_k) U[(s1' s1), k] and
 * GB[s2', s2, k] = sqrt(sigma_k) conj(V)[(s2' s2), k], so that
 * G = sum_k GA[:, :, k] (x) GB[:, :, k] up to the discarded terms.
 * Gauge: the first entry of U[:, k] whose modulus is within 1e-8 of the
 * column maximum is made real and positive.
 * gate: (batch, d^2, d^2), compute type.  GA, GB: (batch, d, d, r_g), compute
 * type, written.  sigma: (batch, d^2) NTU_F64, written: all singular values
 * in descending order.
 */
ntu_status ntu_gate_split(ntu_ctx* ctx, int batch, const ntu_tensor* gate, ntu_tensor* GA, ntu_tensor* GB,
                          ntu_tensor* sigma);

/*
 * Manifestly Hermitian purification, Sec. IV: Eq. (11) with the basis of
 * Fig. 8.  For each item, the real matrix of rho -> G rho G^dagger on the
 * products O^a x O^b of the spin-1/2 Hermitian basis O = (X, Y, Z, 1):
 *   G (O^a x O^b) G^dagger = sum_{a' b'} S[(a' b'), (a b)] O^a' x O^b'.
 * The half rho(beta/2) of Eq. (7), written in this basis, is an iPEPS with
 * real tensors and a physical index a of dimension 4; S is its two-site gate
 * (pass it to ntu_gate_split; for the gate of Eq. (10) its operator-Schmidt
 * rank is 4, so r_g = 4).
 * gate: (batch, 4, 4), NTU_F64 or NTU_C128, rows (s1' s2'), columns
 * (s1 s2).  S: (batch, 16, 16) NTU_F64, written, rows (a' b'), columns (a b).
 * The context must have d = 4 and d_anc = 1 (NTU_ERR_SHAPE otherwise).
 */
ntu_status ntu_superop_gate(ntu_ctx* ctx, int batch, const ntu_tensor* gate, ntu_tensor* S);

/*
 * Reduction, Fig. 2(b).  Applies the gate factor to the site tensor and takes
 * the thin QR decomposition of the result:
 *   side 0 (X): W[(s',a,t,l,b), (r,k)] = sum_s GA[s',s,k] X[(s,a),t,l,b,r]
 *   side 1 (Y): W[(s',a,t,b,r), (l,k)] = sum_s GB[s',s,k] Y[(s,a),t,l,b,r]
 *   W = Q R,  Q: (p D^3) x R with orthonormal (or zero) columns,
 *   R: R x R upper triangular with real non-negative diagonal.
 * Q is computed by Gram-Schmidt with the projection applied twice; a column
 * whose orthogonal part has norm <= 1e-10 * (largest column norm of W) is
 * dependent: its Q column and R diagonal are exactly zero.
 * site: (batch, p, D, D, D, D) in the compute type, or NTU_C64 with a
 * complex context; D is taken from it.  gate_factor: (batch, d, d, r_g).
 * Q: (batch, p D^3, R), written.  R: (batch, R, R), written.
 */
ntu_status ntu_reduce_qr(ntu_ctx* ctx, int batch, const ntu_tensor* site, const ntu_tensor* gate_factor,
                         int side, ntu_tensor* Q, ntu_tensor* R);

/*
 * Environment contraction, Fig. 4.  Builds the bond metric
 *   g[(a' b'), (a b)] = sum_e conj(Phi_{a'b'}(e)) Phi_{ab}(e)
 * where Phi_{ab} is the eight-site cluster (Fig. 4(b)) with QX[:, a] and
 * QY[:, b] in the two central sites and the six nearest neighbours
 * nbr = [L, TX, BX, TY, BY, Rn] around them: L left of X, TX/BX above/below X,
 * TY/BY above/below Y, Rn right of Y, with bonds TX.r-TY.l and BX.r-BY.l
 * parallel to the updated one.  Physical legs of the neighbours and their
 * virtual legs that leave the cluster are closed by contracting ket with bra
 * (Fig. 4(a,b)).  The result is Hermitian and non-negative up to rounding.
 * QX: (batch, p D^3, R), rows (p,t,l,b), as ntu_reduce_qr side 0.
 * QY: (batch, p D^3, R), rows (p,t,b,r), as ntu_reduce_qr side 1.
 * nbr: six descriptors, each (batch, p, D, D, D, D) site tensors (compute
 * type); D is taken from nbr[0].  precision: NTU_PREC_*.
 * g: (batch, R^2, R^2), compute type, written.
 */
ntu_status ntu_env_contract(ntu_ctx* ctx, int batch, const ntu_tensor* QX, const ntu_tensor* QY,
                            const ntu_tensor nbr[6], int precision, ntu_tensor* g);

/*
 * Metric repair.  The exact metric is Hermitian and non-negative (abstract;
 * Sec. II).  NTU_FIX_HERM replaces g by (g + g^H)/2.  NTU_FIX_HERM_CLIP also
 * sets negative eigenvalues to zero: g <- V max(Lambda, 0) V^H.  Rows and
 * columns that are exactly zero are left out of the eigenproblem; when the
 * remaining block is certified positive definite (Gershgorin discs right of
 * zero, else a Cholesky factor exists) the clip is the identity and is
 * skipped.  Complex g, and real g with n < 128: Jacobi eigen-decomposition.
 * Real g with n >= 128: g <- (g + g S) / 2 with S = sign(g) from a
 * polynomial iteration of matrix products on the FP64 matrix cores; every
 * eigenvalue of magnitude >= 1e-15 ||g||_F is resolved to rounding and a
 * smaller one contributes at most its own size.
 * g: (batch, n, n) in place, compute type, n = (D r_g)^2 for a D of the
 * context.
 * stats (may be NULL): (batch, 8) NTU_F64, written
 *   [0] ||g - g^H||_F / ||g||_F  (input)      [1] ||g||_F (input)
 *   [2] smallest eigenvalue (NaN if not computed)
 *   [3] largest eigenvalue  (NaN if not computed)
 *   [4] clipped mass sum(-lambda_neg)/sum|lambda| (0 if certified; from
 *       trace(g) and trace(g S) after the sign iteration)
 *   [5] 1 if the eigen-decomposition ran, 2 if the sign iteration ran
 *       ([2], [3] NaN), 0 if certified
 *   [6] number of non-finite entries in the input
 *   [7] Jacobi sweeps of the eigen-decomposition, or steps of the sign
 *       iteration (0 when none was needed)
 */
ntu_status ntu_metric_fix(ntu_ctx* ctx, int batch, ntu_tensor* g, int mode, ntu_tensor* stats);

/* Options of the bond fit (Eqs. (3)-(5)). */
typedef struct ntu_fit_opts {
  int n_iter;        /* maximum ALS iterations (one = an X and a Y half-step) */
  int early_stop;    /* 0: always n_iter; 1: stop when an iteration lowers the
                        error by <= conv_tol * N                                */
  double conv_tol;
  double kappa;      /* rank threshold (default 1e-10): kept singular values
                        S_i > kappa S_0                                          */
  int n_tol;         /* pseudo-inverse tolerance ladder, ascending, relative   */
  double tol[16];    /*   to the largest eigenvalue of g_X (Eq. (4))           */
  double tie;        /* errors within tie * N count as equal; the larger
                        tolerance wins                                          */
} ntu_fit_opts;

/* Fills o with the defaults: 20 iterations, no early stop, kappa 1e-10,
   ladder 1e-15 ... 1e-8, tie 1e-15. */
void ntu_fit_opts_default(ntu_fit_opts* o);

/* Number of doubles per item in the stats buffer of ntu_bond_fit. */
#define NTU_FIT_STATS_LEN(n_iter, D) (16 + 4 * (n_iter) + (D))

/*
 * Bond fit, Fig. 5 and Eqs. (2)-(5), with the SVDU initial guess (Fig. 2(c,d))
 * and the final balancing (Fig. 5(d)).
 *   P = RX RY^T;  SVDU: P ~ U S V^H truncated to Dn = min(D, #{S_i > kappa S_0});
 *   error eps = d^H g d,  d = vec(MX MY^T - P) (row-major (a, b));
 *   ALS: before the X half-step MY is made isometric with the product kept
 *   (the tilt of Fig. 5), then MX = pinv(g_X) J_X with K = I (x) MY,
 *   g_X = K^H g K, J_X = K^H g vec(P); the pseudo-inverse tolerance is the
 *   ladder value minimising eps, evaluated directly.  The Y half-step mirrors
 *   it.  Finally SVD of MX MY^T, singular values divided by the largest,
 *   MX = U S^1/2, MY = conj(V) S^1/2, zero-padded to D columns.
 * g: (batch, R^2, R^2) (Hermitian, non-negative).  RX, RY: (batch, R, R).
 * MX, MY: (batch, R, D), written; D is taken from MX.
 * stats (may be NULL): (batch, NTU_FIT_STATS_LEN(n_iter, D)) NTU_F64, written:
 *   [0] N = vec(P)^H g vec(P)  [1] eps of the SVDU guess  [2] final eps
 *   [3] final eps / N          [4] Dn   [5] Dk (kept after balancing)
 *   [6] iterations done        [7] half-steps solved by eigendecomposition
 *   [8] non-finite flag        [9] how g was certified well conditioned:
 *       0 not certified, 1 Gershgorin discs, 2 Cholesky of g - s I
 *       (s = 10 * largest ladder tolerance * ||g||_F; a certified half-step
 *       is solved by conjugate gradients instead of the ladder),
 *       3 certified by the metric repair of the same Trotter step (the
 *       clip's shifted test, run with the same s; ntu_trotter_step only)
 *   [10..14] GPU clock cycles spent in: set-up, half-step matrices, solves,
 *            error evaluations, balancing (when a bond's fit is spread over
 *            several workgroups, those of the first, and set-up includes each
 *            half-step's isometry, right-hand side and starting point)
 *   [15] mean conjugate-gradient iterations per certified half-step
 *   [16 + 2i + h]              eps after half-step h of iteration i
 *   [16 + 2 n_iter + 2i + h]   chosen tolerance of that half-step
 *   [16 + 4 n_iter + j]        normalised singular value j (0 beyond Dk)
 */
ntu_status ntu_bond_fit(ntu_ctx* ctx, int batch, const ntu_tensor* g, const ntu_tensor* RX,
                        const ntu_tensor* RY, const ntu_fit_opts* opts, ntu_tensor* MX, ntu_tensor* MY,
                        ntu_tensor* stats);

/*
 * Recombination, Fig. 2(e): X' = QX MX (new leg r), Y' = QY MY (new leg l),
 * written as site tensors (p, t, l, b, r).
 * QX, QY: (batch, p D^3, R) as from ntu_reduce_qr.  MX, MY: (batch, R, D);
 * D is taken from MX.  Xn, Yn: (batch, p, D, D, D, D), compute type, written
 * (must not alias QX/QY).
 */
ntu_status ntu_recombine(ntu_ctx* ctx, int batch, const ntu_tensor* QX, const ntu_tensor* QY,
                         const ntu_tensor* MX, const ntu_tensor* MY, ntu_tensor* Xn, ntu_tensor* Yn);

/* Options of a Trotter step. */
typedef struct ntu_step_opts {
  int n_bonds;          /* number of bond updates in the sweep (<= 8)          */
  int order[8];         /* NTU_BOND_* in sweep order (first order: H1,H2,V1,V2) */
  int precision;        /* NTU_PREC_* for the environment contraction          */
  int fix_mode;         /* NTU_FIX_*                                            */
  ntu_fit_opts fit;
  int scheme;           /* NTU_SCHEME_* (default NTU)                           */
  int graph;            /* 0: launch eagerly.  1: the first call captures the
                           step into a HIP graph kept by the context, and later
                           calls with the same arguments (buffers, batch, D,
                           options) replay it; other arguments capture anew.
                           Not allowed while the caller's stream is itself
                           being captured (NTU_ERR_ARG).                       */
} ntu_step_opts;

void ntu_step_opts_default(ntu_step_opts* o);

/* Number of doubles per item and bond update in the stats of ntu_trotter_step. */
#define NTU_STEP_STATS_LEN(n_iter, D) (8 + NTU_FIT_STATS_LEN(n_iter, D))

/*
 * One Trotter step of the two-site checkerboard iPEPS (Secs. I, III): the
 * bond updates of opts->order, one after another, each a full NTU update
 * (reduce, environment, metric repair, fit, recombination) of the bond in the
 * canonical frame: H1 updates A.r-B.l (X = A, Y = B); H2 updates B.r-A.l;
 * V1 and V2 are H1 and H2 after rotating both tensors by 90 degrees clockwise
 * (new (t, l, b, r) = old (l, b, r, t)), i.e. the bonds A.t-B.b and B.t-A.b.
 * The environment of each update is made of the current A and B.
 * A, B: (batch, p, D, D, D, D) in place, in the compute type, or both
 *   NTU_C64 with a complex context (storage in complex64: read with an
 *   upcast at the start of the step, the sweep runs in complex128, the new
 *   tensors are written back rounded to complex64).  D is taken from A.
 * gate_factors: (batch, 4, 2, d, d, r_g): for bond j (NTU_BOND_*) the
 *   factors (GA, GB) of its gate, GA acting on X.  Items are independent.
 * stats (may be NULL): (batch, n_bonds, NTU_STEP_STATS_LEN) NTU_F64, written:
 *   [0..7] metric stats of the update, then the bond-fit stats.
 * With opts->scheme == NTU_SCHEME_SVDU every update is an SVDU update (no
 *   environment, metric repair or ALS fit; precision, fix_mode and the fit's
 *   n_iter, conv_tol and ladder are not used, kappa is): the fit stats then
 *   hold N = eps = 0, D_n, D_k and the normalised singular values, and the
 *   metric stats [0..7] are not written.
 */
ntu_status ntu_trotter_step(ntu_ctx* ctx, int batch, ntu_tensor* A, ntu_tensor* B,
                            const ntu_tensor* gate_factors, const ntu_step_opts* opts, ntu_tensor* stats);

/*
 * Autotuning of the split-precision environment contraction (launch
 * parameters, not part of the method): the number of K chunks of the final
 * assembly g = L2 Right^T (Fig. 4(d,e)), whose FP64 partial sums are then
 * added, and for NTU_PREC_FP16X3 the width of that assembly's output tiles
 * (128 or 256 columns of the real-embedded g; 128 rows each, eight waves).
 * More chunks and narrower tiles fill the GPU better at small batch; fewer
 * chunks move fewer partial sums, wider tiles read each row of L2 fewer
 * times.  Any choice gives the same metric up to FP64 rounding of the chunk
 * sums.
 *
 * ntu_tune_env times ntu_env_contract on the caller's operands (same
 * arguments; g is overwritten) for every candidate (K split 1 .. 4, and the
 * built-in heuristic's choice when larger; for FP16X3 each with both tile
 * widths), reps timed calls each after one untimed call, with HIP events on
 * the context stream, and synchronises.  It keeps the fastest for
 * (D, precision) in the context, where ntu_env_contract, ntu_trotter_step
 * and ntu_cell_step then use it, and returns its K split in best_ks (and
 * its mean time in best_ms), either may be NULL; ntu_get_env_tile gives its
 * tile width.  The choice is made for this batch size.  Precision must be
 * one of the split precisions (NTU_ERR_ARG otherwise); reps >= 1.  The
 * operands are those of ntu_env_contract (D taken from nbr[0]).
 * ntu_set_env_ksplit sets the K split directly (ks = 0: the heuristic
 * again); ntu_get_env_ksplit returns it (0: the heuristic).
 * ntu_set_env_tile sets the FP16X3 tile width (0: the default, 128 columns;
 * 128 or 256; other precisions NTU_ERR_ARG); ntu_get_env_tile returns it
 * (0: the default).
 * ntu_tune_save writes the context's choices to a text file, one line
 * "D precision ksplit tile_width" each (0: not set); ntu_tune_load reads
 * such a file (or lines of the first three fields) into the context
 * (entries for D > max_D or other precisions are skipped; a malformed line
 * gives NTU_ERR_ARG, after the lines before it are taken).
 */
ntu_status ntu_tune_env(ntu_ctx* ctx, int batch, int precision, const ntu_tensor* QX, const ntu_tensor* QY,
                        const ntu_tensor nbr[6], ntu_tensor* g, int reps, int* best_ks, float* best_ms);
ntu_status ntu_set_env_ksplit(ntu_ctx* ctx, int D, int precision, int ks);
int ntu_get_env_ksplit(ntu_ctx* ctx, int D, int precision);
ntu_status ntu_set_env_tile(ntu_ctx* ctx, int D, int precision, int width);
int ntu_get_env_tile(ntu_ctx* ctx, int D, int precision);
ntu_status ntu_tune_save(ntu_ctx* ctx, const char* path);
ntu_status ntu_tune_load(ntu_ctx* ctx, const char* path);

/*
 * Event profiler (measurement support, not part of the method).  When enabled,
 * the context records a HIP event on its stream before and after every
 * kernel class it launches (events are created here, never inside calls).
 * ntu_profile_read synchronises on the last event, fills ms[k] (summed
 * milliseconds) and count[k] (number of timed launches) for the first n
 * kernel classes, clears the record and returns the number of classes.
 * ntu_profile_kind_name(k) names class k (static string).
 */
ntu_status ntu_profile_enable(ntu_ctx* ctx, int on);
int ntu_profile_read(ntu_ctx* ctx, double* ms, int* count, int n);
const char* ntu_profile_kind_name(int kind);

/*
 * CTMRG expectation values (the corner transfer matrix renormalisation the
 * paper uses for observables, Secs. II, III and V) of the two-site
 * checkerboard state (A, B): A on the sites (x, y) with x + y even, the r leg
 * of (x, y) joined to the l leg of (x + 1, y), the t leg to the b leg of
 * (x, y + 1); bonds H1 = A.r - B.l, H2 = B.r - A.l, V1 = A.t - B.b, V2 =
 * B.t - A.b.  The network is the double layer sum_s conj(T[s']) T[s] of every
 * site (with an operator O[s', s] on the physical index for expectation
 * values), its environment built on a 2 x 2 cell by directional moves: each
 * iteration is four left moves, the lattice turned a quarter turn clockwise
 * after each; a left move absorbs a column into the left environment, the
 * fused legs on each cut between two rows going through the chi leading left
 * singular vectors of rho, the half-system density matrix of the 2 x 2 block
 * around the cut.  Starting boundary: bond dimension 1 with the ket-bra
 * identity on the inner legs.  Computation in complex128 on the GPU (one
 * workgroup per cut for the singular vectors: chi D^2 <= 1024).
 *
 * ntu_ctm_create: for physical dimension p (the full site index: d, d times
 * the ancilla, or the 4 basis operators of the Hermitian purification), bond
 * dimension D <= 8 and environment dimension chi (chi D^2 <= 1024);
 * allocates its device memory once: 96 tensors of max(chi^2 D^2, D^8)
 * complex entries, a scratch arena of
 * 10 chi^2 D^6 + 64 chi^2 D^4 + 2 (chi D^2)^2 + 8 D^8 + 8 p D^4 + 128 entries
 * (16 bytes each; e.g. 0.2 GB at D = 2, chi = 80, 40 GB at D = 8, chi = 16)
 * and 4 MB of partial sums for products split along their sums.
 * NTU_ERR_SHAPE outside those limits, NTU_ERR_HIP if the memory is not
 * there.  After an error of ntu_ctm_run or ntu_ctm_expect the environment
 * is dropped: the next ntu_ctm_run starts from the boundary and
 * ntu_ctm_expect returns NTU_ERR_ARG until then.
 * ntu_ctm_run: n_iter iterations for the state A, B ((p, D, D, D, D),
 * NTU_F64 or NTU_C128, device) from the starting boundary (reset != 0, or
 * the first call) or from the environment of the previous call.
 * ntu_ctm_expect: expectation values in the current environment, written to
 * out ((2 n1 + 4), NTU_C128, device): out[2k], out[2k + 1] = <O_k> at A and
 * at B for the one-site operators ops1 ((n1, p, p), NTU_C128, n1 <= 16, row
 * index s', column s); out[2 n1 + b], b = H1, H2, V1, V2, = <h> for the
 * two-site operator h = sum_t ops2[t, 0] (x) ops2[t, 1] ((n2, 2, p, p),
 * NTU_C128, 1 <= n2 <= 16), the first factor on A.r's site for H1, B's for
 * H2, the lower site for V1 and V2.  Each value is the ratio of the network
 * with the operators inserted to the norm network.
 * All three run on the stream set by ntu_ctm_set_stream (default the null
 * stream).  ntu_ctm_expect does not synchronise; ntu_ctm_run does on its
 * first call (it copies the starting boundary from the host) and, for
 * chi D^2 > 64, inside each cut's SVD (it reads the rotation count of the
 * last Jacobi sweep back between batches of sweeps).  Errors:
 * ntu_ctm_last_error.
 */
typedef struct ntu_ctm ntu_ctm;
ntu_status ntu_ctm_create(ntu_ctm** out, int device, int p, int D, int chi);
ntu_status ntu_ctm_destroy(ntu_ctm* ctm);
ntu_status ntu_ctm_set_stream(ntu_ctm* ctm, void* stream);
const char* ntu_ctm_last_error(const ntu_ctm* ctm);
ntu_status ntu_ctm_run(ntu_ctm* ctm, const ntu_tensor* A, const ntu_tensor* B, int n_iter, int reset);
ntu_status ntu_ctm_expect(ntu_ctm* ctm, const ntu_tensor* A, const ntu_tensor* B, const ntu_tensor* ops1,
                          const ntu_tensor* ops2, ntu_tensor* out);

/*
 * One Trotter sweep of a larger unit cell (Sec. II: the environment of each
 * update is its cluster of nearest neighbours, so updates whose clusters do
 * not touch are independent and run side by side).  The cell holds Lx x Ly
 * distinct site tensors on the torus the cell repeats on; bonds are updated
 * in the given order, each a full NTU (or SVDU) update of bond (x, y, dir):
 * dir 0 joins (x, y).r to (x + 1, y).l (X = (x, y), Y = (x + 1, y)); dir 1
 * joins (x, y).t to (x, y + 1).b and runs in the frame turned a quarter turn
 * clockwise (X = (x, y), Y = (x, y + 1)), as the vertical bonds of
 * ntu_trotter_step.  The cluster of a horizontal bond is L = (x - 1, y),
 * TX = (x, y + 1), BX = (x, y - 1), TY = (x + 1, y + 1), BY = (x + 1, y - 1),
 * Rn = (x + 2, y) (coordinates modulo the cell); of a vertical bond, in the
 * turned frame, L = (x, y - 1), TX = (x - 1, y), BX = (x + 1, y),
 * TY = (x - 1, y + 1), BY = (x + 1, y + 1), Rn = (x, y + 2).
 * Consecutive bonds of the order of which none changes a site of another's
 * cluster are one launch group (at most min(max_batch, 48) bonds): their
 * clusters are gathered into batches, updated by one chain of batched
 * launches and scattered back; since such updates commute, the result is
 * that of updating the bonds one after another.  Order the bonds so that
 * independent ones are adjacent (e.g. horizontal bonds with rows and columns
 * in classes of 3 and 4, then vertical ones) to form large groups.
 * T: (Lx Ly, p, D, D, D, D) in place, the compute type; site (x, y) is item
 *   x + Lx y.  Lx, Ly >= 2, Lx Ly <= 4096.
 * bonds: host array of n_bonds triples (x, y, dir), 0 <= x < Lx,
 *   0 <= y < Ly, in sweep order.
 * gate_factors: (n_bonds, 2, d, d, r_g): bond k's (GA, GB), GA acting on X.
 * opts: precision, fix_mode, fit and scheme as for ntu_trotter_step (n_bonds,
 *   order and graph are not used; the sweep runs eagerly).
 * work: one-dimensional device array of the compute type with at least
 *   8 min(max_batch, 48) p D^4 elements (the gathered clusters).
 * stats (may be NULL): (n_bonds, NTU_STEP_STATS_LEN) NTU_F64, bond k's row as
 *   in ntu_trotter_step.
 * n_groups (host, may be NULL): the launch groups the sweep took.
 * Errors: every argument is checked before anything runs.
 */
ntu_status ntu_cell_step(ntu_ctx* ctx, int Lx, int Ly, ntu_tensor* T, int n_bonds, const int* bonds,
                         const ntu_tensor* gate_factors, const ntu_step_opts* opts, ntu_tensor* work,
                         ntu_tensor* stats, int* n_groups);

/*
 * A time-evolution run measured with CTMRG (Sec. III: the quench from a
 * polarised state, observables from the CTM environment, each run ended once
 * the energy per site has moved away from its initial value by more than a
 * tolerance, 0.01 there).  Measurement 0 is taken before the first step,
 * then one after every measure_every Trotter steps.  A measurement is
 * ntu_ctm_run (ctm_iters iterations from the identity boundary, or from the
 * previous measurement's environment when ctm_continue) and ntu_ctm_expect
 * with ops1 and the bond operator hb; its energy per site is half the real
 * part of the sum of <hb> over the four bonds H1, H2, V1, V2 (each site has
 * two of them; hb carries a quarter of each one-site field on each of its
 * sites).  The run ends after n_steps steps, or after the first measurement
 * whose energy differs from measurement 0's by more than energy_tol (when
 * energy_tol > 0).
 * ctx, ctm: a context and a CTMRG object (ntu_ctm_create with the state's p
 *   and D) on one device.  Every launch goes to the context's stream (the
 *   CTMRG object's stream is set to it for the run and restored after).  The
 *   call waits for that stream at every measurement (the stop decision reads
 *   the energy on the host), so it cannot be captured into a graph.
 * A, B: (1, p, D, D, D, D) NTU_C128 or NTU_F64, evolved in place (one state;
 *   complex64 storage returns NTU_ERR_UNSUPPORTED before anything runs).
 * gate_factors, step: as for ntu_trotter_step with batch 1 (any sweep order,
 *   e.g. the second-order sweep of half-step gates).
 * ops1: (n1, p, p) one-site operators; hb: (n2, 2, p, p) the bond operator
 *   as operator-Schmidt terms, as ntu_ctm_expect takes them.
 * history: (max_meas, 2 n1 + 4) NTU_C128 on the device: row m is measurement
 *   m's ntu_ctm_expect output ([<O_k>_A, <O_k>_B] per operator, then <hb>
 *   on H1, H2, V1, V2); max_meas >= n_steps / measure_every + 1.
 * energy: host array of max_meas doubles (may be NULL): the energies.
 * n_meas, steps_done: host; the measurements written and the steps taken.
 * Errors: arguments are checked before anything runs (NTU_ERR_ARG,
 *   NTU_ERR_SHAPE, NTU_ERR_DTYPE, NTU_ERR_UNSUPPORTED).  An error of a
 *   Trotter step is reported by ntu_last_error(ctx), every other by
 *   ntu_ctm_last_error(ctm); A, B then hold the steps taken (steps_done).
 */
typedef struct ntu_evolve_opts {
  int n_steps;        /* Trotter steps at most (>= 0)                          */
  int measure_every;  /* steps between measurements (>= 1)                     */
  int ctm_iters;      /* CTMRG iterations per measurement (>= 1)               */
  int ctm_continue;   /* 0: each measurement from the identity boundary; 1: from
                         the previous measurement's environment               */
  double energy_tol;  /* stop tolerance on |e - e_0| (<= 0: run every step)   */
} ntu_evolve_opts;

ntu_status ntu_evolve(ntu_ctx* ctx, ntu_ctm* ctm, ntu_tensor* A, ntu_tensor* B, const ntu_tensor* gate_factors,
                      const ntu_step_opts* step, const ntu_evolve_opts* ev, const ntu_tensor* ops1,
                      const ntu_tensor* hb, ntu_tensor* history, double* energy, int* n_meas, int* steps_done);

/*
 * Metric repair without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same operation and kernels as ntu_metric_fix, with
 * no context.  Its scratch space is a device array of
 * NTU_NOALLOC_SCRATCH_BYTES held by the library on every GPU it runs on
 * until the process ends; the call itself allocates nothing.
 * stream: a hipStream_t of the current device (NULL: the null stream).
 * g: (batch, n, n) in place, NTU_F64 or NTU_C128 (which selects real or
 * complex arithmetic), n <= 1024, on the current device.
 * stats (may be NULL): (batch, 8) NTU_F64, written as by ntu_metric_fix.
 * The scratch needed is about 2 n^2 elements of g's type per item (the
 * eigen-solve's two matrices; 3 n^2 doubles for real g with n >= 128, the
 * sign iteration's three): 2 MiB per complex item at n = 256, so up to 16
 * such items per call; larger requests return NTU_ERR_WORKSPACE before any
 * launch.  Errors are described by ntu_last_error(NULL).
 * Every call on one GPU uses that GPU's one scratch array: calls that
 * overlap on a GPU (different streams or threads without ordering between
 * them) race and give wrong results.  Nothing in the scratch needs to start
 * at zero; it keeps the last call's contents.
 */
#define NTU_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
ntu_status ntu_metric_fix_noalloc(void* stream, int batch, ntu_tensor* g, int mode, ntu_tensor* stats);

#ifdef __cplusplus
}
#endif
#endif /* NTU_H */
