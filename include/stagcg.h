/*
 * stagcg.h - C ABI of libstagcg.so, the MI355X (gfx950) staggered-fermion CG library.
 *
 * The library solves (4 m^2 - D_eo D_oe) x_e = b_e, where D is the staggered
 * Dirac operator of Kim and Lee, "Multi GPU Performance of Conjugate Gradient
 * Algorithm with Staggered Fermions" (Lattice 2010): Eq. (5) with the staggered
 * phases folded into the links (Sec. 2), plus a three-hop (Naik) term with
 * coefficient c_N, and Eq. (3) written on even sites.  The solver is the CG of
 * Fig. 1, optionally with mixed-precision storage and reliable updates (the
 * mixed precision that Sec. 5 announces), batching of many right-hand sides and
 * lattices, and a learned preconditioner inside flexible CG.
 *
 * Conventions shared by every entry point
 *  - dims = {Lx, Ly, Lz, Lt}; each even and >= 2.  Direction mu = 0..3 is x, y, z, t.
 *  - Staggered phase eta_mu(n) = (-1)^(n_0 + ... + n_{mu-1}); time may be
 *    antiperiodic, in which case a forward hop of length k from n picks up
 *    (-1)^floor((n_t + k) / Lt).
 *  - Link fields (inputs to stag_load_links): device complex128
 *    [4][Lt][Lz][Ly][Lx][3][3] (real, imaginary interleaved); element [mu][n] is
 *    U_mu(n), which multiplies the colour vector at n + mu (one-hop "fat" field)
 *    or at n + 3 mu (three-hop "long" field).
 *  - Colour-vector fields on one parity: device complex128 [nrhs][V/2][3],
 *    site index cb = lex >> 1 with lex = x + Lx (y + Ly (z + Lz t)); parity of a
 *    site is (x + y + z + t) mod 2.
 *  - Streams: every call enqueues its device work on `stream` (a hipStream_t
 *    passed as void*, NULL = the null stream).  stag_dslash and stag_apply_m are
 *    asynchronous; the solvers synchronise before returning.
 *  - Ownership: the caller owns every pointer it passes.  The library copies and
 *    repacks links during stag_load_links; the inputs may be freed once the
 *    stream has passed the call.  A lattice owns its packed links and all solver
 *    workspace; stag_destroy_lattice frees them.
 *  - Errors: every call returns a stag_status.  Arguments are validated before
 *    any side effect (STAG_ERR_ARG).  HIP failures return STAG_ERR_HIP.  The
 *    message of the last failure on the calling thread is stag_last_error().
 *    No exception crosses the ABI.
 *  - Thread safety: calls on different lattices may run concurrently; calls on
 *    one lattice must be serialised by the caller.
 */
#ifndef STAGCG_H
#define STAGCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stag_lattice_s* stag_lattice_t;
typedef struct stag_net_s* stag_net_t;

typedef enum {
  STAG_OK = 0,
  STAG_ERR_ARG = 1,            /* invalid argument (null pointer, bad size, odd extent, unpacked precision) */
  STAG_ERR_HIP = 2,            /* a HIP runtime call failed */
  STAG_ERR_NOMEM = 3,          /* device allocation failed */
  STAG_ERR_STATE = 4,          /* call out of order (e.g. dslash before load_links) */
  STAG_ERR_NOT_CONVERGED = 5,  /* max_iter or max_restarts reached; x holds the last iterate */
  STAG_ERR_NAN = 6             /* a NaN/Inf or a non-positive d^dag A d appeared in a reduction */
} stag_status;

typedef enum { STAG_F64 = 0, STAG_F32 = 1, STAG_F16 = 2 } stag_prec;
#define STAG_PREC_BIT(p) (1u << (p))
/* stag_load_links flag: the three-hop links are SU(3) matrices; store two rows each (12 real
 * parameters) and rebuild the third as (a x b)^* (Sec. 3.3, Eq. SU3rec), which moves 16% fewer bytes
 * per Dslash.  Only correct for special unitary long links; needs lng != NULL and naik_coeff != 0
 * (STAG_ERR_ARG otherwise). */
#define STAG_LONG_SU3 (1u << 8)

typedef enum { STAG_PRECOND_NONE = 0, STAG_PRECOND_NET = 1 } stag_precond;

/* Solver parameters.  Fill with stag_cg_params_default() and then override. */
typedef struct {
  double tol;                /* target true residual ||b - M x|| / ||b|| (default 1e-10) */
  int32_t max_iter;          /* inner iterations per restart; <= 0: 3V/2 (the dimension N_dim of Fig. 1) */
  int32_t prec;              /* stag_prec of the inner iteration; STAG_F64 = plain CG of Fig. 1 */
  int32_t reliable_interval; /* mixed precision: at most this many iterations between FP64 residual
                                recomputations ("reliable updates", default 50) */
  double reliable_delta;     /* mixed precision: also update once ||r|| fell below reliable_delta times its value
                                at the previous update (default 0.1; <= 0 disables this trigger) */
  int32_t check_interval;    /* iterations between host convergence polls (default 16) */
  int32_t max_restarts;      /* true-residual restarts after the iterated residual converged (default 5) */
  int32_t precond;           /* stag_precond; STAG_PRECOND_NET runs flexible CG (single problem only) with the
                                network as preconditioner, then plain CG if it stalls or breaks down */
  stag_net_t net;            /* network for STAG_PRECOND_NET (built on the solve's lattice) */
  int32_t stall_window;      /* FCG: every stall_window iterations (default 10) the smallest ||r|| seen so far
                                is compared with the smallest seen one window earlier; if it did not fall
                                below stall_ratio times that value, plain CG finishes from the current x.
                                The test follows the window's last residual update and precedes the next
                                network application, so a right-hand side handed over costs no extra one */
  double stall_ratio;        /* default 0.9 */
  int32_t profile;           /* k > 0: time the Dslash launches of every k-th inner iteration with HIP events
                                (stag_cg_info.dslash_ms); each timed iteration idles the GPU for a few us
                                per event, so k of 10 or more keeps the solve time representative */
  int32_t history_len;       /* record the first history_len (alpha, beta) pairs per RHS into history */
  double* history;           /* host [nrhs][history_len][2] or NULL */
  int32_t autotune;          /* 1: time the Dslash launch shapes on first use of a (lattices, nrhs, prec) key
                                (a mixed-precision solve also tunes the FP64 key of its reliable updates) */
  int32_t reserved[7];
} stag_cg_params;

/* Per right-hand side result of a solve. */
typedef struct {
  int32_t iters;             /* inner iterations summed over restarts */
  int32_t restarts;          /* true-residual restarts taken */
  int32_t n_reliable;        /* mixed precision: FP64 residual recomputations */
  int32_t fell_back;         /* FCG: 1 if the preconditioner stalled and plain CG finished the solve */
  int32_t converged;         /* 1 if true_resid <= tol */
  int32_t status;            /* stag_status of this right-hand side */
  double true_resid;         /* ||b - M x|| / ||b|| of the returned x, computed in FP64 on the GPU */
  double ms;                 /* wall time of the whole call (same for every RHS of a call) */
  double dslash_ms;          /* profile>0: summed time of the timed inner-iteration Dslash launches: the two
                                launches of one operator application are bracketed by one event pair, and
                                pairs whose right-hand sides had all stopped are left out */
  int32_t dslash_calls;      /* profile>0: number of launches in that time */
  int32_t dslash_prec;       /* precision of the timed Dslash launches (inner iteration precision) */
  double dslash_sites;       /* profile>0: output sites x RHS processed per timed launch, averaged */
  int32_t dslash_wg;         /* launch shape used by the inner-iteration Dslash: sites per workgroup */
  int32_t dslash_rhs;        /* ... right-hand sides per lane */
  int32_t dslash_lds;        /* ... LDS staging of the x/y neighbour window (1) or not (0) */
  int32_t dslash_order;      /* ... the tile order (0 lattice order, 1 XCD blocks, 2 time streaming) */
  int32_t dslash_chunks;     /* ... and its z blocks per XCD (order 1) or time chunks (order 2) */
} stag_cg_info;

/* A Dslash launch shape and its measured time. */
typedef struct {
  int32_t wg;                /* output sites per workgroup: 64, 128 or 256 */
  int32_t rhs_per_lane;      /* right-hand sides each lane applies a loaded link to: 1, 2, 4 or 8,
                                dividing nrhs */
  int32_t lds_stage;         /* 1: the workgroup first copies the colour vectors of sites
                                [first - 3 Lx/2, last + 3 Lx/2] into LDS and reads its x and y
                                neighbours from there (same result); needs
                                rhs_per_lane x (wg + 3 Lx) x bytes-per-vector <= 64 KiB */
  int32_t tile_order;        /* 0: workgroups take tiles in lattice order (t slowest); 1: the z extent
                                is cut into 8 t_chunks blocks, t_chunks per XCD, and each XCD sweeps t
                                through one block after the other, so that its L2 still holds the
                                t-neighbour slices; needs Lz divisible by 8 t_chunks and wg dividing
                                Ly x Lx / 2.  Same result.
                                2: time streaming (FP16 only): each wave owns 64 sites of the slice plane
                                and one time parity and walks t, so that every input slice is used in the
                                step it is loaded; needs wg 64, rhs_per_lane 8 (one lane per site) or 4
                                (two lanes per site, 32 sites per wave), nrhs divisible by 8, Lx Ly Lz / 2
                                divisible by 64 / (8 / rhs_per_lane) and Lt by 2 t_chunks.  Same Dslash
                                result as 0 and 1 */
  int32_t t_chunks;          /* tile_order 1: z blocks per XCD (1, 2, 3, ...); tile_order 2: the time
                                extent is walked in this many chunks (1, 2, 4, ...); tile_order 0:
                                ignored (0 or 1) */
  double us;                 /* average launch time (stag_tune_dslash), 0 if not timed */
} stag_shape;

/* One problem of a batched solve: a lattice with its own right-hand sides and masses. */
typedef struct {
  stag_lattice_t lat;
  int32_t nrhs;
  const double* mass;        /* host [nrhs] */
  const void* b;             /* device complex128 [nrhs][V/2][3] */
  void* x;                   /* device complex128 [nrhs][V/2][3]; in: initial guess, out: solution */
} stag_problem;

void stag_cg_params_default(stag_cg_params* prm);

/* Lattice geometry (Sec. 2: the even-odd decomposition of the operator).
 * dims: host int32[4] = {Lx, Ly, Lz, Lt}, each even and >= 2, product < 2^31.
 * t_antiperiodic: 1 = antiperiodic time direction, 0 = periodic.
 * Uses the current HIP device; the lattice stays bound to it. */
stag_status stag_create_lattice(const int32_t dims[4], int32_t t_antiperiodic, stag_lattice_t* out);
stag_status stag_destroy_lattice(stag_lattice_t lat);
stag_status stag_lattice_info(stag_lattice_t lat, int32_t dims[4], int64_t* half_volume);

/* Fold the phases, boundary signs and c_N into the links and repack them (Sec. 2,
 * Eq. (5): the staggered phases are absorbed into the stored links; Sec. 3.1
 * coalesced layout).
 * fat, lng: device complex128 link fields (layout above); lng = NULL drops the
 * three-hop term, leaving the paper's one-hop Eq. (5).  naik_coeff: c_N (-1/24
 * for the improved action).  prec_mask: STAG_PREC_BIT of every storage precision
 * to build (FP64 is always built: the true residual needs it), optionally or'ed with STAG_LONG_SU3.
 * Replaces any previously loaded links. */
stag_status stag_load_links(stag_lattice_t lat, const void* fat, const void* lng, double naik_coeff,
                            uint32_t prec_mask, void* stream);

/* out = D_{p,1-p} in (Eq. (5) restricted to output parity p = out_parity).
 * in: device complex128 [nrhs][V/2][3] on parity 1-p; out: same shape on parity p;
 * in and out must not overlap.  prec selects the stored links and the
 * arithmetic: STAG_F64 computes in FP64; STAG_F32 / STAG_F16 round `in` to that
 * storage format, compute in FP32 and return the rounded result widened to
 * complex128. */
stag_status stag_dslash(stag_lattice_t lat, int32_t out_parity, const void* in, void* out,
                        int32_t nrhs, int32_t prec, void* stream);

/* The Dslash of one time slab, for domain decomposition along t (the paper's multi-GPU split,
 * Sec. 4; one GPU per slab, here exercised on one GPU): out = D_{p,1-p} in on the slices
 * [t0, t0 + lt) only, the input read from an extended field that holds the 3 slices before t0, the lt
 * slices, and the 3 slices after (indices mod Lt) - what a GPU owning the slab holds once its two
 * 3-slice faces (the Naik term's depth) have arrived from its neighbours.  A face is contiguous in
 * the even-odd layout (slices are the slowest index), so the exchange is one copy per face.
 * t0, lt: even, lt >= 2, t0 + lt <= Lt.  in_ext: device complex128 [nrhs][(lt + 6) * S][3] on parity
 * 1-p, S = Lx Ly Lz / 2 sites per slice and parity; out: [nrhs][lt * S][3] on parity p; not
 * overlapping.  The links are the lattice's own (loaded for the whole lattice); prec as stag_dslash.
 * The result equals the rows [t0 S, (t0 + lt) S) of stag_dslash bit for bit. */
stag_status stag_dslash_slab(stag_lattice_t lat, int32_t out_parity, int32_t t0, int32_t lt, const void* in_ext,
                             void* out, int32_t nrhs, int32_t prec, void* stream);

/* Time-slice sums for the staggered pion correlator of point-source propagators (the paper's closing
 * remarks: the solver runs in production for hadron spectra).  For a source on an even site x0 with
 * colour c, chi = (4m^2 - D_eo D_oe)^{-1} delta solves Eq. (3) and the propagator of M = 2m + D is
 * G_e = 2m chi, G_o = -D_oe chi; the correlator C(t) sums |G|^2 over time slice t, the sink colour and
 * the three source colours.  This call computes, for each group g of `group` consecutive right-hand
 * sides of v and each time slice t,
 *   out[g][t] = (accumulate ? out[g][t] : 0) + weight * sum_{r in g} sum_{sites of slice t} |v_r|^2,
 * so that C = slice_norm2(chi, 3, 4m^2) followed by slice_norm2(D_oe chi, 3, 1, accumulate).  The sites
 * of one slice and parity are a contiguous even-odd range, so v may hold either parity.
 * v: device complex128 [nrhs][V/2][3]; out: device double [nrhs / group][Lt]; group divides nrhs.
 * Summation order is fixed (same result for every call).  NULL pointers, group not dividing nrhs, a
 * non-finite weight or accumulate not 0/1: STAG_ERR_ARG. */
stag_status stag_slice_norm2(stag_lattice_t lat, const void* v, int32_t nrhs, int32_t group, double weight,
                             int32_t accumulate, double* out, void* stream);

/* The pion correlator of nsrc point-source propagators in one call: chi holds the even-site solutions
 * of the three source colours of each source (3 nsrc consecutive right-hand sides, as for
 * stag_slice_norm2); the library forms G_o = -D_oe chi with its FP64 Dslash and writes
 *   out[s][t] = 4 m^2 sum_{c, slice t} |chi_(3s+c)|^2 + sum_{c, slice t} |(D_oe chi_(3s+c))|^2.
 * chi: device complex128 [3 nsrc][V/2][3]; out: device double [nsrc][Lt]; mass: the solve's m.
 * Asynchronous on `stream`; the odd-parity temporary is lattice workspace (grown on demand).
 * NULL pointers, nsrc < 1 or a non-finite mass: STAG_ERR_ARG. */
stag_status stag_pion_correlator(stag_lattice_t lat, const void* chi, int32_t nsrc, double mass, double* out,
                                 void* stream);

/* out = M in = 4 m^2 in - D_eo D_oe in on even sites (Eq. (3)), FP64.
 * mass: host double[nrhs]; in, out: device complex128 [nrhs][V/2][3], not overlapping. */
stag_status stag_apply_m(stag_lattice_t lat, const double* mass, const void* in, void* out,
                         int32_t nrhs, void* stream);

/* Link fattening: the one-hop (fat) and three-hop (long) link fields that stag_load_links takes, built
 * from a thin gauge field.  The paper's operator (Sec. 1 and Sec. 2: the improved staggered action of
 * the MILC ensembles) uses smeared one-hop links and three-hop Naik links but does not give the
 * smearing; this is the published asqtad recipe (Orginos, Toussaint and Sugar 1999; Lepage 1999):
 *   fat_mu  = 5/8 U_mu + 1/16 (3-link staples) + 1/64 (5-link) + 1/384 (7-link) - 1/16 (Lepage paths),
 *             every path of l links scaled by u0^(1-l) (u0 = 1: no tadpole factor);
 *   long_mu(n) = U_mu(n) U_mu(n + mu) U_mu(n + 2 mu)  (pass naik = -1/(24 u0^2) to stag_load_links).
 * Periodic in every direction (the antiperiodic time sign belongs to the operator).  FP64.
 * thin, fat, lng: device complex128 [4][Lt][Lz][Ly][Lx][3][3] (the stag_load_links layout), pairwise
 * non-overlapping; fat and lng are written.  Workspace: six link fields (144 B per site each) of
 * lattice workspace, grown on demand and freed with the lattice.  Asynchronous on `stream`.
 * The lattice needs no links loaded.  NULL pointers, overlap or u0 not finite and > 0: STAG_ERR_ARG. */
stag_status stag_fatten_links(stag_lattice_t lat, const void* thin, double u0, void* fat, void* lng,
                              void* stream);

/* stag_apply_m without any allocation, for callers that cannot allocate device memory (code under
 * stream or graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * result as stag_apply_m (the same kernels, so the same bits).  The odd-parity temporary and the
 * launch's parameter block live in a fixed array of 64 MiB per GPU, compiled into the library and
 * held until the process ends; the call only launches kernels (no allocation, memset or host copy).
 * Limits: 1 <= nrhs <= 64 and nrhs * V/2 * 48 bytes <= 64 MiB - 16 KiB, else STAG_ERR_ARG.
 * Every lattice and stream on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (different streams, or different host threads) race and give undefined results; calls ordered on
 * one stream are safe.  Other errors as stag_apply_m. */
stag_status stag_apply_m_noalloc(stag_lattice_t lat, const double* mass, const void* in, void* out,
                                 int32_t nrhs, void* stream);

/* Solve M x = b for each right-hand side by the CG of Fig. 1 (prm->prec = STAG_F64),
 * by mixed-precision CG with reliable updates (STAG_F32 / STAG_F16), or by flexible
 * CG with a network preconditioner (prm->precond).  Every solve ends with the
 * FP64 true residual ||b - M x|| / ||b||, and restarts from x while it exceeds tol.
 * mass: host double[nrhs]; b: device complex128 [nrhs][V/2][3]; x: same shape, the
 * initial guess on entry (zero it for a cold start) and the solution on return.
 * info: host [nrhs], filled on every return but STAG_ERR_ARG.  Returns STAG_OK if
 * every RHS converged, otherwise the first failing RHS's status. */
stag_status stag_cg_solve(stag_lattice_t lat, const double* mass, const void* b, void* x, int32_t nrhs,
                          const stag_cg_params* prm, stag_cg_info* info, void* stream);

/* Solve several problems (lattices of different shapes, each with its own
 * right-hand sides and masses) as one batch: every CG stage is one launch over
 * all problems.  probs: host [nprob], nprob <= 16, each lattice at most once (merge its
 * right-hand sides), all with the same long-link storage (STAG_LONG_SU3 or not);
 * info: host [sum of nrhs], in problem order.  Network preconditioning is for
 * single-problem solves only. */
stag_status stag_cg_solve_batch(int32_t nprob, const stag_problem* probs, const stag_cg_params* prm,
                                stag_cg_info* info, void* stream);

/* Autotuner of the Dslash launch shape (multi-right-hand-side batching, Sec. 3.4's occupancy tuning
 * done by measurement).  stag_tune_dslash times every candidate shape for `nrhs` right-hand sides in
 * precision `prec` on this lattice (on library-owned scratch vectors, on `stream`), keeps the fastest
 * for later stag_dslash / stag_cg_solve calls with the same key, and returns it in *best; if all is
 * non-NULL, up to max_all timed candidates are written there and their count to *n_all.
 * stag_set_dslash_shape pins *shape (host; its us is ignored) for the key; shape NULL or shape->wg = 0
 * removes the entry; a combination stag_shape rules out is STAG_ERR_ARG.  The table is process-wide;
 * stag_tune_cache_save / _load write and read it as JSON (path: a host C string). */
stag_status stag_tune_dslash(stag_lattice_t lat, int32_t prec, int32_t nrhs, stag_shape* best, stag_shape* all,
                             int32_t max_all, int32_t* n_all, void* stream);
stag_status stag_set_dslash_shape(stag_lattice_t lat, int32_t prec, int32_t nrhs, const stag_shape* shape);
stag_status stag_tune_cache_save(const char* path);
stag_status stag_tune_cache_load(const char* path);

/* Learned preconditioner (the project's third change to the method; the paper has none): a
 * gauge-covariant linear network.  Layer l maps ch[l] to ch[l+1] colour-vector channels on the full
 * lattice, y_c(n) = sum_c' [W_0 psi_c'(n) + sum_{d=1..8} W_d (T_d psi_c')(n)] with T_{+mu}, T_{-mu} the
 * parallel transports along the one-hop links (phases and boundary signs folded in, as in Eq. (5)).
 * Channels run 1 -> channels -> ... -> channels -> 1; the input is an even-site vector embedded on the
 * full lattice, the output its restriction to even sites.  Activations are complex64.
 * Weights (host) are complex128, concatenated per layer as [9][ch[l+1]][ch[l]] with direction order
 * d = 0 (site), 1..4 (+x,+y,+z,+t), 5..8 (-x,-y,-z,-t).
 * The network needs the lattice's FP32 links (stag_load_links with STAG_PREC_BIT(STAG_F32)); it keeps
 * pointers into them, so reload links only with the same lattice and destroy nets before the lattice.
 * channels: 1, 2, 4 or 8; layers in [1, 16]; seed: initial weights. */
#define STAG_NET_HERMITIAN 1u  /* tie the second half of the layers to the adjoints of the first half in reverse
                                  order, N = K^dag K: Hermitian positive semi-definite, as CG needs of a
                                  preconditioner (layers must be even) */
stag_status stag_net_create(stag_lattice_t lat, int32_t layers, int32_t channels, uint32_t flags, uint64_t seed,
                            stag_net_t* out);
stag_status stag_net_destroy(stag_net_t net);
stag_status stag_net_num_weights(stag_net_t net, int64_t* n_complex);
/* set: with STAG_NET_HERMITIAN the second half of the layers is rederived from the first half. */
stag_status stag_net_set_weights(stag_net_t net, const double* w, int64_t n_complex);   /* host complex128 */
stag_status stag_net_get_weights(stag_net_t net, double* w, int64_t n_complex);
/* out = N(in) for nrhs even-site vectors: device complex128 [nrhs][V/2][3]; in and out must not overlap. */
stag_status stag_net_apply(stag_net_t net, const void* in, void* out, int32_t nrhs, void* stream);
/* Training losses over pairs (b_i, x_i = M^{-1} b_i) (gradients are per layer, every layer's weights
 * treated as independent; the trainer adds the tied layers' gradients):
 *   loss_kind 0 (solution):  L = sum_i ||N(b_i) - x_i||^2 / ||x_i||^2
 *   loss_kind 1 (residual):  L = sum_i ||M (N(b_i) - x_i)||^2 / ||b_i||^2 = sum_i ||M N(b_i) - b_i||^2 / ||b_i||^2,
 *                            M = 4 mass^2 - D_eo D_oe applied in FP64 (weights the modes a local
 *                            network can represent; kind 0 is dominated by the lowest modes).
 * stag_net_loss_grad returns L and, if grad is not NULL, dL/dconj(W) in the weight layout (host
 * complex128); b, x: device complex128 [npairs][V/2][3].  Synchronises. */
stag_status stag_net_loss_grad(stag_net_t net, const void* b, const void* x, int32_t npairs, int32_t loss_kind,
                               double mass, double* loss, double* grad, void* stream);

typedef struct {
  int32_t epochs;            /* passes over the training pairs (default 10) */
  int32_t batch;             /* pairs per optimiser step (default 8) */
  double lr;                 /* Adam step size (default 1e-3) */
  double beta1, beta2, eps;  /* Adam moments (0.9, 0.999, 1e-8) */
  uint64_t seed;             /* shuffling of the pairs (default 1) */
  int32_t loss_kind;         /* 0: solution error, 1: residual (see stag_net_loss_grad; default 1) */
  int32_t reserved0;
  double mass;               /* mass of M for loss_kind 1 */
  int32_t reserved[6];
} stag_train_params;

typedef struct {
  double loss_first;         /* mean loss over the pairs in the first epoch */
  double loss_last;          /* ... in the last epoch */
  int32_t epochs;
  int32_t steps;             /* optimiser steps taken */
  double ms;                 /* wall time */
} stag_train_info;

void stag_train_params_default(stag_train_params* prm);
/* Train the weights with Adam on (b_i, x_i = M^{-1} b_i) pairs (device complex128 [npairs][V/2][3]),
 * minimising the loss of stag_net_loss_grad.  Synchronises. */
stag_status stag_net_train(stag_net_t net, const void* b, const void* x, int32_t npairs,
                           const stag_train_params* prm, stag_train_info* info, void* stream);

/* Measurement helper (not part of the solver): stream `bytes` of device memory at buf with 16-byte
 * non-temporal loads, one 32 KiB chunk per single-wave workgroup, all loads of a lane in flight at once,
 * and write one XOR-folded word per chunk to sink (device uint32 [bytes / 32768]).  It is the read-only
 * HBM ceiling the bandwidth-bound kernels are compared with.  bytes must be a positive multiple of
 * 32768; NULL pointers or another size: STAG_ERR_ARG.  Asynchronous on `stream`. */
stag_status stag_stream_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* stag_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STAGCG_H */
