/*
 * usfft.h — C ABI of the MI355X (gfx950) uniform sparse FFT hot path.
 *
 * The method is Alg. 1 of Kaemmerer, Potts, Taubert, "The uniform sparse FFT
 * with application to PDEs with random coefficients": a dimension-incremental
 * sparse FFT over the random parameters y that detects ONE frequency set I
 * shared by the functions u(x_g, .) at all G spatial nodes, using one PDE
 * solve per sampling node y for all nodes at once (Sec. 3.1).
 *
 * Conventions for every call:
 *  - Every function returns usfft_status (0 = OK, < 0 = error).  No exception
 *    or abort crosses the ABI; usfft_last_error() returns a thread-local
 *    message describing the last failure.
 *  - "_dev" pointers are device (HIP) memory owned by the caller; "_host"
 *    pointers are host memory owned by the caller.  The library never keeps a
 *    caller pointer beyond the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Work
 *    is enqueued on it; calls that must read sizes back (detect, family,
 *    compact) synchronise that stream before returning.
 *  - A plan holds workspaces: calls on one plan must not overlap (one thread
 *    at a time).  Different plans may run concurrently, each on its own
 *    stream.
 *  - Index sets are int32 row-major (n x t) and lexicographically ordered
 *    where stated.  Coefficient/sample matrices are row-major with an explicit
 *    leading dimension.
 */
#ifndef USFFT_H
#define USFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  USFFT_OK = 0,
  USFFT_EINVAL = -1,    /* bad argument, shape or unsupported size          */
  USFFT_ENOMEM = -2,    /* device or host allocation failed                 */
  USFFT_EHIP = -3,      /* a HIP runtime call failed (message has details)  */
  USFFT_ENOCONV = -4,   /* a PCG solve missed its tolerance within maxit    */
  USFFT_ELATTICE = -5   /* no lattice family within lattice_max attempts    */
} usfft_status;

enum { USFFT_SAMPLER_PDE = 0, USFFT_SAMPLER_TRIG_POLY = 1, USFFT_SAMPLER_PDE_MESH = 2 };
enum { USFFT_FP64 = 0, USFFT_FP32_REFINE = 1 };
enum { USFFT_OUT_MAG2 = 0, USFFT_OUT_COMPLEX = 1 };
enum { USFFT_PRECOND_DST = 0, USFFT_PRECOND_JACOBI = 1 };
/* Coefficient models (Sec. 1) and their periodizations (Sec. 3.2).  The
 * usFFT samples at nodes t in [0,1)^d; the sampler maps them to the model's
 * parameter y and usfft_eval maps evaluation points y back to t:
 *   PERIODIC:  a = a0 + sum_j amp_j sin(2 pi t_j) psi_j,           y = t
 *   AFFINE:    a = a0 + sum_j amp_j y_j psi_j, y_j = phi(t_j), tent
 *              phi(t) = beta - |(beta - alpha)(1 - 2t)| (eq. (3.2)),
 *              t = (y - alpha) / (2 (beta - alpha))
 *   LOGNORMAL: a = a0 + exp(sum_j amp_j y_j psi_j), y_j = sqrt(2) erf^-1(2
 *              tau(t_j)), tau the tent shifted by delta onto [-1/2, 1/2]
 *              (eq. (3.3)), t = erf(y / sqrt(2)) / 4 + delta + 1/4.
 * psi_j(x) = B1(mode1_j pi x1) B2(mode2_j pi x2), B = sin (basis 0) or
 * cos (basis 1) per axis. */
enum { USFFT_MODEL_PERIODIC = 0, USFFT_MODEL_AFFINE = 1, USFFT_MODEL_LOGNORMAL = 2 };

typedef struct usfft_plan_s* usfft_plan_t;
typedef struct usfft_result_s* usfft_result_t;
typedef struct usfft_server_s* usfft_server_t;

/* Problem of Alg. 1 ("Input": Gamma, u, T_G).  All arrays are host memory and
 * are copied by usfft_plan_create.
 *  Gamma = box prod_j [k_lo[j], k_hi[j]] (Alg. 1 input; Table 4.1 uses
 *  [-N, N]^d).
 *  PDE sampler (eq. (1.1), (1.2), periodic model of Sec. 3.2 with
 *  Theta_j(y) = sin(2 pi y_j)):
 *     -div(a grad u) = 1 on (0,1)^2, u = 0 on the boundary,
 *     a(x,y) = a0 + sum_j amp[j] sin(2 pi y_j) sin(mode1[j] pi x1) sin(mode2[j] pi x2),
 *  P1 elements on the uniform mesh h = 1/mesh_n, every cell split along its
 *  (i,j)-(i+1,j+1) diagonal, a evaluated at triangle centroids; T_G = the
 *  G = (mesh_n-1)^2 interior nodes, g = (j-1)(mesh_n-1) + (i-1).
 *  PDE_MESH sampler: the same equation and coefficient family (amp, mode1,
 *  mode2, a0, model, basis) on a general triangulation of the unit square
 *  (the discretisation of the paper's Sec. 4): mesh_nv vertices mesh_xy
 *  (nv x 2), mesh_nt triangles mesh_tri (nt x 3 vertex indices), mesh_boundary
 *  (nv bytes, nonzero = Dirichlet vertex).  T_G = the other vertices in vertex
 *  order; a at triangle centroids; float64 Jacobi-PCG per sample, with the
 *  sample's matrix and vectors in LDS up to G = 2048 inner vertices and
 *  8 (nt + nnz + G) <= 150 KB, else in a plan-owned global scratch of
 *  8 (nnz + nt + 7 G) bytes per resident workgroup (two per CU).
 *  TRIG_POLY sampler (test functions of Theorem 1.1):
 *     u_g(y) = Re sum_{a<n_poly} c[a,g] exp(2 pi i poly_k[a].y),
 *  poly_c is n_poly x G x 2 doubles (re, im). */
typedef struct {
  int32_t d;
  const int32_t* k_lo;
  const int32_t* k_hi;
  int32_t sampler;
  /* PDE */
  int32_t mesh_n;        /* 4 <= mesh_n <= 512                               */
  double a0;
  const double* amp;     /* d                                                */
  const int32_t* mode1;  /* d                                                */
  const int32_t* mode2;  /* d                                                */
  /* TRIG_POLY */
  int64_t G_poly;
  int64_t n_poly;
  const int32_t* poly_k; /* n_poly x d                                       */
  const double* poly_c;  /* n_poly x G_poly x 2                              */
  /* PDE coefficient model (all zero: the periodic model with sine modes)   */
  int32_t model;         /* USFFT_MODEL_*                                    */
  double alpha, beta;    /* AFFINE: parameter interval, alpha < beta         */
  double delta;          /* LOGNORMAL: tent shift in (0, 1/2); <= 0 takes
                            1/(4 M_max), M_max = lattice_mmax (Lemma 3.1 for
                            the largest admissible lattice: no lattice or
                            line node falls on a pole of the map)            */
  int32_t basis1, basis2;/* 0: sin, 1: cos along x1 / x2                     */
  /* PDE_MESH (the PDE fields above give the coefficient; mesh_n unused)     */
  int32_t mesh_nv, mesh_nt;
  const double* mesh_xy;          /* nv x 2                                  */
  const int32_t* mesh_tri;        /* nt x 3, vertex indices                  */
  const uint8_t* mesh_boundary;   /* nv, nonzero: boundary (u = 0) vertex    */
  /* Node set T_G given by points (Sec. 3.1: the solver's values at nodes
   * that are not mesh vertices are interpolated).  n_nodes = 0: T_G = the
   * mesh's inner vertices (as above).  n_nodes > 0 (PDE and PDE_MESH
   * samplers): T_G = the points nodes_xy (n_nodes x 2, in [0,1]^2); every
   * sample is the P1 solution at the points, sum over the vertices of the
   * containing triangle of barycentric coordinate x vertex value (0 at
   * boundary vertices), computed on the device from the solve at the mesh
   * vertices.  G = n_nodes everywhere (results, usfft_sample rows, eval).
   * EINVAL for points outside the domain or the triangulation. */
  int64_t n_nodes;
  const double* nodes_xy;
} usfft_problem;

/* Parameters of Alg. 1 ("Input": s, s_local, Algorithm A, theta, r) and of
 * this implementation. */
typedef struct {
  int32_t s, s_local, r;   /* sparsity parameters and detection iterations   */
  double theta;            /* threshold                                      */
  int32_t theta_relative;  /* 1: theta_abs = theta * max |c| of stage t=1,i=1 */
  double tie_rel;          /* values within tie_rel of tau_g^2 are ties (2^-30) */
  int32_t precision;       /* USFFT_FP64 or USFFT_FP32_REFINE                */
  double lattice_c;        /* lattice size factor c (2)                      */
  int32_t lattice_tries;   /* generator candidates per attempt (8)           */
  int32_t lattice_max;     /* attempts before USFFT_ELATTICE (64)            */
  int32_t lattice_mmax;    /* largest lattice size (<= 9601; FP32_REFINE:
                              <= 19201, the float32 transform of one node
                              pair then fills one CU's LDS)                  */
  double pcg_rtol;         /* relative residual of every solve (1e-12)       */
  int32_t pcg_maxit;       /* PCG iterations per solve (or inner solve)      */
  double inner_rtol;       /* FP32_REFINE: float32 residual drop that triggers
                              a float64 true-residual replacement (2e-4:
                              the fastest at h = 1/64 with the DST solver)  */
  int32_t refine_every;    /* FP32_REFINE: a float64 true residual at least
                              every this many iterations (200)              */
  int32_t solver_config;   /* Jacobi solver: -1 autotune at plan time, -2
                              built-in choice, >= 0 force that shape.
                              DST solver: < 0 default (2 for FP32_REFINE, 1
                              for FP64); 0 edge grids in global scratch, 1
                              LDS-resident, 2 compact float32 (float32 edges
                              in LDS, float64 edges in global scratch for the
                              true residual; FP32_REFINE only)             */
  int32_t precond;         /* USFFT_PRECOND_DST (fast-Poisson preconditioner:
                              on chip for mesh_n <= 65, with the CG vectors
                              in a global workspace and float64 arithmetic
                              for 65 < mesh_n <= 129; for even
                              129 < mesh_n <= 256 two-level, scaled Jacobi
                              plus the fast-Poisson solve on the mesh of
                              width 2h) or USFFT_PRECOND_JACOBI; odd meshes
                              above 129 and meshes above 256 use the
                              streaming Jacobi solver                        */
  int32_t trace;           /* nonzero: usfft_detect keeps the detected sets of
                              every increment (usfft_result_trace); costs one
                              small readback per increment                  */
  int32_t autotune;        /* nonzero: time the candidates of every kernel
                              choice not yet in the tuning cache (the DST
                              solver's scratch variant at plan creation when
                              solver_config < 0, the lattice-DFT workgroup
                              shape per transform length on first use) and
                              keep the fastest; 0: cached or built-in
                              choices.  Choices change only rounding (bin 0
                              of a transform, the solver's arithmetic within
                              pcg_rtol); a saved cache makes them repeatable */
} usfft_params;

/* Statistics of one usfft_detect run. */
typedef struct {
  int64_t samples;          /* PDE solves (sampling nodes) used              */
  int64_t samples_step1;
  int64_t samples_step2;
  int64_t samples_step3;
  int64_t lattices;         /* rank-1 lattices over all families             */
  int64_t max_candidates;   /* largest |J_t|                                 */
  int64_t pcg_iterations;   /* sum over solves (inner iterations for FP32)   */
  int64_t sample_launches;  /* sampler kernel launches                       */
  int64_t dft_launches;     /* line + lattice DFT kernel launches            */
  int64_t solver_block;     /* workgroup size of the PDE solver              */
  int64_t solver_npt;       /* mesh nodes per thread of the PDE solver       */
  int64_t solver_kind;      /* 0 DST-preconditioned PCG, 1 Jacobi PCG on
                               chip, 2 streaming Jacobi PCG, 3 general-mesh
                               Jacobi PCG, 4 streaming DST-preconditioned
                               PCG (65 < mesh_n <= 129), 5 streaming
                               two-level PCG (even 129 < mesh_n <= 256),
                               -1 no PDE solve                               */
  double theta_abs;         /* absolute threshold used                       */
  double ms_sample;         /* device time in the sampler kernels            */
  double ms_dft;            /* device time in DFT kernels                    */
  double ms_select;         /* device time in selection kernels              */
  double ms_total;          /* wall time of the call                         */
  double dft_bytes;         /* algorithmic bytes moved by lattice DFTs       */
  int64_t max_batch;        /* largest sampler batch (samples in one launch) */
  int64_t max_family;       /* largest lattice family (samples of one
                               iteration): the smallest samples_max of the
                               _ws calls that runs this job                  */
  int64_t workspace_bytes;  /* _ws calls: bytes of the caller's workspace the
                               bounds took (usfft_plan_workspace's value)    */
  int64_t plan_reused;      /* server jobs: 1 when the job ran on a pooled
                               plan of an earlier job                        */
} usfft_stats;

const char* usfft_last_error(void);
const char* usfft_version(void);

/* Tuning cache (process-wide; see usfft_params.autotune): usfft_tune_save
 * writes it as JSON ({"version": 1, "entries": [{"key", "a", "b",
 * "time_ms"}, ...]}), usfft_tune_load merges such a file into it (entries of
 * the file win), usfft_tune_clear empties it.  Keys name the choice and its
 * shape: "jacobi n= d= prec=" (a = Jacobi solver shape), "dst n= d= prec=
 * model=" (a = DST solver scratch variant), "rader L= fp32= G=" (a =
 * workgroup size, b = node pairs per workgroup of the lattice DFT).
 * Errors: EINVAL (unreadable or malformed file). */
usfft_status usfft_tune_save(const char* path);
usfft_status usfft_tune_load(const char* path);
usfft_status usfft_tune_clear(void);

/* Plan: validate and copy the problem, upload static tables (coefficient
 * tables of eq. (1.2) at triangle centroids, polynomial coefficients), size
 * nothing data-dependent yet.  Errors: EINVAL, ENOMEM, EHIP. */
usfft_status usfft_plan_create(const usfft_problem* prob, const usfft_params* par,
                               usfft_plan_t* out);
void usfft_plan_destroy(usfft_plan_t plan);
/* G of the plan's node set T_G. */
int64_t usfft_plan_nodes(usfft_plan_t plan);

/* Alg. 1, steps 1 to 3, on the device.  Output: the detected set I
 * (lexicographic) and the coefficients c_k(u_{x_g}), k in I, for every node
 * (Alg. 1 "Output").  Synchronises `stream`.  With the environment variable
 * USFFT_LOG set to a non-zero value, one progress line per step and per
 * increment t goes to stderr (candidates, lattices, samples, kept
 * frequencies, elapsed seconds).  Errors: ENOCONV, ELATTICE, ENOMEM, EHIP. */
usfft_status usfft_detect(usfft_plan_t plan, uint64_t seed, void* stream,
                          usfft_result_t* out);

/* Caller-provided device workspace (Alg. 1 "Input"/"Output" unchanged).
 * usfft_plan_workspace returns the bytes of device memory that
 * usfft_detect_ws / usfft_coefficients_ws need on this plan for jobs whose
 * candidate sets (every |J_t| and the output set) have at most n_cand_max
 * entries and whose sampler batches hold at most samples_max samples (a
 * batch is one lattice family of an increment, repeated for as many of its r
 * iterations as fit; step 1 always runs as one batch of r sum_t K_t line
 * samples, which the size includes; a smaller samples_max only splits the
 * r iterations over more sampler launches, down to one family per launch).
 * A run reports its largest |J_t|, batch and family in usfft_stats
 * (max_candidates, max_batch, max_family).
 * The _ws calls carve every transient buffer (sample matrix, magnitudes,
 * sets, lattice-planner state) and the output coefficient matrix from ws_dev
 * (256-byte aligned, ws_bytes long, owned by the caller) and allocate no
 * device memory: the plan already holds its static tables and the lattice
 * tables of every admissible size (built into that memory on first use).
 * The result's coefficients live in the workspace: they stay valid while the
 * caller keeps the workspace and does not reuse it for another call.
 * Results are the same as usfft_detect / usfft_coefficients.  Errors: ENOMEM
 * (ws_bytes below the size for these bounds, or a job that exceeds them:
 * the message names the bound), EINVAL, ENOCONV, ELATTICE, EHIP. */
usfft_status usfft_plan_workspace(usfft_plan_t plan, int64_t n_cand_max, int64_t samples_max,
                                  size_t* bytes);
usfft_status usfft_detect_ws(usfft_plan_t plan, uint64_t seed, int64_t n_cand_max, int64_t samples_max,
                             void* ws_dev, size_t ws_bytes, void* stream, usfft_result_t* out);
usfft_status usfft_coefficients_ws(usfft_plan_t plan, const int32_t* freqs_host, int64_t n, uint64_t seed,
                                   int64_t n_cand_max, int64_t samples_max, void* ws_dev,
                                   size_t ws_bytes, void* stream, usfft_result_t* out);

/* Several jobs (one plan each, distinct plans) run together: each on its own
 * thread and stream, with the PDE solves of every sampler batch fused across
 * the jobs.  Whenever a job needs solves it waits until every other job
 * still running needs its next batch of solves (or has finished); then one
 * persistent solver launch per class of jobs (same mesh_n, precision, DST
 * solver variant and solver tolerances; the coefficient family, d, box, s
 * and the batch sizes may differ) serves all of their batches through a
 * table of (job, sample
 * range) segments.  Jobs whose plans do not use the DST-preconditioned
 * solver run alone, unfused.  Results are those of usfft_detect on each job
 * alone (a solve does not depend on its batch).  out[i] receives job i's
 * result (NULL if it failed), statuses[i] (may be NULL) its status;
 * fuse_stats (may be NULL): solver launches, launches that served more than
 * one job, and job segments over all launches.  Returns after every job has
 * finished: USFFT_OK, or the status of the first failed job.  1 <= n <= 64. */
usfft_status usfft_detect_batch(usfft_plan_t* plans, int32_t n, const uint64_t* seeds,
                                usfft_result_t* out, usfft_status* statuses, int64_t* fuse_stats);

/* Step 3 of Alg. 1 alone on a given frequency set (Sec. 4.5: a-priori index
 * sets such as axis crosses, hyperbolic crosses and weighted l1 balls):
 * freqs_host (n x d int32, row-major, no repeated rows; any order) replaces
 * the detected set, and its coefficients for every node are computed with the
 * multiple rank-1 lattice family of step 3 (seeded like usfft_detect's
 * step 3).  The result lists the frequencies in the caller's order; n = 0
 * gives an empty result.  The plan's sampler, mesh, precision and lattice
 * parameters apply; s, s_local, r and theta are not used.
 * Errors: EINVAL (repeated rows), ENOCONV, ELATTICE, ENOMEM, EHIP. */
usfft_status usfft_coefficients(usfft_plan_t plan, const int32_t* freqs_host, int64_t n,
                                uint64_t seed, void* stream, usfft_result_t* out);

usfft_status usfft_result_info(usfft_result_t res, int64_t* n_freq, int32_t* d,
                               int64_t* G, usfft_stats* stats);
/* freqs_host: n_freq x d int32 (lexicographic); coeffs_host: n_freq x G x 2
 * doubles (re, im), may be NULL. */
usfft_status usfft_result_copy(usfft_result_t res, int32_t* freqs_host, double* coeffs_host);
/* Detection trace of a usfft_detect result made with params.trace != 0: the
 * intermediate sets of Alg. 1.  stage in [0, d): the 1-D set I^(t) of step
 * 1&2a, t = stage + 1 (width 1, n_cand = K_t, the box extent); stage in
 * [d, 2d - 1): the set I^(1..t) of step 2e, t = stage - d + 2 (width t,
 * n_cand = |J_t| = |I^(1..t-1)| |I^(t)|), lexicographic.  *n receives the
 * set size; set_host (n x width int32) may be NULL to query sizes first.
 * Errors: EINVAL (no trace kept, stage out of range). */
usfft_status usfft_result_trace(usfft_result_t res, int32_t stage, int64_t* n, int32_t* width,
                                int64_t* n_cand, int32_t* set_host);
/* Destroys a result.  Its device coefficient buffer goes back to a per-device
 * pool of the library (up to 1 GiB in all) for later results, after a device
 * synchronization (as a device free would do); beyond the pool it is freed.
 * NULL is ignored. */
void usfft_result_destroy(usfft_result_t res);

/* Evaluation formula of Sec. 3.1 (eq. (3.1) with the model's inverse
 * periodization of Sec. 3.2, see USFFT_MODEL_*):
 * out_dev[j*G + g] = Re sum_{k in I} c_k(u_{x_g}) exp(2 pi i k.phi^{-1}(y_j)),
 * y_dev: n x d doubles, parameters of the model (periodic: nodes in [0,1)).
 * Computed as a float64 matrix product on the matrix cores in chunks of
 * points.  Device workspace of at most ~256 MB (the frequency set, uploaded
 * once, plus each chunk's points and phases) stays with the result: it is
 * allocated on the first call, grown when a later call needs more, reused
 * otherwise and freed by usfft_result_destroy.  Calls on one result
 * (usfft_eval, usfft_statistics, usfft_errors) are serialised by the
 * library.  Returns after the stream has finished.  Errors: EINVAL, ENOMEM,
 * EHIP. */
usfft_status usfft_eval(usfft_result_t res, const double* y_dev, int64_t n,
                        double* out_dev, void* stream);

/* usfft_eval without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same evaluation and the same kernels, with the
 * frequency set, the mapped points and the phase matrix of each chunk held
 * in a fixed 64 MiB device array of the library instead of the result's
 * evaluation workspace (which usfft_eval allocates on a result's first
 * call and grows when a call needs more).  Limit: the frequency set (n_freq x d int32, padded to 256
 * bytes) plus 64 points x (d + 2 n_freq) doubles must fit in 64 MiB, i.e.
 * up to about 65 000 frequencies; larger results give EINVAL and leave the
 * output untouched.  Each GPU holds one such array for the life of the
 * process (looked up on its first call on that device), and every call on
 * that GPU shares it: calls that overlap on one GPU (other threads, other
 * streams) race and must be serialised by the caller.  Returns after the
 * stream has finished.  Errors: EINVAL, EHIP. */
usfft_status usfft_eval_noalloc(usfft_result_t res, const double* y_dev, int64_t n,
                                double* out_dev, void* stream);

/* Statistics of the approximation per node (Sec. 4, Sec. 4.1), from the
 * result's coefficients alone.  Device outputs, each may be NULL:
 *   mean_dev[2g], [2g+1]  Re, Im of E(u_usFFT(x_g, .)) = sum_k c_k D_k, with
 *                         D_k = [k = 0] (periodic), prod_j D_{k_j},
 *                         D_{k_j} = 2i/(pi k_j) for odd k_j, 1 for k_j = 0,
 *                         0 otherwise (affine), times e^{2 pi i k_j delta}
 *                         (lognormal, delta of the problem);
 *   var_dev[g]            variance sum_{k != 0} |c_k|^2;
 *   gsi_dev[(l-1)*G + g]  global sensitivity index of J_l = {k : exactly l
 *                         nonzero components}, l = 1..d (0 where the
 *                         variance is 0).
 * Uses the result's evaluation workspace (see usfft_eval).  Returns after
 * the stream has finished.  Errors: EINVAL, ENOMEM, EHIP. */
usfft_status usfft_statistics(usfft_result_t res, double* mean_dev, double* var_dev,
                              double* gsi_dev, void* stream);

/* Error measures of Sec. 4 over n test parameters y_dev (n x d doubles in
 * the model's parameter domain, drawn by the caller from its distribution):
 * finite-element solves of plan's problem at each y (float64 results; the
 * plan's solver and precision), the approximation at the same y, and per node
 *   errp_dev[g]   = ( (1/n) sum_j |u_FE(x_g, y_j) - u_usFFT(x_g, y_j)|^p )^(1/p),
 *   errinf_dev[g] = max_j |u_FE(x_g, y_j) - u_usFFT(x_g, y_j)|.
 * res must come from a plan of the same problem (same d and G).  p >= 1.
 * Works in chunks of points, in the result's evaluation workspace (see
 * usfft_eval; up to ~1.3 GB here).
 * Returns after the stream has finished.  Errors: EINVAL, ENOMEM, ENOCONV
 * (a test solve missed pcg_rtol), EHIP. */
usfft_status usfft_errors(usfft_plan_t plan, usfft_result_t res, const double* y_dev,
                          int64_t n, double p, double* errp_dev, double* errinf_dev,
                          void* stream);

/* ---- Stage entry points: each step of the hot path as its own call ---- */

/* Black-box sampler (Sec. 2.1; Alg. 1 steps 1&2a and 2c): one solve per row
 * of y_dev (n x d doubles, sampling nodes t in [0,1)^d, mapped to the model's
 * parameter by the periodization of Sec. 3.2), sample of node g written to
 * u_dev[g*ld + col0 + row] as float64 (out_fp32 = 0) or float32 (1).  With
 * the plan's precision: FP64 = float64 PCG; FP32_REFINE = float32 PCG with
 * float64 reliable updates (preconditioner per params.precond).  iters_dev
 * (n int32, may be NULL) receives the iteration count of each solve (-1 = not
 * converged).  Errors: EINVAL (ld < col0 + n), ENOCONV, EHIP. */
usfft_status usfft_sample(usfft_plan_t plan, const double* y_dev, int64_t n,
                          void* u_dev, int32_t out_fp32, int64_t ld, int64_t col0,
                          int32_t* iters_dev, void* stream);

/* Sampling nodes of one stage (Alg. 1 step 1&2a: l/K in coordinate `line`,
 * tail elsewhere; step 2b / step 3: rank-1 lattice nodes (m z mod M)/M in the
 * first t coordinates (App. A), tail in the others).  line >= 0 selects the
 * 1-D form with K = M_host[0]; otherwise nlat lattices with sizes M_host and
 * generators z_host (nlat x t).  Writes y_dev (sum M x d doubles). */
usfft_status usfft_nodes(int32_t d, int32_t line, int32_t t, int32_t nlat,
                         const int32_t* M_host, const int32_t* z_host,
                         const double* tail_host, double* y_dev, void* stream);

/* Length-K DFT of Alg. 1 step 1&2a for every node: for candidate a with
 * bin b_a = bins_host[a] mod K,
 *   F = (1/K) sum_l u[g*ld + col0 + l] exp(-2 pi i l b_a / K),
 * read through the canonical bin min(b, K-b) (conjugated above K/2).
 * out: USFFT_OUT_MAG2 -> |F|^2 doubles at out_dev[g*ldo + a];
 *      USFFT_OUT_COMPLEX -> (re, im) doubles at out_dev[(a*G + g)*2]. */
usfft_status usfft_line_dft(const void* u_dev, int32_t u_fp32, int64_t G, int64_t ld,
                            int64_t col0, int32_t K, const int32_t* bins_host, int32_t nb,
                            int32_t out_kind, void* out_dev, int64_t ldo, void* stream);

/* Lattice DFT of Algorithm A (App. A): the length-M DFT of every node's
 * samples along a rank-1 lattice of prime size M (M-1 7-smooth)
 * evaluated at the requested bins (same normalisation, canonical-bin rule
 * and output layouts as usfft_line_dft; candidate a written at column
 * pos_dev[a] of the output).  bins_dev, pos_dev: nb int32 device arrays.
 * M <= 9601 for float64 samples, <= 19201 for float32 samples.
 * Errors: EINVAL (M not admissible). */
usfft_status usfft_lattice_dft(const void* u_dev, int32_t u_fp32, int64_t G, int64_t ld,
                               int64_t col0, int32_t M, const int32_t* bins_dev,
                               const int32_t* pos_dev, int32_t nb, int32_t out_kind,
                               void* out_dev, int64_t ldo, void* stream);

/* Algorithm A alone (App. A): the coefficients of the candidates J_dev
 * (n x t int32 device array, row-major) read from one rank-1 lattice of
 * prime size M (M - 1 7-smooth; M <= 9601, or 19201 with float32 samples)
 * with generator z_host (t int64,
 * host): for every node g and candidate a with bin b_a = k_a.z mod M
 * (computed here in exact 64-bit arithmetic),
 *   out_dev[(a G + g) 2 + {0,1}] = Re, Im of (1/M) sum_m u[g ld + col0 + m]
 *                                  exp(-2 pi i m b_a / M),
 * read through the canonical bin min(b, M - b) (conjugated above M/2).  u_dev
 * holds the samples at the lattice nodes (m z mod M)/M, m < M, node-major
 * (float64, or float32 with u_fp32 = 1).  A coefficient is exact for
 * functions supported on candidates whose bins no other candidate shares.
 * Synchronises `stream`.  Errors: EINVAL. */
usfft_status usfft_lattice_coeffs(const void* u_dev, int32_t u_fp32, int64_t G, int64_t ld,
                                  int64_t col0, int32_t M, int32_t t, const int64_t* z_host,
                                  const int32_t* J_dev, int64_t n, double* out_dev, void* stream);

/* Per-node selection and uniform union (Alg. 1 step 1&2a and 2d/2e): for
 * every node g, tau_g^2 = s_tilde-th largest of v_dev[g*ld + a], a < n
 * (0 when n < s_tilde); keep a when v >= max(theta2, (1 - tie_rel) tau_g^2);
 * mask_dev (ceil(n/32) words, bit a) |= OR over g of keep.  theta2 is read
 * from the device scalar theta2_dev.  thr_dev (G doubles, may be NULL)
 * receives the per-node threshold. */
usfft_status usfft_select(const double* v_dev, int64_t G, int64_t n, int64_t ld,
                          int32_t s_tilde, const double* theta2_dev, double tie_rel,
                          uint32_t* mask_dev, double* thr_dev, void* stream);

/* Join (Alg. 1 step 2): Cartesian product J = parent x child in parent-major
 * order (lexicographic when both inputs are): out_dev (np*nc) x (t+1). */
usfft_status usfft_product(const int32_t* parent_dev, int64_t np, int32_t t,
                           const int32_t* child_dev, int64_t nc, int32_t* out_dev,
                           void* stream);

/* Compaction of a detected set (Alg. 1 step 2e): rows of J_dev (n x t) whose
 * mask bit is set, order kept.  *count_host receives the number of rows. */
usfft_status usfft_compact(const int32_t* J_dev, const uint32_t* mask_dev, int64_t n,
                           int32_t t, int32_t* out_dev, int64_t* count_host, void* stream);

/* Algorithm A's sampling set for a candidate set (App. A; multiple rank-1
 * lattices, Remark 4.2): greedy family on J_dev (n x t), reading of this
 * build: sizes = admissible primes from min(max(3, ceil(c n)), mmax/2) up to
 * mmax (cycled), `tries` SplitMix64 generators per attempt (stream kind
 * `kind`, t-code `tcode`), keep the one freeing most uncovered candidates
 * (lowest try on ties), drop lattices that free none.  Outputs: *nlat_host,
 * M_host (cap entries), z_host (cap x t), assign_dev / bins_dev (n int32:
 * lattice index and bin k.z mod M of each candidate).  Errors: ELATTICE,
 * EINVAL (cap too small). */
usfft_status usfft_family(const int32_t* J_dev, int64_t n, int32_t t, double c, int32_t mmax,
                          int32_t tries, int32_t lmax, uint64_t seed, int32_t kind,
                          int32_t tcode, int32_t cap, int32_t* nlat_host, int32_t* M_host,
                          int32_t* z_host, int32_t* assign_dev, int32_t* bins_dev,
                          void* stream);

/* ---- Serving: continuous batching of whole usFFT jobs ----
 * A server runs up to max_active jobs at once, each on its own worker thread
 * and non-blocking HIP stream, so the kernels of different jobs overlap on the
 * device.  Jobs are admitted in arrival order as soon as a slot is free and
 * their estimated device footprint fits in hbm_budget bytes next to the
 * running jobs and the idle plans (the estimate, from G, s, the box and the
 * precision, bounds the sample matrix and candidate magnitudes of the largest
 * stage).  A finished job's plan, with its tables and workspaces, stays in a
 * pool (at most 2 max_active idle plans; the oldest are freed first when an
 * admission needs their memory) and serves the next job of the same sampler,
 * coefficient family, mesh, node set, precision and solver parameters; the
 * box, s, s_local, r, theta and the lattice-planner parameters are set per
 * job.  A job's result stays with the server until taken by
 * usfft_server_poll.  Each job's result is the same as running it alone on a
 * new plan (all per-sample and per-node arithmetic is independent of what
 * else runs, and every workspace is rewritten before it is read). */
typedef struct {
  int32_t max_active;   /* concurrent jobs (>= 1)                            */
  uint64_t hbm_budget;  /* bytes the running jobs may occupy (0 = no limit)  */
} usfft_server_cfg;

usfft_status usfft_server_create(const usfft_server_cfg* cfg, usfft_server_t* out);
/* Copies problem and params; returns the job id.  Errors: EINVAL (the job
 * alone exceeds hbm_budget, or invalid problem). */
usfft_status usfft_server_submit(usfft_server_t srv, const usfft_problem* prob, const usfft_params* par,
                                 uint64_t seed, uint64_t* job);
/* Non-blocking (wait = 0) or blocking (wait = 1) completion check.  When the
 * job has finished: *out receives the result (ownership passes to the caller;
 * NULL if the job failed), *job_status the job's status, *latency_s the time
 * from submit to completion and *queue_s the time spent waiting for
 * admission; the call returns USFFT_OK.  When still pending (wait = 0) *out
 * is set to NULL and the call returns USFFT_OK with *job_status = 1. */
usfft_status usfft_server_poll(usfft_server_t srv, uint64_t job, int32_t wait, usfft_result_t* out,
                               int32_t* job_status, double* latency_s, double* queue_s);
/* Waits for every submitted job, then stops the workers; untaken results are
 * destroyed. */
void usfft_server_destroy(usfft_server_t srv);

#ifdef __cplusplus
}
#endif
#endif /* USFFT_H */
