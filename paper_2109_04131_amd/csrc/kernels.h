// Internal launch interface between the host driver and the HIP kernels.
#pragma once
#include "common.h"

namespace usfft {

constexpr int kMaxD = 64;          // largest parameter dimension d
constexpr int kMaxMesh = 64;       // largest mesh_n of the on-chip solver
constexpr int kMaxMeshStream = 512;  // largest mesh_n of the streaming solver
constexpr int kStreamBlocks = 512;   // persistent workgroups of the streaming solver
// Largest lattice sizes: the length-(M-1) complex transform of one node
// pair stays in one CU's LDS (150 KB): 9600 float64 or 19200 float32 values.
constexpr int kMaxLattice64 = 9601;
constexpr int kMaxLattice = 19201;

// PDE sampler tables on the device (see sampler.hip).
struct PdeDev {
  int n, d;
  double a0, h2;
  const double* amp;  // d
  const double* tab;  // centroid basis tables (sin or cos per axis), pde_device.h
  int model;          // USFFT_MODEL_*
  double alpha, beta, delta;
  int raw = 0;        // 1: the solver inputs are parameters y, not sampling nodes t
};

// Pitch of the padded x2 tables that follow the four d x n tables: entry
// 1 + cj holds row cj, the ends repeat rows 0 and n - 1, so that any 17
// consecutive rows starting at cj >= -1 (cj < n) are one contiguous read.
__host__ __device__ constexpr int row_tab_pitch(int n) { return n + 16; }

// General triangulation (pcgmesh.hip): CSR pattern of the inner vertices,
// per-entry (triangle, weight) contributions, load, basis at the centroids.
constexpr int kMaxMeshRows = 2048;          // inner vertices the LDS solver holds
constexpr int64_t kMaxMeshLds = 150 << 10;  // LDS of coefficients, values, direction
struct MeshDev {
  int G, nt, nnz;
  const int* rowptr;  // G + 1
  const int* col;     // nnz
  const int* diag;    // G: CSR position of each diagonal entry
  const int* cptr;    // nnz + 1
  const int* ctri;    // contributions: triangle
  const double* cw;   // contributions: |T| grad(phi_a) . grad(phi_b)
  const double* load; // G: sum |T| / 3
  const double* psi;  // d x nt: basis of term k at the centroid of T
};
int64_t mesh_lds_bytes(const MeshDev& M);
bool mesh_fits_lds(const MeshDev& M);             // else the global-scratch solver runs
int64_t mesh_scratch_doubles(const MeshDev& M);  // per workgroup, global-scratch solver
int mesh_persistent_blocks(const MeshDev& M);
void launch_pde_solve_mesh(const PdeDev& P, const MeshDev& M, const double* Y, int64_t ns, double rtol, int maxit,
                           void* out, int out_fp32, int64_t ld, int64_t col0, int* iters, int blocks, double* scr,
                           hipStream_t st);

// ---- sampler.hip
void launch_nodes(int d, int line, int t, int nlat, const int64_t* off, const int32_t* Ms, const int32_t* zs,
                  const double* tail, double* Y, int64_t ns, hipStream_t st);
// step 1: all d x r lines (loff: d r + 1 sample offsets, tails: d r x d)
void launch_line_nodes(int d, int r, const int64_t* loff, const int32_t* Kt, const double* tails, double* Y,
                       int64_t ns, hipStream_t st);
// step 2: nrep copies of a family's nodes with tails nrep x d (copy b at Y + b ns d)
void launch_lattice_nodes_rep(int d, int t, int nlat, const int64_t* off, const int32_t* Ms, const int32_t* zs,
                              const double* tails, double* Y, int64_t ns, int nrep, hipStream_t st);
int solver_config_count();
bool solver_config_fits(int c, int n);  // n = mesh_n
void solver_config_shape(int c, int* block, int* npt);
int solver_default_config(int n);
// Float32 solves run persistent: wscr holds 2 (n+1)^2 (rounded) doubles per
// workgroup for wblocks = persistent_blocks(cfg, n) workgroups.
int persistent_blocks(int cfg, int n);
int64_t edge_scratch_doubles(int n, int blocks);
void launch_pde_solve(int cfg, const PdeDev& P, int precision, const double* Y, int64_t ns, double rtol,
                      int maxit, double inner_rtol, int refine_every, void* out, int out_fp32, int64_t ld,
                      int64_t col0, int* iters, double* wscr, int wblocks, hipStream_t st);
int64_t stream_workspace_doubles(int n, int blocks);
void launch_pde_solve_stream(const PdeDev& P, const double* Y, int64_t ns, double rtol, int maxit, void* out,
                             int out_fp32, int64_t ld, int64_t col0, int* iters, double* ws, int blocks,
                             hipStream_t st);
// ---- pcgdst.hip: DST-preconditioned solver for meshes with n - 1 <= 64
int dst_padded(int n);             // MP = 32 or 64, 0 if the mesh is too large
// streaming DST-preconditioned float64 PCG for 65 < mesh_n <= 129 (pcgdst.hip)
bool dst_stream_ok(int n);
int dst_stream_blocks();
int64_t dst_stream_workspace_doubles(int n, int blocks);
void dst_stream_tables_build(int n, void* frag, float* lam, hipStream_t st);  // MP = 128 fragments and eigenvalues
void launch_pde_solve_dst_stream(const PdeDev& P, const double* Y, int64_t ns, double rtol, int maxit, void* out,
                                 int out_fp32, int64_t ld, int64_t col0, int* iters, double* ws, int blocks,
                                 const void* frag, const float* lam, hipStream_t st);
// streaming PCG with the two-level preconditioner (coarse DST at n / 2) for
// even 129 < mesh_n <= 256 (pcgdst.hip)
bool tl_stream_ok(int n);
int tl_stream_blocks();
int64_t tl_stream_workspace_doubles(int blocks);
void launch_pde_solve_tl_stream(const PdeDev& P, const double* Y, int64_t ns, double rtol, int maxit, void* out,
                                int out_fp32, int64_t ld, int64_t col0, int* iters, double* ws, int blocks,
                                const void* frag, const float* lam, hipStream_t st);
int64_t dst_frag_bytes(int mp);    // S fragment table of one mesh size
void dst_tables_build(int n, void* frag, float* lam, hipStream_t st);  // lam: MP floats
// variant 0: edge grids and scaling in a global scratch slot per workgroup
// (more resident workgroups); 1: all of it in LDS (one workgroup per CU).
int dst_persistent_blocks(int n, int precision, int variant);
int64_t dst_edge_stride(int mp);   // doubles per scratch grid
int64_t dst_scratch_doubles(int n, int variant, int blocks);
// One job's batch of solves in a DST solver launch: samples begin ..
// begin + (next segment's begin) of the launch, sampling nodes Y (rows from
// 0), node g of local sample j written to out[g ld + col0 + j], iteration
// counts to iters[j].  Every segment of a launch has the same mesh; the
// coefficient family (d, amplitudes, model) may differ.
struct SolveSeg {
  PdeDev pde;
  const double* Y;
  void* out;
  int64_t ld, col0, begin;
  int* iters;
};
// segs: device array of nseg segments, ascending begin, segs[0].begin = 0;
// ns = all samples of the launch; n = the segments' mesh_n
void launch_pde_solve_dst(const SolveSeg* segs, int nseg, int n, int precision, int variant, int64_t ns,
                          double rtol, int maxit, double inner_rtol, int refine_every, int out_fp32, double* wscr,
                          int wblocks, const void* frag, const float* lam, hipStream_t st);
// samples at a point set from samples at the mesh's inner vertices (G points,
// three (vertex row or -1, weight) pairs each; um: rows of ldm, same type as out)
void launch_interp(const void* um, int fp32, int64_t ldm, const int32_t* idx, const double* w, int64_t G, int64_t ns,
                   void* out, int64_t ld, int64_t col0, hipStream_t st);
void launch_trigpoly(int d, const double* Y, int64_t ns, const int32_t* K, int64_t np, const double* C,
                     int64_t G, void* out, int out_fp32, int64_t ld, int64_t col0, hipStream_t st);

// ---- fft.hip
// Per-size tables of Rader's algorithm for a prime M with smooth L = M-1.
struct RaderTables {
  void* base = nullptr;       // one block holding every table below
  bool owned = false;         // base was allocated by rader_build
  int M = 0, L = 0, gen = 0;
  int nrad = 0;
  int radix[24] = {0};
  int32_t* perm = nullptr;    // L: gen^q mod M
  int32_t* dlog = nullptr;    // M: q with gen^q = m (entry 0 unused)
  int32_t* outidx = nullptr;  // M: index p with b = gen^(-p) mod M (entry 0 unused)
  // twiddles exp(-2 pi i j q ts / L) of every radix stage s (block size N_s,
  // R_s, M_s = N_s / R_s, ts = L / N_s), stage-major: stage s from
  // element twoff[s], butterfly j's R_s - 1 factors (q = 1 .. R_s - 1)
  // contiguous at j (R_s - 1); at most 2 L elements
  int twoff[24] = {0};
  void* tw64 = nullptr;       // complex double
  void* tw32 = nullptr;       // complex float, the same values rounded
  void* B64 = nullptr;        // L complex double: DFT_L(b) / L, b_j = exp(-2 pi i gen^(-j) / M)
  void* B32 = nullptr;        // L complex float
};
// Radix plan of one length-L transform.
struct FftPlanDev {
  int L, nrad;
  int radix[24];
  int twoff[24];  // first element of each stage's twiddles (RaderTables::twoff)
};
// One lattice DFT of a batched launch: the tables of its size, its samples
// (columns col0 .. col0 + M of every node row), the bins of its candidates
// and where their values go (output column pos[a] or pos_base + a, in the
// block that starts out_off elements into the output).
struct LatItem {
  FftPlanDev F;
  int M;
  const int32_t* dlog;
  const int32_t* outidx;
  const void* tw;  // twiddles and kernel spectrum in the launch's precision
  const void* B;
  int64_t col0;
  const int32_t* bins;
  const int32_t* pos;
  int pos_base, nb;
  int64_t out_off;
};
bool lattice_size_ok(int M);                    // prime, 7-smooth M - 1, M <= kMaxLattice
inline int lattice_mmax_for(int fp32) { return fp32 ? kMaxLattice : kMaxLattice64; }
size_t rader_table_bytes(int M);                        // bytes of one size's tables
// wide: the radix plan of float32 transforms (radices 9 and 16 run two levels
// in registers); float64 transforms keep radices up to 8 (register budget)
void rader_build(RaderTables& T, int M, bool wide, hipStream_t st);  // allocates + fills (synchronous)
void rader_build_at(RaderTables& T, int M, bool wide, void* mem, hipStream_t st);  // fills mem (synchronous)
void rader_free(RaderTables& T);                        // frees what rader_build allocated
// Output column of candidate a: pos[a], or pos_base + a when pos is null.
void launch_lattice_dft(const RaderTables& T, const void* u, int u_fp32, int64_t G, int64_t ld, int64_t col0,
                        const int32_t* bins, const int32_t* pos, int pos_base, int nb, int out_kind, void* out,
                        int64_t ldo, hipStream_t st);
void fill_lat_item(LatItem& it, const RaderTables& T, int u_fp32);  // F, M and the table pointers
// Every item of items_dev (device array) in one launch; Lmax = the largest
// transform length L = M - 1 among them.
// shape_block / shape_cols > 0 choose the workgroup size (128, 256, 512) and
// node pairs per workgroup (1, 2, 4) instead of the built-in rule
void launch_lattice_dft_batch(const LatItem* items_dev, int nitems, int Lmax, const void* u, int u_fp32, int64_t G,
                              int64_t ld, int out_kind, void* out, int64_t ldo, hipStream_t st, int shape_block = 0,
                              int shape_cols = 0);
bool rader_shape_ok(int Lmax, int u_fp32, int block, int cols);
// mask_out bit pos[q] |= mask_in bit q, q < n (grouped order back to candidate order).
void launch_ungroup_mask(const uint32_t* mask_in, const int32_t* pos, int64_t n, uint32_t* mask_out, hipStream_t st);
// all d r step-1 lines at once: line y (coordinate t = y / line_r) from column
// loff[y], K_t = lineK[t] bins from cands (coordinates in order), |X|^2 to
// columns y * line_stride of out (G x ldo, doubles)
void launch_line_dft_lines(const void* u, int u_fp32, int64_t G, int64_t ld, const int64_t* loff,
                           const int32_t* lineK, const int32_t* cands, int nlines, int line_r, int Kmax,
                           int64_t line_stride, double* out, int64_t ldo, hipStream_t st);
void launch_line_dft(const void* u, int u_fp32, int64_t G, int64_t ld, int64_t col0, int K, const int32_t* bins,
                     int nb, int out_kind, void* out, int64_t ldo, hipStream_t st);

// ---- select.hip
// the step-1 lines of launch_line_dft_lines in one launch; line y ORs into
// the mask words of its coordinate (after those of the coordinates before)
void launch_select_lines(const double* v, int64_t G, int64_t ld, int nlines, int line_r, int64_t line_stride,
                         const int32_t* lineK, int Kmax, int s_tilde, const double* theta2, double tie_rel,
                         uint32_t* mask, hipStream_t st);
void launch_select(const double* v, int64_t G, int64_t n, int64_t ld, int s_tilde, const double* theta2,
                   double tie_rel, uint32_t* mask, double* thr, hipStream_t st);
// niter column blocks of n candidates (block b at columns b * iter_stride)
// in one launch, all ORed into the same mask
void launch_select_iters(const double* v, int64_t G, int64_t n, int64_t ld, int niter, int64_t iter_stride,
                         int s_tilde, const double* theta2, double tie_rel, uint32_t* mask, hipStream_t st);
void launch_max_to_theta(const double* v, int64_t G, int64_t n, int64_t ld, double theta, double* theta2,
                         uint64_t* scratch, hipStream_t st);

// ---- sets.hip
void launch_product(const int32_t* parent, int64_t np, int t, const int32_t* child, int64_t nc, int32_t* out,
                    hipStream_t st);
// Compaction; *count_dev receives the row count.
void launch_compact(const int32_t* J, const uint32_t* mask, int64_t n, int t, int32_t* out, int64_t* count_dev,
                    hipStream_t st);
// The T tries of lattice attempt a (one workgroup each): generators z (T x t),
// bins (T x n), alias counts (T x M) and scores (T), all overwritten
void launch_lattice_try(uint64_t seed, int kind, int tcode, int a, int T, int t, int M, const int32_t* J, int64_t n,
                        const uint8_t* covered, int32_t* z, int32_t* bins, int32_t* counts, int32_t* scores,
                        hipStream_t st);
// device choice of one attempt (state: uncovered, taken; log: best, freed) and its commit
void launch_lattice_pick_take(const int32_t* scores, int T, const int64_t* state_in, int64_t* state_out,
                              int32_t* log, const int32_t* bins, const int32_t* counts, uint8_t* covered, int64_t n,
                              int M, int32_t* assign, int32_t* bin_out, hipStream_t st);

// ---- eval.hip
// Y (n x d) holds parameters of the model; T[q * ldt + j] gets phi^{-1}(Y[j]).
void launch_node_map(const double* Y, int64_t n, int d, int model, double alpha, double beta, double delta,
                     double* T, int64_t ldt, hipStream_t st);
// B (2 nI x ldb): cos / -sin rows of 2 pi k_a . t_j
void launch_phases(const int32_t* I, int64_t nI, int d, const double* T, int64_t ldt, int64_t n, double* B,
                   int64_t ldb, hipStream_t st);
// out[j * ldo + g] = Re sum_a c_{a,g} e^{2 pi i k_a . t_j}
void launch_evgemm_values(const double* C, int64_t G, int64_t nI, const double* B, int64_t ldb, int64_t n,
                          double* out, int64_t ldo, hipStream_t st);
int64_t evgemm_tiles_j(int64_t n);
// error partials against U (G x ldu) and their accumulation into acc_s / acc_m
// (psum / pmax: evgemm_tiles_j(n) x G each)
void launch_evgemm_errors(const double* C, int64_t G, int64_t nI, const double* B, int64_t ldb, int64_t n,
                          const double* U, int64_t ldu, double p, double* psum, double* pmax, int first,
                          double* acc_s, double* acc_m, hipStream_t st);
void launch_err_final(double* errp, int64_t G, int64_t n, double p, hipStream_t st);
// D (2 nI) and ord (nI) are scratch; mean (2 G), var (G), gsi (d x G) may be null
void launch_stats(const int32_t* I, int64_t nI, int d, const double* C, int64_t G, int model, double delta,
                  double* D, int32_t* ord, double* mean, double* var, double* gsi, hipStream_t st);

}  // namespace usfft
