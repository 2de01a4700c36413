// Host driver of the usFFT hot path and the C ABI (include/usfft.h).
//
// Alg. 1 is run stage by stage on one HIP stream: every step (sampling nodes,
// PDE solves, DFTs, selection, union, join, lattice alias tests) is a kernel;
// the host only draws the SplitMix64 numbers of the stage, keeps the
// lattice-family greedy loop (it needs the per-try scores back) and sizes
// buffers from the set sizes it reads back once per dimension increment.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <fstream>
#include <functional>
#include <sstream>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "kernels.h"
#include "rng.h"

namespace usfft {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }


// ---------------------------------------------------------------- buffers
// Owning device buffer; move-only so that swaps and container moves never
// duplicate (and later double-free) an allocation.
// A borrowed buffer is a slice of a caller's workspace: it never grows (a
// larger request is USFFT_ENOMEM) and is never freed.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool borrowed = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), borrowed(o.borrowed) {
    o.p = nullptr;
    o.bytes = 0;
    o.borrowed = false;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      borrowed = o.borrowed;
      o.p = nullptr;
      o.bytes = 0;
      o.borrowed = false;
    }
    return *this;
  }
  void borrow(void* q, size_t b) {
    release();
    p = q;
    bytes = b;
    borrowed = true;
  }
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (borrowed)
      throw Error{USFFT_ENOMEM, "the caller's workspace is too small: a buffer of " + std::to_string(bytes) +
                                    " bytes needs " + std::to_string(b) +
                                    " (raise n_cand_max / samples_max of usfft_plan_workspace)"};
    if (p) USFFT_HIP(hipFree(p));
    p = nullptr;
    bytes = 0;
    const size_t nb = std::max<size_t>(b, 256);
    const hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error{USFFT_ENOMEM, "device allocation of " + std::to_string(nb) + " bytes failed"};
    }
    bytes = nb;
  }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
  void release() {
    if (p && !borrowed) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    borrowed = false;
  }
  ~DevBuf() { release(); }
};

struct FuseGroup;

struct Family {
  std::vector<int> M;
  std::vector<int32_t> z;  // nlat x t
  std::vector<int64_t> off;
  std::vector<int32_t> lat_first, lat_count;  // slices of the grouped (pos, bin) lists
  // the family's offsets, sizes and generators on the device (uploaded with
  // the grouped lists by group_by_lattice)
  const int64_t* d_off = nullptr;
  const int32_t* d_M = nullptr;
  const int32_t* d_z = nullptr;
  int t = 0;
  int64_t total() const { return off.empty() ? 0 : off.back(); }
};

}  // namespace usfft

struct usfft_plan_s {
  usfft_problem prob{};
  usfft_params par{};
  std::vector<int32_t> k_lo, k_hi, mode1, mode2, poly_k;
  std::vector<double> amp, poly_c;
  int64_t G = 0;
  int solver_cfg = 0;
  // static device tables
  usfft::DevBuf d_amp, d_tab, d_polyk, d_polyc, d_stream, d_wscr, d_sfrag, d_lam;
  // general triangulation
  usfft::DevBuf m_rowptr, m_col, m_diag, m_cptr, m_ctri, m_cw, m_load, m_psi;
  // node set T_G given by points (Sec. 3.1): the solver's values at the
  // mesh's inner vertices (G_mesh of them, in Umesh) are interpolated to the
  // G points through three (inner vertex or -1, weight) pairs per point
  bool interp = false;
  int64_t G_mesh = 0;
  usfft::DevBuf d_iidx, d_iw, Umesh;
  // the one-segment table of this plan's own DST solver launches
  usfft::DevBuf segbuf;
  // set while the plan runs in usfft_detect_batch: DST solver launches go
  // through the batch's rendezvous and are fused with the other jobs'
  usfft::FuseGroup* fuse = nullptr;
  usfft::MeshDev mesh{};
  int mesh_blocks = 0;
  // pinned staging of small uploads: a copy from it needs no host wait; the
  // arena is reused only after a stream synchronisation
  char* stage = nullptr;
  size_t stage_cap = 0, stage_used = 0;
  // pinned landing buffer of small readbacks (valid until the next readback)
  char* back = nullptr;
  size_t back_cap = 0;
  std::vector<char> back_host;
  usfft::DevBuf famlog, famstate;
  int wblocks = 0;  // persistent workgroups of the float32 / DST solver
  bool streaming = false;  // mesh larger than the on-chip solvers hold
  bool dst_stream = false; // 65 < mesh_n <= 129: streaming DST-preconditioned solver
  bool tl_stream = false;  // even 129 < mesh_n <= 256: streaming two-level solver
  bool dst = false;        // DST-preconditioned solver
  int dst_variant = 1;     // 0: scratch in global memory, 1: LDS-resident, 2: compact float32
  usfft::PdeDev pde{};
  // Rader tables per lattice size, built on first use into the plan's table
  // arena (every admissible size up to lattice_mmax has its slot, sized at
  // plan creation, so no call allocates them later)
  std::map<int, usfft::RaderTables> rader;
  std::map<int, size_t> rader_off;
  usfft::DevBuf d_rader;
  // caller workspace mode (usfft_detect_ws / usfft_coefficients_ws): every
  // transient buffer is a borrowed slice; sampler batches hold at most
  // ws_nsamp samples
  bool ws_mode = false;
  int64_t ws_nsamp = 0, ws_ncand = 0;
  // workspaces (grown on demand, kept across calls)
  usfft::DevBuf Y, U, V, iters, cnt, theta2, scratch, J, Jnext, Iprev, mask, gmask, cands, assign, famz, fambins,
      famcounts, famcov, famscores, lists, latM, latoff, tail, latitems;
  std::vector<usfft::DevBuf> I1;  // step-1 sets per coordinate
  std::vector<int64_t> I1n;
  std::mutex mu;
  ~usfft_plan_s() {
    if (stage) (void)hipHostFree(stage);
    if (back) (void)hipHostFree(back);
  }
};

struct usfft_result_s {
  int dev = -1;  // device of C when it came from the result buffer pool
  int32_t d = 0;
  int64_t G = 0;
  int32_t model = USFFT_MODEL_PERIODIC;  // evaluation maps y back to the node t
  double alpha = -1.0, beta = 1.0, delta = 0.0;
  std::vector<int32_t> I;  // n x d
  usfft::DevBuf C;         // n x G x 2 doubles
  usfft_stats stats{};
  // detection trace (params.trace): the step-1 sets I^(t), t = 1..d, then the
  // step-2 sets I^(1..t), t = 2..d, each with its width and candidate count
  std::vector<std::vector<int32_t>> trace_set;
  std::vector<int32_t> trace_width;
  std::vector<int64_t> trace_cand;
  // evaluation state kept across usfft_eval / _statistics / _errors calls:
  // the frequency set on the device (uploaded on first use) and grow-only
  // workspaces, so repeated calls allocate nothing; emu serialises the calls
  std::mutex emu;
  bool Iup = false;
  usfft::DevBuf Idev;
  usfft::DevBuf ews[8];
};

namespace usfft {

// ---------------------------------------------------------------- helpers
// Coefficient buffers of destroyed results, kept per device for the next
// results (at most kResultPoolBytes in all): a job then neither allocates its
// output nor pays its predecessor's free.  A buffer is handed back after a
// device synchronization, as a free would do, so no kernel still reads it.
struct PooledBuf {
  int dev;
  void* p;
  size_t bytes;
};
constexpr size_t kResultPoolBytes = size_t(1) << 30;
static std::mutex g_rpool_mu;
static std::vector<PooledBuf>* const g_rpool = new std::vector<PooledBuf>();  // never destroyed
static size_t g_rpool_bytes = 0;

static void result_buffer(usfft_result_s* R, size_t need) {
  DevBuf& C = R->C;
  if (C.borrowed || C.bytes >= need) {
    C.ensure(need);
    return;
  }
  int dev = 0;
  USFFT_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_rpool_mu);
    int best = -1;
    for (int i = 0; i < (int)g_rpool->size(); ++i) {
      const PooledBuf& b = (*g_rpool)[i];
      if (b.dev == dev && b.bytes >= need && b.bytes <= 2 * need + (size_t(1) << 20) &&
          (best < 0 || b.bytes < (*g_rpool)[best].bytes))
        best = i;
    }
    if (best >= 0) {
      C.release();
      C.p = (*g_rpool)[best].p;
      C.bytes = (*g_rpool)[best].bytes;
      g_rpool_bytes -= C.bytes;
      g_rpool->erase(g_rpool->begin() + best);
      R->dev = dev;
      return;
    }
  }
  C.ensure(need);
  R->dev = dev;
}

static void result_recycle(usfft_result_s* R) {
  DevBuf& C = R->C;
  if (!C.p || C.borrowed || R->dev < 0) return;
  std::lock_guard<std::mutex> lk(g_rpool_mu);
  if (g_rpool_bytes + C.bytes > kResultPoolBytes) return;  // the destructor frees it
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return;
  if (cur != R->dev && hipSetDevice(R->dev) != hipSuccess) return;
  const bool idle = hipDeviceSynchronize() == hipSuccess;
  if (cur != R->dev) (void)hipSetDevice(cur);
  if (!idle) return;
  g_rpool->push_back(PooledBuf{R->dev, C.p, C.bytes});
  g_rpool_bytes += C.bytes;
  C.p = nullptr;
  C.bytes = 0;
}

static const RaderTables& rader_for(usfft_plan_s* P, int M, hipStream_t st) {
  auto it = P->rader.find(M);
  if (it != P->rader.end()) return it->second;
  auto o = P->rader_off.find(M);
  USFFT_REQUIRE(o != P->rader_off.end(), USFFT_EINVAL, "lattice size " + std::to_string(M) + " has no table slot");
  RaderTables T;
  rader_build_at(T, M, P->par.precision == USFFT_FP32_REFINE, P->d_rader.as<char>() + o->second, st);
  return P->rader.emplace(M, T).first->second;
}

// The admissible lattice sizes in [lo, hi], from a table built once.
static std::vector<int> admissible_sizes(int lo, int hi) {
  static const std::vector<int> all = [] {
    std::vector<int> v;
    for (int m = 3; m <= kMaxLattice; ++m)
      if (lattice_size_ok(m)) v.push_back(m);
    return v;
  }();
  return std::vector<int>(std::lower_bound(all.begin(), all.end(), std::max(lo, 3)),
                          std::upper_bound(all.begin(), all.end(), hi));
}

// Largest sample matrix (bytes) one batched sampler launch of step 2 fills.
constexpr uint64_t kSampleBatchBytes = 4ull << 30;

// Small per-stage uploads; synchronous because the host vectors are reused.
template <typename T>
static void h2d(usfft::DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  b.ensure(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!v.empty()) {
    USFFT_HIP(hipMemcpyAsync(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, st));
    USFFT_HIP(hipStreamSynchronize(st));
  }
}

// Upload through the plan's pinned arena, asynchronously on st.
template <typename T>
static void h2d_async(usfft_plan_s* P, usfft::DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  const size_t bytes = sizeof(T) * v.size();
  b.ensure(std::max<size_t>(bytes, sizeof(T)));
  if (bytes == 0) return;
  if (P->stage_used + bytes > P->stage_cap) {
    USFFT_HIP(hipStreamSynchronize(st));  // every earlier copy out of the arena is done
    P->stage_used = 0;
    if (bytes > P->stage_cap && !P->ws_mode) {
      if (P->stage) USFFT_HIP(hipHostFree(P->stage));
      P->stage = nullptr;
      P->stage_cap = 0;
      const size_t cap = std::max<size_t>(bytes, 4u << 20);
      USFFT_HIP(hipHostMalloc(reinterpret_cast<void**>(&P->stage), cap, hipHostMallocDefault));
      P->stage_cap = cap;
    }
  }
  if (P->ws_mode && bytes > P->stage_cap) {
    // no new pinned memory in workspace mode: a synchronous pageable copy
    USFFT_HIP(hipMemcpyAsync(b.p, v.data(), bytes, hipMemcpyHostToDevice, st));
    USFFT_HIP(hipStreamSynchronize(st));
    return;
  }
  std::memcpy(P->stage + P->stage_used, v.data(), bytes);
  USFFT_HIP(hipMemcpyAsync(b.p, P->stage + P->stage_used, bytes, hipMemcpyHostToDevice, st));
  P->stage_used += (bytes + 255) / 256 * 256;
}

// Pinned host memory for a readback of `bytes` (grown as needed).
static char* back_buffer(usfft_plan_s* P, size_t bytes) {
  if (bytes > P->back_cap && P->ws_mode) {
    // no new pinned memory in workspace mode: pageable landing buffer
    P->back_host.resize(bytes);
    return P->back_host.data();
  }
  if (bytes > P->back_cap) {
    if (P->back) USFFT_HIP(hipHostFree(P->back));
    P->back = nullptr;
    P->back_cap = 0;
    const size_t cap = std::max<size_t>(bytes, 1u << 20);
    USFFT_HIP(hipHostMalloc(reinterpret_cast<void**>(&P->back), cap, hipHostMallocDefault));
    P->back_cap = cap;
  }
  return P->back;
}

// Greedy multiple rank-1 lattice family (reading stated in usfft.h).  The
// attempts run on the device in batches: generators, alias counts, scores,
// the choice of the best try and its commit, with one readback of the batch's
// choices; the host rebuilds the family from them.
constexpr int kFamilyBatch = 4;

static void plan_family(usfft_plan_s* P, const int32_t* J, int64_t n, int t, uint64_t seed, int kind, int tcode,
                        Family& F, int32_t* assign, int32_t* bins_out, hipStream_t st) {
  const usfft_params& par = P->par;
  F = Family{};
  F.t = t;
  F.off.push_back(0);
  if (n == 0) return;
  int lo = std::max<int64_t>(3, (int64_t)std::ceil(par.lattice_c * (double)n));
  lo = std::min(lo, par.lattice_mmax / 2);
  const std::vector<int> sizes = admissible_sizes(lo, par.lattice_mmax);
  USFFT_REQUIRE(!sizes.empty(), USFFT_ELATTICE, "no admissible lattice size in range");
  const int T = par.lattice_tries;
  P->famcov.ensure(n);
  USFFT_HIP(hipMemsetAsync(P->famcov.p, 0, n, st));
  P->fambins.ensure(sizeof(int32_t) * n * T);
  P->famscores.ensure(sizeof(int32_t) * T);
  P->famz.ensure(sizeof(int32_t) * (size_t)T * t);
  P->famcounts.ensure(sizeof(int32_t) * (size_t)T * par.lattice_mmax);
  P->famlog.ensure(sizeof(int32_t) * 2 * (size_t)par.lattice_max);
  // (uncovered, lattices taken), double-buffered: attempt a reads slot a % 2
  // and writes slot (a + 1) % 2
  h2d_async(P, P->famstate, std::vector<int64_t>{n, 0, 0, 0}, st);
  int64_t* slot = P->famstate.as<int64_t>();
  for (int attempt = 0;;) {
    const int nb = std::min(kFamilyBatch, par.lattice_max - attempt);
    for (int b = 0; b < nb; ++b) {
      const int a = attempt + b;
      const int M = sizes[a % sizes.size()];
      launch_lattice_try(seed, kind, tcode, a, T, t, M, J, n, P->famcov.as<uint8_t>(), P->famz.as<int32_t>(),
                         P->fambins.as<int32_t>(), P->famcounts.as<int32_t>(), P->famscores.as<int32_t>(), st);
      launch_lattice_pick_take(P->famscores.as<int32_t>(), T, slot + 2 * (a & 1), slot + 2 * ((a + 1) & 1),
                               P->famlog.as<int32_t>() + 2 * a, P->fambins.as<int32_t>(),
                               P->famcounts.as<int32_t>(), P->famcov.as<uint8_t>(), n, M, assign, bins_out, st);
    }
    char* hb = back_buffer(P, 2 * sizeof(int64_t) + sizeof(int32_t) * 2 * kFamilyBatch);
    int64_t* state = reinterpret_cast<int64_t*>(hb);
    int32_t* lg = reinterpret_cast<int32_t*>(hb + 2 * sizeof(int64_t));
    USFFT_HIP(hipMemcpyAsync(state, slot + 2 * ((attempt + nb) & 1), 2 * sizeof(int64_t), hipMemcpyDeviceToHost,
                             st));
    USFFT_HIP(hipMemcpyAsync(lg, P->famlog.as<int32_t>() + 2 * attempt, sizeof(int32_t) * 2 * nb,
                             hipMemcpyDeviceToHost, st));
    USFFT_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < nb; ++b) {
      if (lg[2 * b + 1] == 0) continue;
      const int a = attempt + b;
      const int M = sizes[a % sizes.size()];
      F.M.push_back(M);
      for (int j = 0; j < t; ++j) F.z.push_back(rng::lattice_z(seed, kind, tcode, a, lg[2 * b], j, M));
      F.off.push_back(F.off.back() + M);
    }
    attempt += nb;
    if (state[0] == 0) break;
    USFFT_REQUIRE(attempt < par.lattice_max, USFFT_ELATTICE,
                  "lattice family incomplete after " + std::to_string(par.lattice_max) + " attempts");
  }
}

// Group candidates by lattice: pos lists (ascending) and bins, uploaded to
// P->lists in one copy together with the family's offsets, sizes and
// generators (F.d_off, F.d_M, F.d_z point into it).  bins = assign + n reads
// both back in one copy.
static void group_by_lattice(usfft_plan_s* P, Family& F, const int32_t* assign, const int32_t* bins, int64_t n,
                             hipStream_t st) {
  int32_t* ha = reinterpret_cast<int32_t*>(back_buffer(P, 2 * sizeof(int32_t) * std::max<int64_t>(n, 1)));
  int32_t* hb = ha + n;
  if (n > 0) {
    if (bins == assign + n) {
      USFFT_HIP(hipMemcpyAsync(ha, assign, 2 * sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    } else {
      USFFT_HIP(hipMemcpyAsync(ha, assign, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
      USFFT_HIP(hipMemcpyAsync(hb, bins, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
    }
    USFFT_HIP(hipStreamSynchronize(st));
  }
  const int nl = (int)F.M.size();
  F.lat_count.assign(nl, 0);
  for (int64_t a = 0; a < n; ++a) F.lat_count[ha[a]]++;
  F.lat_first.assign(nl, 0);
  for (int l = 1; l < nl; ++l) F.lat_first[l] = F.lat_first[l - 1] + F.lat_count[l - 1];
  std::vector<int32_t> lists(2 * std::max<int64_t>(n, 1));
  std::vector<int32_t> fill(F.lat_first);
  for (int64_t a = 0; a < n; ++a) {
    const int l = ha[a];
    lists[fill[l]] = (int32_t)a;  // positions
    lists[n + fill[l]] = hb[a];   // bins
    fill[l]++;
  }
  const size_t lb = sizeof(int32_t) * lists.size();
  const size_t o_off = (lb + 7) / 8 * 8;
  const size_t o_M = o_off + sizeof(int64_t) * F.off.size();
  const size_t o_z = o_M + sizeof(int32_t) * F.M.size();
  std::vector<char> pack(o_z + sizeof(int32_t) * F.z.size());
  std::memcpy(pack.data(), lists.data(), lb);
  std::memcpy(pack.data() + o_off, F.off.data(), sizeof(int64_t) * F.off.size());
  if (!F.M.empty()) std::memcpy(pack.data() + o_M, F.M.data(), sizeof(int32_t) * F.M.size());
  if (!F.z.empty()) std::memcpy(pack.data() + o_z, F.z.data(), sizeof(int32_t) * F.z.size());
  h2d_async(P, P->lists, pack, st);
  F.d_off = reinterpret_cast<const int64_t*>(P->lists.as<char>() + o_off);
  F.d_M = reinterpret_cast<const int32_t*>(P->lists.as<char>() + o_M);
  F.d_z = reinterpret_cast<const int32_t*>(P->lists.as<char>() + o_z);
}

// One solver launch at the mesh's own nodes.  params: Y holds parameters y
// of the model instead of sampling nodes t.
// Rendezvous of the DST solver launches of jobs run together
// (usfft_detect_batch).  A job's sampler call waits until every job still
// running has made its next call or finished; the last one to arrive then
// launches one persistent solver kernel per class (mesh, precision, solver
// variant) over a segment table of all the waiting jobs' batches, on the
// first such job's stream, after every job's stream has reached its call,
// and each job's stream waits for that launch before it goes on.  Every
// solve is independent of its batch, so each job's results are those it
// gets alone.
struct FuseReq {
  usfft_plan_s* P;
  SolveSeg seg;
  int64_t ns;
  int out_fp32;
  hipStream_t st;
  hipEvent_t ready = nullptr, done = nullptr;
};
struct FuseGroup {
  std::mutex mu;
  std::condition_variable cv;
  int active = 0;
  uint64_t round = 0;
  std::vector<FuseReq*> reqs;
  std::string error;
  // device segment tables, a ring of slots, each reused only after the
  // launch that read it has finished
  static constexpr int kSlots = 4, kMaxSeg = 64;
  DevBuf segs[kSlots];
  hipEvent_t slot_done[kSlots] = {};
  int next_slot = 0;
  int64_t launches = 0, fused_launches = 0, segments = 0;
  ~FuseGroup() {
    for (hipEvent_t e : slot_done)
      if (e) (void)hipEventDestroy(e);
  }
};

// Launches the collected requests (called with the group's lock held).
static void fuse_launch(FuseGroup* F) {
  std::vector<FuseReq*> todo = F->reqs;
  while (!todo.empty()) {
    FuseReq* lead = todo.front();
    usfft_plan_s* LP = lead->P;
    std::vector<FuseReq*> cls, rest;
    for (FuseReq* r : todo)
      (r->P->prob.mesh_n == LP->prob.mesh_n && r->P->par.precision == LP->par.precision &&
               r->P->dst_variant == LP->dst_variant && r->out_fp32 == lead->out_fp32 &&
               r->P->par.pcg_rtol == LP->par.pcg_rtol && r->P->par.pcg_maxit == LP->par.pcg_maxit &&
               r->P->par.inner_rtol == LP->par.inner_rtol && r->P->par.refine_every == LP->par.refine_every &&
               (int)cls.size() < FuseGroup::kMaxSeg
           ? cls
           : rest)
          .push_back(r);
    todo.swap(rest);
    std::vector<SolveSeg> tab;
    int64_t ns = 0;
    for (FuseReq* r : cls) {
      SolveSeg sg = r->seg;
      sg.begin = ns;
      tab.push_back(sg);
      ns += r->ns;
    }
    const int slot = F->next_slot;
    F->next_slot = (F->next_slot + 1) % FuseGroup::kSlots;
    if (F->slot_done[slot]) {
      USFFT_HIP(hipEventSynchronize(F->slot_done[slot]));
    } else {
      USFFT_HIP(hipEventCreateWithFlags(&F->slot_done[slot], hipEventDisableTiming));
    }
    F->segs[slot].ensure(sizeof(SolveSeg) * FuseGroup::kMaxSeg);
    USFFT_HIP(hipMemcpy(F->segs[slot].p, tab.data(), sizeof(SolveSeg) * tab.size(), hipMemcpyHostToDevice));
    const hipStream_t st = lead->st;
    for (FuseReq* r : cls) USFFT_HIP(hipStreamWaitEvent(st, r->ready, 0));
    const usfft_params& par = LP->par;
    launch_pde_solve_dst(F->segs[slot].as<SolveSeg>(), (int)tab.size(), LP->prob.mesh_n, par.precision,
                         LP->dst_variant, ns, par.pcg_rtol, par.pcg_maxit, par.inner_rtol, par.refine_every,
                         lead->out_fp32, LP->d_wscr.as<double>(), LP->wblocks, LP->d_sfrag.p, LP->d_lam.as<float>(),
                         st);
    USFFT_HIP(hipEventRecord(F->slot_done[slot], st));
    for (FuseReq* r : cls) USFFT_HIP(hipEventRecord(r->done, st));
    F->launches++;
    F->fused_launches += cls.size() > 1 ? 1 : 0;
    F->segments += (int64_t)cls.size();
  }
  F->reqs.clear();
}

// The rendezvous of one sampler call (see FuseGroup).
static void fused_solve(usfft_plan_s* P, const SolveSeg& seg, int64_t ns, int out_fp32, hipStream_t st) {
  FuseGroup* F = P->fuse;
  FuseReq r{P, seg, ns, out_fp32, st};
  USFFT_HIP(hipEventCreateWithFlags(&r.ready, hipEventDisableTiming));
  USFFT_HIP(hipEventCreateWithFlags(&r.done, hipEventDisableTiming));
  struct Ev {
    FuseReq& r;
    ~Ev() {
      (void)hipEventDestroy(r.ready);
      (void)hipEventDestroy(r.done);
    }
  } ev{r};
  USFFT_HIP(hipEventRecord(r.ready, st));
  {
    std::unique_lock<std::mutex> lk(F->mu);
    USFFT_REQUIRE(F->error.empty(), USFFT_EHIP, "fused launch failed: " + F->error);
    F->reqs.push_back(&r);
    if ((int)F->reqs.size() == F->active) {
      try {
        fuse_launch(F);
      } catch (const Error& e) {
        F->error = e.msg;
        F->reqs.clear();
      }
      F->round++;
      F->cv.notify_all();
    } else {
      const uint64_t r0 = F->round;
      F->cv.wait(lk, [&] { return F->round != r0; });
    }
    USFFT_REQUIRE(F->error.empty(), USFFT_EHIP, "fused launch failed: " + F->error);
  }
  USFFT_HIP(hipStreamWaitEvent(st, r.done, 0));
  // the events may be destroyed now: their work is enqueued
}

// A job of the batch leaves the rendezvous (finished or failed); if every
// job still running is waiting, their launch happens now.
static void fuse_leave(FuseGroup* F) {
  std::lock_guard<std::mutex> lk(F->mu);
  F->active--;
  if (F->active > 0 && (int)F->reqs.size() == F->active) {
    try {
      fuse_launch(F);
    } catch (const Error& e) {
      F->error = e.msg;
      F->reqs.clear();
    }
    F->round++;
    F->cv.notify_all();
  }
}

static void solve_batch(usfft_plan_s* P, const double* Y, int64_t ns, void* U, int out_fp32, int64_t ld,
                        int64_t col0, int32_t* iters, hipStream_t st, bool params);

// Sampler call on rows [0, ns) of Y into U columns [col0, col0 + ns): the
// solver's values at the nodes T_G (interpolated when T_G is a point set).
static void run_sampler(usfft_plan_s* P, const double* Y, int64_t ns, void* U, int out_fp32, int64_t ld,
                        int64_t col0, int32_t* iters, hipStream_t st, bool params = false) {
  if (ns <= 0) return;
  if (!P->interp) {
    solve_batch(P, Y, ns, U, out_fp32, ld, col0, iters, st, params);
    return;
  }
  const int64_t ldm = ceil_div(ns, 64) * 64;
  P->Umesh.ensure((out_fp32 ? sizeof(float) : sizeof(double)) * P->G_mesh * ldm);
  solve_batch(P, Y, ns, P->Umesh.p, out_fp32, ldm, 0, iters, st, params);
  launch_interp(P->Umesh.p, out_fp32, ldm, P->d_iidx.as<int32_t>(), P->d_iw.as<double>(), P->G, ns, U, ld, col0, st);
}

static void solve_batch(usfft_plan_s* P, const double* Y, int64_t ns, void* U, int out_fp32, int64_t ld,
                        int64_t col0, int32_t* iters, hipStream_t st, bool params) {
  const usfft_params& par = P->par;
  PdeDev pde = P->pde;
  pde.raw = params ? 1 : 0;
  if (P->prob.sampler == USFFT_SAMPLER_PDE_MESH) {
    launch_pde_solve_mesh(pde, P->mesh, Y, ns, par.pcg_rtol, par.pcg_maxit, U, out_fp32, ld, col0, iters,
                          P->mesh_blocks, mesh_fits_lds(P->mesh) ? nullptr : P->d_wscr.as<double>(), st);
  } else if (P->prob.sampler == USFFT_SAMPLER_PDE && P->dst) {
    const SolveSeg seg{pde, Y, U, ld, col0, 0, iters};
    if (P->fuse) {
      fused_solve(P, seg, ns, out_fp32, st);
    } else {
      h2d_async(P, P->segbuf, std::vector<SolveSeg>{seg}, st);
      launch_pde_solve_dst(P->segbuf.as<SolveSeg>(), 1, P->prob.mesh_n, par.precision, P->dst_variant, ns,
                           par.pcg_rtol, par.pcg_maxit, par.inner_rtol, par.refine_every, out_fp32,
                           P->d_wscr.as<double>(), P->wblocks, P->d_sfrag.p, P->d_lam.as<float>(), st);
    }
  } else if (P->prob.sampler == USFFT_SAMPLER_PDE && P->tl_stream) {
    launch_pde_solve_tl_stream(pde, Y, ns, par.pcg_rtol, par.pcg_maxit, U, out_fp32, ld, col0, iters,
                               P->d_stream.as<double>(), P->wblocks, P->d_sfrag.p, P->d_lam.as<float>(), st);
  } else if (P->prob.sampler == USFFT_SAMPLER_PDE && P->dst_stream) {
    launch_pde_solve_dst_stream(pde, Y, ns, par.pcg_rtol, par.pcg_maxit, U, out_fp32, ld, col0, iters,
                                P->d_stream.as<double>(), P->wblocks, P->d_sfrag.p, P->d_lam.as<float>(), st);
  } else if (P->prob.sampler == USFFT_SAMPLER_PDE && P->streaming) {
    launch_pde_solve_stream(pde, Y, ns, par.pcg_rtol, par.pcg_maxit, U, out_fp32, ld, col0, iters,
                            P->d_stream.as<double>(), kStreamBlocks, st);
  } else if (P->prob.sampler == USFFT_SAMPLER_PDE) {
    launch_pde_solve(P->solver_cfg, pde, par.precision, Y, ns, par.pcg_rtol, par.pcg_maxit, par.inner_rtol,
                     par.refine_every, U, out_fp32, ld, col0, iters, P->d_wscr.as<double>(), P->wblocks, st);
  } else {
    launch_trigpoly(P->prob.d, Y, ns, P->d_polyk.as<int32_t>(), P->prob.n_poly, P->d_polyc.as<double>(), P->G, U,
                    out_fp32, ld, col0, st);
    if (iters) USFFT_HIP(hipMemsetAsync(iters, 0, sizeof(int32_t) * ns, st));
  }
}

// Bin k.z mod M of every candidate (App. A), in exact 64-bit arithmetic.
struct GenVec {
  int64_t z[kMaxD];
};
__global__ void lattice_bin_kernel(const int32_t* __restrict__ J, int64_t n, int t, GenVec z, int64_t M,
                                   int32_t* __restrict__ bins) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  int64_t b = 0;
  for (int j = 0; j < t; ++j) b = (b + (int64_t)J[a * t + j] * z.z[j] % M) % M;
  bins[a] = (int32_t)((b + M) % M);
}

__global__ void iter_stats_kernel(const int32_t* __restrict__ it, int64_t n, unsigned long long* __restrict__ acc) {
  unsigned long long bad = 0, sum = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int v = it[i];
    if (v < 0)
      ++bad;
    else
      sum += (unsigned long long)v;
  }
  bad = wave_sum(bad);
  sum = wave_sum(sum);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    if (bad) atomicAdd(&acc[0], bad);
    if (sum) atomicAdd(&acc[1], sum);
  }
}

static void accumulate_iters(usfft_plan_s* P, int64_t ns, hipStream_t st) {
  if (ns <= 0) return;
  const unsigned grid = (unsigned)std::min<int64_t>(256, ceil_div(ns, 256));
  hipLaunchKernelGGL(iter_stats_kernel, dim3(grid), dim3(256), 0, st, P->iters.as<int32_t>(), ns,
                     P->cnt.as<unsigned long long>());
  USFFT_HIP(hipGetLastError());
}

struct Timer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];
  hipStream_t st;
  explicit Timer(hipStream_t s) : st(s) {}
  int open(int cat) {
    hipEvent_t a, b;
    USFFT_HIP(hipEventCreate(&a));
    USFFT_HIP(hipEventCreate(&b));
    USFFT_HIP(hipEventRecord(a, st));
    ev[cat].push_back({a, b});
    return (int)ev[cat].size() - 1;
  }
  void close(int cat, int i) { USFFT_HIP(hipEventRecord(ev[cat][i].second, st)); }
  double total(int cat) {
    double s = 0;
    for (auto& e : ev[cat]) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) s += ms;
    }
    return s;
  }
  ~Timer() {
    for (auto& v : ev)
      for (auto& e : v) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
};
enum { kTSample = 0, kTDft = 1, kTSelect = 2 };

static std::pair<int, int> rader_tuned_shape(usfft_plan_s* P, int Lmax, int ufp32, int64_t G,
                                             const std::function<void(int, int)>& launch, hipStream_t st);

// ---------------------------------------------------------------- Alg. 1
// given: step 3 alone on the set given_I (host, given_n x d)
// Progress lines on stderr, one per step of Alg. 1 and per increment, when
// the environment sets USFFT_LOG to a non-zero value (read once per process).
static bool progress_log() {
  static const bool on = [] {
    const char* v = std::getenv("USFFT_LOG");
    return v != nullptr && v[0] != '\0' && v[0] != '0';
  }();
  return on;
}

static double seconds_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

static void detect(usfft_plan_s* P, uint64_t seed, hipStream_t st, usfft_result_s* R, bool given = false,
                   const int32_t* given_I = nullptr, int64_t given_n = 0) {
  const usfft_problem& pb = P->prob;
  const usfft_params& par = P->par;
  const int d = pb.d;
  const int64_t G = P->G;
  const int ufp32 = par.precision == USFFT_FP32_REFINE ? 1 : 0;
  const size_t ub = ufp32 ? sizeof(float) : sizeof(double);
  Timer tm(st);
  usfft_stats& S = R->stats;
  auto sample_timed = [&](const double* Y, int64_t ns, int64_t ld) {
    const int e = tm.open(kTSample);
    run_sampler(P, Y, ns, P->U.p, ufp32, ld, 0, P->iters.as<int32_t>(), st);
    tm.close(kTSample, e);
    S.max_batch = std::max(S.max_batch, ns);
    accumulate_iters(P, ns, st);
    S.sample_launches += ns > 0 ? 1 : 0;
  };
  const auto t0 = std::chrono::steady_clock::now();

  P->cnt.ensure(3 * sizeof(unsigned long long));
  USFFT_HIP(hipMemsetAsync(P->cnt.p, 0, 2 * sizeof(unsigned long long), st));
  P->theta2.ensure(sizeof(double));
  P->scratch.ensure(64);
  if (!par.theta_relative) {
    const double th2 = par.theta * par.theta;
    USFFT_HIP(hipMemcpyAsync(P->theta2.p, &th2, sizeof(double), hipMemcpyHostToDevice, st));
    USFFT_HIP(hipStreamSynchronize(st));
  }
  P->tail.ensure(sizeof(double) * kMaxD);
  // P->cnt: (solves that missed pcg_rtol, PCG iterations, rows kept by the
  // last step-2 compaction); one pinned readback of all three
  auto check_conv = [&]() -> int64_t {
    const unsigned long long* h = reinterpret_cast<const unsigned long long*>(back_buffer(P, 3 * sizeof(int64_t)));
    USFFT_HIP(hipMemcpyAsync(const_cast<unsigned long long*>(h), P->cnt.p, 3 * sizeof(int64_t),
                             hipMemcpyDeviceToHost, st));
    USFFT_HIP(hipStreamSynchronize(st));
    S.pcg_iterations = (int64_t)h[1];
    USFFT_REQUIRE(h[0] == 0, USFFT_ENOCONV,
                  std::to_string(h[0]) + " PCG solves missed pcg_rtol within pcg_maxit");
    return (int64_t)h[2];
  };

  int64_t nprev = 0;
  Family F;
  if (given) {
    // a-priori index set (Sec. 4.5): steps 1 and 2 are skipped and step 3
    // computes the coefficients of the caller's frequencies
    nprev = given_n;
    P->Iprev.ensure(sizeof(int32_t) * std::max<int64_t>(1, nprev * d));
    if (nprev > 0)
      USFFT_HIP(hipMemcpyAsync(P->Iprev.p, given_I, sizeof(int32_t) * nprev * d, hipMemcpyHostToDevice, st));
  } else {
    // ---------------- step 1 & 2a
    // The d x r line stages are independent: their sampling nodes are
    // generated into one batch, solved in one sampler launch, then
    // transformed and selected line by line (the threshold of a relative theta
    // comes from line (1, 1), which runs first).
    P->I1.resize(d);
    P->I1n.assign(d, 0);
    bool theta_set = !par.theta_relative;
    {
      const int r = par.r;
      std::vector<int32_t> Kt(d), ks;
      std::vector<int64_t> off(d * r + 1, 0), coff(d + 1, 0), woff(d + 1, 0);
      int Kmax = 1;
      for (int t = 0; t < d; ++t) {
        Kt[t] = pb.k_hi[t] - pb.k_lo[t] + 1;
        Kmax = std::max(Kmax, Kt[t]);
        for (int a = 0; a < Kt[t]; ++a) ks.push_back(pb.k_lo[t] + a);
        coff[t + 1] = coff[t] + Kt[t];
        woff[t + 1] = woff[t] + ceil_div(Kt[t], 32);
        for (int i = 0; i < r; ++i) off[t * r + i + 1] = off[t * r + i] + Kt[t];
      }
      const int64_t ns = off.back(), ld = ceil_div(ns, 64) * 64;
      h2d_async(P, P->cands, ks, st);
      h2d_async(P, P->latM, Kt, st);
      P->U.ensure(ub * G * ld);
      const int nl = d * r;                   // step-1 lines, line (t, i) = t r + i
      const int64_t ldv = (int64_t)nl * Kmax;  // |X|^2 of line y in columns y Kmax ..
      P->V.ensure(sizeof(double) * G * ldv);
      P->Y.ensure(sizeof(double) * ns * d);
      P->iters.ensure(sizeof(int32_t) * ns);
      P->mask.ensure(sizeof(uint32_t) * woff[d]);
      USFFT_HIP(hipMemsetAsync(P->mask.p, 0, sizeof(uint32_t) * woff[d], st));
      std::vector<double> tails((size_t)d * r * d);
      for (int t = 0; t < d; ++t)
        for (int i = 0; i < r; ++i)
          for (int j = 0; j < d; ++j)
            tails[((size_t)t * r + i) * d + j] = rng::uniform01(seed, rng::stream(rng::kTail1, t + 1, i + 1, 0), j);
      h2d_async(P, P->tail, tails, st);
      h2d_async(P, P->latoff, off, st);
      launch_line_nodes(d, r, P->latoff.as<int64_t>(), P->latM.as<int32_t>(), P->tail.as<double>(),
                        P->Y.as<double>(), ns, st);
      sample_timed(P->Y.as<double>(), ns, ld);
      S.samples_step1 += ns;
      // every line's DFT in one launch, then every line's selection in one
      // launch (the relative threshold comes from line (1, 1) in between)
      int e = tm.open(kTDft);
      launch_line_dft_lines(P->U.p, ufp32, G, ld, P->latoff.as<int64_t>(), P->latM.as<int32_t>(),
                            P->cands.as<int32_t>(), nl, r, Kmax, Kmax, P->V.as<double>(), ldv, st);
      tm.close(kTDft, e);
      S.dft_launches += 1;
      if (!theta_set) {
        launch_max_to_theta(P->V.as<double>(), G, Kt[0], ldv, par.theta, P->theta2.as<double>(),
                            P->scratch.as<uint64_t>(), st);
        theta_set = true;
      }
      e = tm.open(kTSelect);
      launch_select_lines(P->V.as<double>(), G, ldv, nl, r, Kmax, P->latM.as<int32_t>(), Kmax, par.s_local,
                          P->theta2.as<double>(), par.tie_rel, P->mask.as<uint32_t>(), st);
      tm.close(kTSelect, e);
      P->scratch.ensure(32 + sizeof(int64_t) * d);
      for (int t = 0; t < d; ++t) {
        P->I1[t].ensure(sizeof(int32_t) * Kt[t]);
        launch_compact(P->cands.as<int32_t>() + coff[t], P->mask.as<uint32_t>() + woff[t], Kt[t], 1,
                       P->I1[t].as<int32_t>(), reinterpret_cast<int64_t*>(P->scratch.as<char>() + 32) + t, st);
      }
      std::vector<int64_t> cnt(d);
      USFFT_HIP(hipMemcpyAsync(cnt.data(), P->scratch.as<char>() + 32, sizeof(int64_t) * d, hipMemcpyDeviceToHost,
                               st));
      check_conv();
      for (int t = 0; t < d; ++t) P->I1n[t] = cnt[t];
      if (progress_log()) {
        int64_t kept = 0;
        for (int t = 0; t < d; ++t) kept += cnt[t];
        std::fprintf(stderr, "usfft: step 1: %d lines, %lld samples, %lld frequencies kept, %.2f s\n", nl,
                     (long long)ns, (long long)kept, seconds_since(t0));
        std::fflush(stderr);
      }
      if (par.trace) {
        for (int t = 0; t < d; ++t) {
          std::vector<int32_t> v((size_t)cnt[t]);
          if (cnt[t] > 0)
            USFFT_HIP(hipMemcpyAsync(v.data(), P->I1[t].p, sizeof(int32_t) * cnt[t], hipMemcpyDeviceToHost, st));
          R->trace_set.push_back(std::move(v));
          R->trace_width.push_back(1);
          R->trace_cand.push_back(Kt[t]);
        }
        USFFT_HIP(hipStreamSynchronize(st));
      }
    }
    {
      double th2 = 0;
      USFFT_HIP(hipMemcpyAsync(&th2, P->theta2.p, sizeof(double), hipMemcpyDeviceToHost, st));
      USFFT_HIP(hipStreamSynchronize(st));
      S.theta_abs = std::sqrt(th2);
    }

    // ---------------- step 2
    {
      // the tails of every increment's iterations, uploaded once: increment t
      // (1 <= t < d), iteration i at ((t - 1) r + i) d
      std::vector<double> tails((size_t)(d > 1 ? d - 1 : 0) * par.r * d);
      for (int t = 1; t < d; ++t) {
        const int r_t = t == d - 1 ? 1 : par.r;
        for (int i = 0; i < r_t; ++i)
          for (int j = 0; j < d; ++j)
            tails[((size_t)(t - 1) * par.r + i) * d + j] = rng::uniform01(seed, rng::stream(rng::kTail2, t + 1, i + 1, 0), j);
      }
      h2d_async(P, P->tail, tails, st);
    }
    nprev = P->I1n[0];
    P->Iprev.ensure(sizeof(int32_t) * std::max<int64_t>(nprev, 1));
    if (nprev > 0)
      USFFT_HIP(hipMemcpyAsync(P->Iprev.p, P->I1[0].p, sizeof(int32_t) * nprev, hipMemcpyDeviceToDevice, st));
    for (int t = 1; t < d; ++t) {
      const bool last = t == d - 1;
      const int r_t = last ? 1 : par.r;
      const int s_t = last ? par.s : par.s_local;
      const int64_t nc = P->I1n[t];
      const int64_t n = nprev * nc;
      S.max_candidates = std::max(S.max_candidates, n);
      if (n == 0) {
        nprev = 0;
        if (par.trace) {
          R->trace_set.emplace_back();
          R->trace_width.push_back(t + 1);
          R->trace_cand.push_back(0);
        }
        continue;
      }
      const int w = t + 1;
      USFFT_REQUIRE(!P->ws_mode || n <= P->ws_ncand, USFFT_ENOMEM,
                    "increment t = " + std::to_string(t + 1) + " has " + std::to_string(n) +
                        " candidates; the workspace holds " + std::to_string(P->ws_ncand) + " (raise n_cand_max)");
      P->J.ensure(sizeof(int32_t) * n * w);
      launch_product(P->Iprev.as<int32_t>(), nprev, t, P->I1[t].as<int32_t>(), nc, P->J.as<int32_t>(), st);
      P->assign.ensure(2 * sizeof(int32_t) * n);  // assignments, then bins
      plan_family(P, P->J.as<int32_t>(), n, w, seed, rng::kLat2, w, F, P->assign.as<int32_t>(),
                  P->assign.as<int32_t>() + n, st);
      group_by_lattice(P, F, P->assign.as<int32_t>(), P->assign.as<int32_t>() + n, n, st);
      S.lattices += (int64_t)F.M.size();
      for (int M : F.M) (void)rader_for(P, M, st);
      const int64_t ns = F.total();
      // V holds the stage's magnitudes in lattice-grouped candidate order (each
      // lattice's bins contiguous per node); the mask is built in that order and
      // mapped back to candidate order before compaction.
      const int64_t words = ceil_div(n, 32);
      P->mask.ensure(sizeof(uint32_t) * words);
      P->gmask.ensure(sizeof(uint32_t) * words);
      USFFT_HIP(hipMemsetAsync(P->mask.p, 0, sizeof(uint32_t) * words, st));
      USFFT_HIP(hipMemsetAsync(P->gmask.p, 0, sizeof(uint32_t) * words, st));
      // the r_t iterations differ only in their tails: their samples are
      // solved together, in batches of at most kSampleBatchBytes of samples
      S.max_family = std::max(S.max_family, ns);
      int rb = r_t;
      if (P->ws_mode) {
        USFFT_REQUIRE(ns <= P->ws_nsamp, USFFT_ENOMEM,
                      "the lattice family of increment t = " + std::to_string(t + 1) + " needs " + std::to_string(ns) +
                          " samples; the workspace holds " + std::to_string(P->ws_nsamp) + " (raise samples_max)");
        rb = (int)std::min<int64_t>(r_t, P->ws_nsamp / ns);
      } else {
        while (rb > 1 && ub * (uint64_t)G * (uint64_t)(rb * ns) > kSampleBatchBytes) --rb;
      }
      P->V.ensure(sizeof(double) * G * n * rb);
      for (int i0 = 0; i0 < r_t; i0 += rb) {
        const int nb = std::min(rb, r_t - i0);
        const int64_t nsb = nb * ns, ldb = ceil_div(nsb, 64) * 64;
        P->U.ensure(ub * G * ldb);
        P->Y.ensure(sizeof(double) * nsb * d);
        P->iters.ensure(sizeof(int32_t) * nsb);
        launch_lattice_nodes_rep(d, w, (int)F.M.size(), F.d_off, F.d_M, F.d_z,
                                 P->tail.as<double>() + ((size_t)(t - 1) * par.r + i0) * d, P->Y.as<double>(), ns,
                                 nb, st);
        sample_timed(P->Y.as<double>(), nsb, ldb);
        S.samples_step2 += nsb;
        // every lattice of every iteration of the batch in one DFT launch
        // (iteration b's magnitudes in columns b n .. of V), then every
        // iteration's selection in one launch
        std::vector<LatItem> items;
        int Lmax = 2;
        for (int b = 0; b < nb; ++b)
          for (size_t l = 0; l < F.M.size(); ++l) {
            if (F.lat_count[l] == 0) continue;
            LatItem it{};
            fill_lat_item(it, rader_for(P, F.M[l], st), ufp32);
            it.col0 = b * ns + F.off[l];
            it.bins = P->lists.as<int32_t>() + n + F.lat_first[l];
            it.pos = nullptr;
            it.pos_base = F.lat_first[l];
            it.nb = F.lat_count[l];
            it.out_off = (int64_t)b * n;
            items.push_back(it);
            Lmax = std::max(Lmax, F.M[l] - 1);
            S.dft_bytes += (double)G * (double)F.M[l] * (double)ub + (double)G * F.lat_count[l] * 8.0;
          }
        h2d_async(P, P->latitems, items, st);
        auto dft = [&](int blk, int cols) {
          launch_lattice_dft_batch(P->latitems.as<LatItem>(), (int)items.size(), Lmax, P->U.p, ufp32, G, ldb,
                                   USFFT_OUT_MAG2, P->V.p, (int64_t)nb * n, st, blk, cols);
        };
        const std::pair<int, int> shape = rader_tuned_shape(P, Lmax, ufp32, G, dft, st);
        int e = tm.open(kTDft);
        dft(shape.first, shape.second);
        tm.close(kTDft, e);
        S.dft_launches += 1;
        e = tm.open(kTSelect);
        launch_select_iters(P->V.as<double>(), G, n, (int64_t)nb * n, nb, n, s_t, P->theta2.as<double>(),
                            par.tie_rel, P->gmask.as<uint32_t>(), st);
        tm.close(kTSelect, e);
      }
      launch_ungroup_mask(P->gmask.as<uint32_t>(), P->lists.as<int32_t>(), n, P->mask.as<uint32_t>(), st);
      P->Jnext.ensure(sizeof(int32_t) * n * w);
      launch_compact(P->J.as<int32_t>(), P->mask.as<uint32_t>(), n, w, P->Jnext.as<int32_t>(),
                     reinterpret_cast<int64_t*>(P->cnt.as<char>() + 2 * sizeof(int64_t)), st);
      const int64_t cntI = check_conv();
      std::swap(P->Iprev, P->Jnext);
      nprev = cntI;
      if (progress_log()) {
        std::fprintf(stderr,
                     "usfft: increment %d/%d: %lld candidates, %zu lattices, %lld samples x %d, %lld kept, %.2f s\n",
                     t + 1, d, (long long)n, F.M.size(), (long long)ns, r_t, (long long)cntI, seconds_since(t0));
        std::fflush(stderr);
      }
      if (par.trace) {
        std::vector<int32_t> v((size_t)(cntI * w));
        if (cntI > 0) {
          USFFT_HIP(hipMemcpyAsync(v.data(), P->Iprev.p, sizeof(int32_t) * cntI * w, hipMemcpyDeviceToHost, st));
          USFFT_HIP(hipStreamSynchronize(st));
        }
        R->trace_set.push_back(std::move(v));
        R->trace_width.push_back(w);
        R->trace_cand.push_back(n);
      }
    }
  }

  // ---------------- step 3
  const int64_t nI = nprev;
  R->d = d;
  if (pb.sampler != USFFT_SAMPLER_TRIG_POLY) {
    R->model = P->pde.model;
    R->alpha = P->pde.alpha;
    R->beta = P->pde.beta;
    R->delta = P->pde.delta;
  }
  R->G = G;
  R->I.assign((size_t)nI * d, 0);
  result_buffer(R, sizeof(double) * 2 * std::max<int64_t>(nI, 1) * G);
  if (nI > 0) {
    USFFT_HIP(hipMemcpyAsync(R->I.data(), P->Iprev.p, sizeof(int32_t) * nI * d, hipMemcpyDeviceToHost, st));
    P->assign.ensure(2 * sizeof(int32_t) * nI);  // assignments, then bins
    plan_family(P, P->Iprev.as<int32_t>(), nI, d, seed, rng::kLat3, 0, F, P->assign.as<int32_t>(),
                P->assign.as<int32_t>() + nI, st);
    group_by_lattice(P, F, P->assign.as<int32_t>(), P->assign.as<int32_t>() + nI, nI, st);
    S.lattices += (int64_t)F.M.size();
    for (int M : F.M) (void)rader_for(P, M, st);
    const int64_t ns = F.total();
    const int64_t ld = ceil_div(ns, 64) * 64;
    S.max_family = std::max(S.max_family, ns);
    USFFT_REQUIRE(!P->ws_mode || ns <= P->ws_nsamp, USFFT_ENOMEM,
                  "the step-3 lattice family needs " + std::to_string(ns) + " samples; the workspace holds " +
                      std::to_string(P->ws_nsamp) + " (raise samples_max)");
    P->U.ensure(ub * G * ld);
    P->Y.ensure(sizeof(double) * ns * d);
    P->iters.ensure(sizeof(int32_t) * ns);
    launch_nodes(d, -1, d, (int)F.M.size(), F.d_off, F.d_M, F.d_z, P->tail.as<double>(), P->Y.as<double>(), ns, st);
    sample_timed(P->Y.as<double>(), ns, ld);
    S.samples_step3 += ns;
    std::vector<LatItem> items;
    int Lmax = 2;
    for (size_t l = 0; l < F.M.size(); ++l) {
      if (F.lat_count[l] == 0) continue;
      LatItem it{};
      fill_lat_item(it, rader_for(P, F.M[l], st), ufp32);
      it.col0 = F.off[l];
      it.bins = P->lists.as<int32_t>() + nI + F.lat_first[l];
      it.pos = P->lists.as<int32_t>() + F.lat_first[l];
      it.pos_base = 0;
      it.nb = F.lat_count[l];
      it.out_off = 0;
      items.push_back(it);
      Lmax = std::max(Lmax, F.M[l] - 1);
      S.dft_bytes += (double)G * (double)F.M[l] * (double)ub + (double)G * F.lat_count[l] * 16.0;
    }
    h2d_async(P, P->latitems, items, st);
    auto dft = [&](int blk, int cols) {
      launch_lattice_dft_batch(P->latitems.as<LatItem>(), (int)items.size(), Lmax, P->U.p, ufp32, G, ld,
                               USFFT_OUT_COMPLEX, R->C.p, G, st, blk, cols);
    };
    const std::pair<int, int> shape = rader_tuned_shape(P, Lmax, ufp32, G, dft, st);
    int e = tm.open(kTDft);
    dft(shape.first, shape.second);
    tm.close(kTDft, e);
    S.dft_launches += 1;
    check_conv();
    if (progress_log()) {
      std::fprintf(stderr, "usfft: step 3: %lld frequencies, %zu lattices, %lld samples, %.2f s\n", (long long)nI,
                   F.M.size(), (long long)ns, seconds_since(t0));
      std::fflush(stderr);
    }
  }
  USFFT_HIP(hipStreamSynchronize(st));
  S.samples = S.samples_step1 + S.samples_step2 + S.samples_step3;
  S.solver_kind = -1;
  if (pb.sampler == USFFT_SAMPLER_PDE && P->dst) {
    S.solver_block = 4 * dst_padded(P->prob.mesh_n);
    S.solver_npt = dst_padded(P->prob.mesh_n) / 4;
    S.solver_kind = 0;
  } else if (pb.sampler == USFFT_SAMPLER_PDE && P->dst_stream) {
    S.solver_block = 512;
    S.solver_npt = 32;
    S.solver_kind = 4;
  } else if (pb.sampler == USFFT_SAMPLER_PDE && P->tl_stream) {
    S.solver_block = 512;
    S.solver_npt = 32;
    S.solver_kind = 5;
  } else if (pb.sampler == USFFT_SAMPLER_PDE && !P->streaming) {
    int blk = 0, npt = 0;
    solver_config_shape(P->solver_cfg, &blk, &npt);
    S.solver_block = blk;
    S.solver_npt = npt;
    S.solver_kind = 1;
  } else if (pb.sampler == USFFT_SAMPLER_PDE) {
    S.solver_kind = 2;
  } else if (pb.sampler == USFFT_SAMPLER_PDE_MESH) {
    S.solver_block = 256;
    S.solver_kind = 3;
  }
  S.ms_sample = tm.total(kTSample);
  S.ms_dft = tm.total(kTDft);
  S.ms_select = tm.total(kTSelect);
  S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- caller workspace
// Every transient device buffer of detect(), in a fixed order, with its
// largest size for candidate sets of at most ncand entries (|J_t| and the
// output set) and sampler batches of at most nsamp samples (step 1 always
// runs as one batch of its r sum_t K_t line samples); the last entry is the
// output coefficient matrix.
struct WsItem {
  DevBuf* buf;
  size_t bytes;
};

static std::vector<WsItem> ws_items(usfft_plan_s* P, DevBuf* C, int64_t ncand, int64_t nsamp) {
  const usfft_problem& pb = P->prob;
  const usfft_params& par = P->par;
  const int64_t d = pb.d, r = par.r, G = P->G, T = par.lattice_tries, Lm = par.lattice_max;
  const int64_t ub = par.precision == USFFT_FP32_REFINE ? 4 : 8;
  int64_t sumK = 0, Kmax = 1, woff = 0;
  for (int t = 0; t < d; ++t) {
    const int64_t K = pb.k_hi[t] - pb.k_lo[t] + 1;
    sumK += K;
    Kmax = std::max(Kmax, K);
    woff += ceil_div(K, 32);
  }
  const int64_t ns1 = r * sumK, nl = d * r;
  const int64_t nsb = ceil_div(std::max(ns1, nsamp), 64) * 64;
  const int64_t nc = std::max<int64_t>(ncand, 1);
  P->I1.resize(d);
  auto sz = [](int64_t b) { return (size_t)std::max<int64_t>(256, ceil_div(b, 256) * 256); };
  std::vector<WsItem> v = {
      {&P->U, sz(ub * G * nsb)},
      {&P->V, sz(8 * G * std::max(nl * Kmax, r * nc))},
      {&P->latitems, sz((int64_t)sizeof(LatItem) * std::max<int64_t>(r, 1) * Lm)},
      {&P->Y, sz(8 * d * nsb)},
      {&P->iters, sz(4 * nsb)},
      {&P->cnt, sz(24)},
      {&P->theta2, sz(8)},
      {&P->scratch, sz(32 + 8 * d)},
      {&P->tail, sz(8 * std::max<int64_t>(kMaxD, d * r * d))},
      {&P->cands, sz(4 * sumK)},
      {&P->latM, sz(4 * std::max(d, Lm))},
      {&P->latoff, sz(8 * (std::max(nl, Lm) + 1))},
      {&P->mask, sz(4 * std::max(woff, ceil_div(nc, 32)))},
      {&P->gmask, sz(4 * ceil_div(nc, 32))},
      {&P->J, sz(4 * nc * d)},
      {&P->Jnext, sz(4 * nc * d)},
      {&P->Iprev, sz(4 * nc * d)},
      {&P->assign, sz(8 * nc)},
      {&P->lists, sz(8 * nc + 8 * (Lm + 2) + 4 * Lm * (d + 1))},
      {&P->famcov, sz(nc)},
      {&P->fambins, sz(4 * nc * T)},
      {&P->famscores, sz(4 * T)},
      {&P->famz, sz(4 * T * d)},
      {&P->famcounts, sz(4 * T * par.lattice_mmax)},
      {&P->famlog, sz(8 * Lm)},
      {&P->famstate, sz(32)},
  };
  for (int t = 0; t < d; ++t) v.push_back({&P->I1[t], sz(4 * (pb.k_hi[t] - pb.k_lo[t] + 1))});
  if (P->interp) v.push_back({&P->Umesh, sz(ub * P->G_mesh * nsb)});
  v.push_back({&P->segbuf, sz(sizeof(SolveSeg))});
  v.push_back({C, sz(16 * nc * G)});
  return v;
}

static size_t ws_total(const std::vector<WsItem>& v) {
  size_t b = 0;
  for (const WsItem& w : v) b += w.bytes;
  return b;
}

// detect() with every transient buffer carved from the caller's workspace;
// the plan's own buffers are set aside and restored afterwards.
static void detect_ws(usfft_plan_s* P, uint64_t seed, int64_t ncand, int64_t nsamp, void* ws, size_t ws_bytes,
                      hipStream_t st, usfft_result_s* R, bool given, const int32_t* given_I, int64_t given_n) {
  USFFT_REQUIRE(ncand >= 1 && nsamp >= 1, USFFT_EINVAL, "n_cand_max and samples_max must be >= 1");
  USFFT_REQUIRE(ws != nullptr, USFFT_EINVAL, "null workspace");
  std::vector<WsItem> items = ws_items(P, &R->C, ncand, nsamp);
  const size_t need = ws_total(items);
  USFFT_REQUIRE(ws_bytes >= need, USFFT_ENOMEM,
                "workspace of " + std::to_string(ws_bytes) + " bytes, these bounds need " + std::to_string(need));
  USFFT_REQUIRE(((uintptr_t)ws & 255) == 0, USFFT_EINVAL, "the workspace must be 256-byte aligned");
  std::vector<DevBuf> saved(items.size());
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    saved[i] = std::move(*items[i].buf);
    items[i].buf->borrow(base + off, items[i].bytes);
    off += items[i].bytes;
  }
  auto restore = [&] {
    // the output matrix stays borrowed: the result refers into the workspace
    for (size_t i = 0; i + 1 < items.size(); ++i) *items[i].buf = std::move(saved[i]);
    P->ws_mode = false;
    P->ws_nsamp = 0;
    P->ws_ncand = 0;
  };
  P->ws_mode = true;
  P->ws_nsamp = nsamp;
  P->ws_ncand = ncand;
  try {
    detect(P, seed, st, R, given, given_I, given_n);
  } catch (...) {
    restore();
    throw;
  }
  restore();
  R->stats.workspace_bytes = (int64_t)need;
}

// ---------------------------------------------------------------- autotune
// One process-wide tuning cache, persisted as JSON by usfft_tune_save and
// read back by usfft_tune_load:
//   {"version": 1, "entries": [{"key": "...", "a": A, "b": B, "time_ms": T}, ...]}
// Keys: "jacobi n=.. d=.. prec=.." (a = solver shape), "dst n=.. d=.. prec=..
// model=.." (a = scratch variant), "rader L=.. fp32=.. G=.." (a = workgroup
// size, b = node pairs per workgroup).  Entries are filled on first use by
// timing every candidate on the device; a loaded entry is used as is.
struct TuneEntry {
  int a = 0, b = 0;
  double time_ms = 0.0;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;

static bool tune_get(const std::string& key, TuneEntry* e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *e = it->second;
  return true;
}
static void tune_put(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = e;
}

// Device time of f() on st (ms), after one untimed call.
template <typename F>
static float time_on(hipStream_t st, F&& f) {
  hipEvent_t a, b;
  USFFT_HIP(hipEventCreate(&a));
  USFFT_HIP(hipEventCreate(&b));
  float ms = 0;
  try {
    f();
    USFFT_HIP(hipEventRecord(a, st));
    f();
    USFFT_HIP(hipEventRecord(b, st));
    USFFT_HIP(hipEventSynchronize(b));
    USFFT_HIP(hipEventElapsedTime(&ms, a, b));
  } catch (...) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

// Seeded sampling nodes for tuning runs (ns x d, uniform on [0,1)).
static void tune_nodes(DevBuf& Y, int64_t ns, int d) {
  std::vector<double> yh((size_t)ns * d);
  for (int64_t e = 0; e < ns * d; ++e) yh[e] = rng::uniform01(12345, 77, e);
  Y.ensure(sizeof(double) * yh.size());
  USFFT_HIP(hipMemcpy(Y.p, yh.data(), sizeof(double) * yh.size(), hipMemcpyHostToDevice));
}

static int autotune_solver(usfft_plan_s* P) {
  const int n = P->prob.mesh_n, d = P->prob.d, prec = P->par.precision;
  const std::string key =
      "jacobi n=" + std::to_string(n) + " d=" + std::to_string(d) + " prec=" + std::to_string(prec);
  TuneEntry e;
  if (tune_get(key, &e)) return e.a;
  const int64_t G = P->G;
  const int64_t ns = 1024;
  hipStream_t st = nullptr;
  DevBuf Y, U, it, scr;
  tune_nodes(Y, ns, d);
  U.ensure(sizeof(double) * G * ns);
  it.ensure(sizeof(int32_t) * ns);
  e.a = solver_default_config(n);
  e.time_ms = 1e30;
  for (int c = 0; c < solver_config_count(); ++c) {
    if (!solver_config_fits(c, n)) continue;
    const int wb = persistent_blocks(c, n);
    scr.ensure(sizeof(double) * (size_t)edge_scratch_doubles(n, wb));
    const float ms = time_on(st, [&] {
      launch_pde_solve(c, P->pde, prec, Y.as<double>(), ns, P->par.pcg_rtol, P->par.pcg_maxit, P->par.inner_rtol,
                       P->par.refine_every, U.p, 0, ns, 0, it.as<int32_t>(), scr.as<double>(), wb, st);
    });
    if (ms < e.time_ms) {
      e.time_ms = ms;
      e.a = c;
    }
  }
  tune_put(key, e);
  return e.a;
}

// Scratch variant of the DST-preconditioned solver (0 global scratch, 1
// LDS-resident, 2 compact float32), timed on 2048 seeded solves.
static int autotune_dst_variant(usfft_plan_s* P, int fallback) {
  const int n = P->prob.mesh_n, d = P->prob.d, prec = P->par.precision;
  const std::string key = "dst n=" + std::to_string(n) + " d=" + std::to_string(d) + " prec=" +
                          std::to_string(prec) + " model=" + std::to_string(P->prob.model);
  TuneEntry e;
  if (tune_get(key, &e) && e.a >= 0 && e.a <= (prec == USFFT_FP32_REFINE ? 2 : 1)) return e.a;
  if (!P->par.autotune) return fallback;
  const int64_t ns = 2048, G = (int64_t)(n - 1) * (n - 1);
  hipStream_t st = nullptr;
  DevBuf Y, U, it, scr;
  tune_nodes(Y, ns, d);
  const int ufp32 = prec == USFFT_FP32_REFINE ? 1 : 0;
  U.ensure((ufp32 ? sizeof(float) : sizeof(double)) * G * ns);
  it.ensure(sizeof(int32_t) * ns);
  DevBuf sg;
  {
    const SolveSeg seg{P->pde, Y.as<double>(), U.p, ns, 0, 0, it.as<int32_t>()};
    sg.ensure(sizeof(SolveSeg));
    USFFT_HIP(hipMemcpy(sg.p, &seg, sizeof(SolveSeg), hipMemcpyHostToDevice));
  }
  e.a = fallback;
  e.time_ms = 1e30;
  for (int v = 0; v <= (ufp32 ? 2 : 1); ++v) {
    const int wb = dst_persistent_blocks(n, prec, v);
    scr.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, dst_scratch_doubles(n, v, wb)));
    const float ms = time_on(st, [&] {
      launch_pde_solve_dst(sg.as<SolveSeg>(), 1, n, prec, v, ns, P->par.pcg_rtol, P->par.pcg_maxit,
                           P->par.inner_rtol, P->par.refine_every, ufp32, scr.as<double>(), wb, P->d_sfrag.p,
                           P->d_lam.as<float>(), st);
    });
    if (ms < e.time_ms) {
      e.time_ms = ms;
      e.a = v;
    }
  }
  tune_put(key, e);
  return e.a;
}

// Workgroup shape of a batched lattice DFT whose longest transform is Lmax:
// the cached one, else (autotune on) every admissible (block, cols) timed on
// the launch itself (the transforms only read the samples, so repeating them
// leaves the same output), else the built-in rule (0, 0).
static std::pair<int, int> rader_tuned_shape(usfft_plan_s* P, int Lmax, int ufp32, int64_t G,
                                             const std::function<void(int, int)>& launch, hipStream_t st) {
  const std::string key = "rader L=" + std::to_string(Lmax) + " fp32=" + std::to_string(ufp32) + " G=" +
                          std::to_string(G);
  TuneEntry e;
  if (tune_get(key, &e) && rader_shape_ok(Lmax, ufp32, e.a, e.b)) return {e.a, e.b};
  if (!P->par.autotune) return {0, 0};
  e.time_ms = 1e30;
  for (int blk : {128, 256, 512})
    for (int cols : {1, 2, 4}) {
      if (!rader_shape_ok(Lmax, ufp32, blk, cols)) continue;
      const float ms = time_on(st, [&] { launch(blk, cols); });
      if (ms < e.time_ms) {
        e.time_ms = ms;
        e.a = blk;
        e.b = cols;
      }
    }
  tune_put(key, e);
  return {e.a, e.b};
}

// ---------------------------------------------------------------- plan
static void validate(const usfft_problem* pb, const usfft_params* par) {
  USFFT_REQUIRE(pb && par, USFFT_EINVAL, "null problem or params");
  USFFT_REQUIRE(pb->d >= 1 && pb->d <= kMaxD, USFFT_EINVAL, "d must be in [1, 64]");
  USFFT_REQUIRE(pb->k_lo && pb->k_hi, USFFT_EINVAL, "missing search box");
  for (int j = 0; j < pb->d; ++j) {
    const int K = pb->k_hi[j] - pb->k_lo[j] + 1;
    USFFT_REQUIRE(K >= 1 && K <= 1024, USFFT_EINVAL, "box extent K_t must be in [1, 1024]");
  }
  USFFT_REQUIRE(par->s >= 1 && par->s_local >= par->s && par->r >= 1, USFFT_EINVAL,
                "need s >= 1, s_local >= s, r >= 1");
  USFFT_REQUIRE(par->theta >= 0 && par->tie_rel >= 0 && par->tie_rel < 1, USFFT_EINVAL, "bad theta / tie_rel");
  USFFT_REQUIRE(par->precision == USFFT_FP64 || par->precision == USFFT_FP32_REFINE, USFFT_EINVAL, "bad precision");
  USFFT_REQUIRE(par->lattice_c > 0 && par->lattice_tries >= 1 && par->lattice_max >= 1 &&
                    par->lattice_mmax >= 3 &&
                    par->lattice_mmax <= lattice_mmax_for(par->precision == USFFT_FP32_REFINE ? 1 : 0),
                USFFT_EINVAL, "bad lattice parameters (lattice_mmax <= 9601, float32: <= 19201)");
  USFFT_REQUIRE(par->pcg_rtol > 0 && par->pcg_maxit >= 1 && par->inner_rtol > 0 && par->refine_every >= 1,
                USFFT_EINVAL, "bad solver parameters");
  USFFT_REQUIRE(par->precond == USFFT_PRECOND_DST || par->precond == USFFT_PRECOND_JACOBI, USFFT_EINVAL,
                "bad preconditioner");
  USFFT_REQUIRE(pb->n_nodes >= 0 && pb->n_nodes <= (int64_t)1 << 30, USFFT_EINVAL, "bad n_nodes");
  if (pb->sampler == USFFT_SAMPLER_PDE || pb->sampler == USFFT_SAMPLER_PDE_MESH) {
    if (pb->sampler == USFFT_SAMPLER_PDE)
      USFFT_REQUIRE(pb->mesh_n >= 4 && pb->mesh_n <= kMaxMeshStream, USFFT_EINVAL, "mesh_n must be in [4, 512]");
    else
      USFFT_REQUIRE(pb->mesh_nv >= 3 && pb->mesh_nt >= 1 && pb->mesh_xy && pb->mesh_tri && pb->mesh_boundary,
                    USFFT_EINVAL, "bad triangulation");
    USFFT_REQUIRE(pb->amp && pb->mode1 && pb->mode2, USFFT_EINVAL, "missing coefficient family");
    USFFT_REQUIRE(pb->model >= USFFT_MODEL_PERIODIC && pb->model <= USFFT_MODEL_LOGNORMAL, USFFT_EINVAL,
                  "unknown coefficient model");
    USFFT_REQUIRE(pb->model != USFFT_MODEL_AFFINE || pb->beta > pb->alpha, USFFT_EINVAL,
                  "affine model needs alpha < beta");
    USFFT_REQUIRE((pb->basis1 == 0 || pb->basis1 == 1) && (pb->basis2 == 0 || pb->basis2 == 1), USFFT_EINVAL,
                  "basis must be 0 (sin) or 1 (cos)");
    USFFT_REQUIRE(pb->model != USFFT_MODEL_LOGNORMAL || pb->delta < 0.5, USFFT_EINVAL,
                  "lognormal shift must lie in (0, 1/2)");
  } else {
    USFFT_REQUIRE(pb->sampler == USFFT_SAMPLER_TRIG_POLY, USFFT_EINVAL, "unknown sampler");
    USFFT_REQUIRE(pb->G_poly >= 1 && pb->n_poly >= 1 && pb->poly_k && pb->poly_c, USFFT_EINVAL,
                  "bad trigonometric polynomial");
  }
}

// Host preparation of a general triangulation: inner-vertex numbering,
// element geometry, the CSR pattern of inner couplings with the (triangle,
// weight) contributions of every entry (triangles in order, vertex pairs in
// order), the load for f = 1 and the basis of every term at the centroids.
static void build_mesh(usfft_plan_s* P, const usfft_problem* pb, const usfft_params* par) {
  const int d = pb->d, nv = pb->mesh_nv, nt = pb->mesh_nt;
  P->amp.assign(pb->amp, pb->amp + d);
  P->mode1.assign(pb->mode1, pb->mode1 + d);
  P->mode2.assign(pb->mode2, pb->mode2 + d);
  P->prob.amp = P->amp.data();
  P->prob.mode1 = P->mode1.data();
  P->prob.mode2 = P->mode2.data();
  P->prob.mesh_xy = nullptr;
  P->prob.mesh_tri = nullptr;
  P->prob.mesh_boundary = nullptr;
  std::vector<int> gid(nv, -1);
  int G = 0;
  for (int v = 0; v < nv; ++v)
    if (!pb->mesh_boundary[v]) gid[v] = G++;
  USFFT_REQUIRE(G >= 1, USFFT_EINVAL, "the mesh needs at least one inner vertex");
  std::vector<double> kgeo((size_t)nt * 9), area(nt), cx(nt), cy(nt);
  for (int t = 0; t < nt; ++t) {
    int v[3];
    for (int a = 0; a < 3; ++a) {
      v[a] = pb->mesh_tri[3 * t + a];
      USFFT_REQUIRE(v[a] >= 0 && v[a] < nv, USFFT_EINVAL, "triangle vertex out of range");
    }
    const double x0 = pb->mesh_xy[2 * v[0]], y0 = pb->mesh_xy[2 * v[0] + 1];
    const double e1x = pb->mesh_xy[2 * v[1]] - x0, e1y = pb->mesh_xy[2 * v[1] + 1] - y0;
    const double e2x = pb->mesh_xy[2 * v[2]] - x0, e2y = pb->mesh_xy[2 * v[2] + 1] - y0;
    const double det = e1x * e2y - e1y * e2x;
    USFFT_REQUIRE(std::fabs(det) > 0.0, USFFT_EINVAL, "degenerate triangle");
    area[t] = 0.5 * std::fabs(det);
    // gradients of the barycentric functions (rows of the inverse Jacobian)
    const double g[3][2] = {{-(e2y - e1y) / det, -(e1x - e2x) / det}, {e2y / det, -e2x / det},
                            {-e1y / det, e1x / det}};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) kgeo[(size_t)t * 9 + a * 3 + b] = area[t] * (g[a][0] * g[b][0] + g[a][1] * g[b][1]);
    cx[t] = (x0 + pb->mesh_xy[2 * v[1]] + pb->mesh_xy[2 * v[2]]) / 3.0;
    cy[t] = (y0 + pb->mesh_xy[2 * v[1] + 1] + pb->mesh_xy[2 * v[2] + 1]) / 3.0;
  }
  // CSR pattern
  std::vector<std::vector<int>> adj(G);
  for (int t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        const int ga = gid[pb->mesh_tri[3 * t + a]], gb = gid[pb->mesh_tri[3 * t + b]];
        if (ga >= 0 && gb >= 0) adj[ga].push_back(gb);
      }
  std::vector<int> rowptr(G + 1, 0), col, diag(G);
  for (int i = 0; i < G; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
    rowptr[i + 1] = rowptr[i] + (int)adj[i].size();
    for (int j : adj[i]) {
      if (j == i) diag[i] = (int)col.size();
      col.push_back(j);
    }
  }
  const int nnz = (int)col.size();
  auto entry = [&](int i, int j) {
    return (int)(std::lower_bound(col.begin() + rowptr[i], col.begin() + rowptr[i + 1], j) - col.begin());
  };
  std::vector<int> cnt(nnz + 1, 0);
  for (int pass = 0; pass < 2; ++pass) {
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    std::vector<int> ctri(pass ? cnt[nnz] : 0);
    std::vector<double> cw(pass ? cnt[nnz] : 0);
    for (int t = 0; t < nt; ++t)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const int ga = gid[pb->mesh_tri[3 * t + a]], gb = gid[pb->mesh_tri[3 * t + b]];
          if (ga < 0 || gb < 0) continue;
          const int e = entry(ga, gb);
          if (!pass) {
            ++cnt[e + 1];
          } else {
            ctri[fill[e]] = t;
            cw[fill[e]++] = kgeo[(size_t)t * 9 + a * 3 + b];
          }
        }
    if (!pass) {
      for (int e = 0; e < nnz; ++e) cnt[e + 1] += cnt[e];
    } else {
      P->m_cptr.ensure(sizeof(int) * cnt.size());
      P->m_ctri.ensure(sizeof(int) * ctri.size());
      P->m_cw.ensure(sizeof(double) * cw.size());
      USFFT_HIP(hipMemcpy(P->m_cptr.p, cnt.data(), sizeof(int) * cnt.size(), hipMemcpyHostToDevice));
      USFFT_HIP(hipMemcpy(P->m_ctri.p, ctri.data(), sizeof(int) * ctri.size(), hipMemcpyHostToDevice));
      USFFT_HIP(hipMemcpy(P->m_cw.p, cw.data(), sizeof(double) * cw.size(), hipMemcpyHostToDevice));
    }
  }
  std::vector<double> load(G, 0.0);
  for (int t = 0; t < nt; ++t)
    for (int a = 0; a < 3; ++a) {
      const int ga = gid[pb->mesh_tri[3 * t + a]];
      if (ga >= 0) load[ga] += area[t] / 3.0;
    }
  std::vector<double> psi((size_t)d * nt);
  auto b1 = [&](double v) { return pb->basis1 == 1 ? std::cos(v) : std::sin(v); };
  auto b2 = [&](double v) { return pb->basis2 == 1 ? std::cos(v) : std::sin(v); };
  for (int k = 0; k < d; ++k)
    for (int t = 0; t < nt; ++t)
      psi[(size_t)k * nt + t] = b1(P->mode1[k] * M_PI * cx[t]) * b2(P->mode2[k] * M_PI * cy[t]);
  auto up = [&](usfft::DevBuf& B, const void* src, size_t bytes) {
    B.ensure(std::max<size_t>(bytes, 8));
    USFFT_HIP(hipMemcpy(B.p, src, bytes, hipMemcpyHostToDevice));
  };
  up(P->m_rowptr, rowptr.data(), sizeof(int) * rowptr.size());
  up(P->m_col, col.data(), sizeof(int) * col.size());
  up(P->m_diag, diag.data(), sizeof(int) * diag.size());
  up(P->m_load, load.data(), sizeof(double) * load.size());
  up(P->m_psi, psi.data(), sizeof(double) * psi.size());
  up(P->d_amp, P->amp.data(), sizeof(double) * d);
  P->G = G;
  MeshDev& M = P->mesh;
  M.G = G;
  M.nt = nt;
  M.nnz = nnz;
  M.rowptr = P->m_rowptr.as<int>();
  M.col = P->m_col.as<int>();
  M.diag = P->m_diag.as<int>();
  M.cptr = P->m_cptr.as<int>();
  M.ctri = P->m_ctri.as<int>();
  M.cw = P->m_cw.as<double>();
  M.load = P->m_load.as<double>();
  M.psi = P->m_psi.as<double>();
  P->mesh_blocks = mesh_persistent_blocks(M);
  // meshes beyond the LDS solver keep each workgroup's state in a scratch slot
  if (!mesh_fits_lds(M))
    P->d_wscr.ensure(sizeof(double) * (size_t)mesh_scratch_doubles(M) * (size_t)P->mesh_blocks);
  P->pde.n = 0;
  P->pde.d = d;
  P->pde.a0 = pb->a0;
  P->pde.h2 = 0.0;
  P->pde.amp = P->d_amp.as<double>();
  P->pde.tab = nullptr;
  P->pde.model = pb->model;
  P->pde.alpha = pb->alpha;
  P->pde.beta = pb->beta;
  P->pde.delta = pb->delta > 0 ? pb->delta : 1.0 / (4.0 * par->lattice_mmax);
}

// Interpolation of the P1 solution to the caller's points (Sec. 3.1): the
// containing triangle of every point and its barycentric coordinates.
// Uniform mesh: the cell from the scaled coordinates, then the triangle below
// or above the cell's diagonal.  General triangulation: candidate triangles
// from a bucket grid over the unit square, in triangle order.  Boundary
// vertices carry the Dirichlet value 0 and drop out.
static void build_interp(usfft_plan_s* P, const usfft_problem* pb) {
  const int64_t np = pb->n_nodes;
  USFFT_REQUIRE(pb->nodes_xy != nullptr, USFFT_EINVAL, "n_nodes > 0 needs nodes_xy");
  USFFT_REQUIRE(pb->sampler == USFFT_SAMPLER_PDE || pb->sampler == USFFT_SAMPLER_PDE_MESH, USFFT_EINVAL,
                "a node set T_G given by points needs a PDE sampler");
  std::vector<int32_t> idx((size_t)np * 3, -1);
  std::vector<double> w((size_t)np * 3, 0.0);
  auto inside_unit = [](double x) { return x >= 0.0 && x <= 1.0; };
  if (pb->sampler == USFFT_SAMPLER_PDE) {
    const int n = pb->mesh_n;
    auto inner = [n](int a, int b) { return (a >= 1 && a <= n - 1 && b >= 1 && b <= n - 1) ? (b - 1) * (n - 1) + (a - 1) : -1; };
    for (int64_t p = 0; p < np; ++p) {
      const double x = pb->nodes_xy[2 * p], y = pb->nodes_xy[2 * p + 1];
      USFFT_REQUIRE(inside_unit(x) && inside_unit(y), USFFT_EINVAL, "a node lies outside the unit square");
      const int i = std::min((int)std::floor(x * n), n - 1), j = std::min((int)std::floor(y * n), n - 1);
      const double xi = x * n - i, eta = y * n - j;
      int v[3][2];
      double l[3];
      if (xi >= eta) {  // triangle (i,j), (i+1,j), (i+1,j+1)
        v[0][0] = i; v[0][1] = j; v[1][0] = i + 1; v[1][1] = j; v[2][0] = i + 1; v[2][1] = j + 1;
        l[0] = 1.0 - xi; l[1] = xi - eta; l[2] = eta;
      } else {          // triangle (i,j), (i,j+1), (i+1,j+1)
        v[0][0] = i; v[0][1] = j; v[1][0] = i; v[1][1] = j + 1; v[2][0] = i + 1; v[2][1] = j + 1;
        l[0] = 1.0 - eta; l[1] = eta - xi; l[2] = xi;
      }
      for (int a = 0; a < 3; ++a) {
        idx[3 * p + a] = inner(v[a][0], v[a][1]);
        w[3 * p + a] = idx[3 * p + a] >= 0 ? l[a] : 0.0;
      }
    }
    P->G_mesh = (int64_t)(n - 1) * (n - 1);
  } else {
    const int nv = pb->mesh_nv, nt = pb->mesh_nt;
    std::vector<int> gid(nv, -1);
    int gm = 0;
    for (int v = 0; v < nv; ++v)
      if (!pb->mesh_boundary[v]) gid[v] = gm++;
    constexpr int NB = 64;
    std::vector<std::vector<int>> bucket(NB * NB);
    auto cell = [](double c) { return std::min(NB - 1, std::max(0, (int)std::floor(c * NB))); };
    for (int t = 0; t < nt; ++t) {
      double x0 = 2, x1 = -1, y0 = 2, y1 = -1;
      for (int a = 0; a < 3; ++a) {
        const int v = pb->mesh_tri[3 * t + a];
        x0 = std::min(x0, pb->mesh_xy[2 * v]);
        x1 = std::max(x1, pb->mesh_xy[2 * v]);
        y0 = std::min(y0, pb->mesh_xy[2 * v + 1]);
        y1 = std::max(y1, pb->mesh_xy[2 * v + 1]);
      }
      for (int bj = cell(y0); bj <= cell(y1); ++bj)
        for (int bi = cell(x0); bi <= cell(x1); ++bi) bucket[bj * NB + bi].push_back(t);
    }
    for (int64_t p = 0; p < np; ++p) {
      const double x = pb->nodes_xy[2 * p], y = pb->nodes_xy[2 * p + 1];
      USFFT_REQUIRE(inside_unit(x) && inside_unit(y), USFFT_EINVAL, "a node lies outside the unit square");
      bool found = false;
      for (int t : bucket[cell(y) * NB + cell(x)]) {
        const int* tv = pb->mesh_tri + 3 * t;
        const double ax = pb->mesh_xy[2 * tv[0]], ay = pb->mesh_xy[2 * tv[0] + 1];
        const double bx = pb->mesh_xy[2 * tv[1]] - ax, by = pb->mesh_xy[2 * tv[1] + 1] - ay;
        const double cx = pb->mesh_xy[2 * tv[2]] - ax, cy = pb->mesh_xy[2 * tv[2] + 1] - ay;
        const double det = bx * cy - by * cx, rx = x - ax, ry = y - ay;
        const double l1 = (rx * cy - ry * cx) / det, l2 = (bx * ry - by * rx) / det, l0 = 1.0 - l1 - l2;
        if (std::min(l0, std::min(l1, l2)) < -1e-12) continue;
        const double l[3] = {l0, l1, l2};
        for (int a = 0; a < 3; ++a) {
          idx[3 * p + a] = gid[tv[a]];
          w[3 * p + a] = gid[tv[a]] >= 0 ? l[a] : 0.0;
        }
        found = true;
        break;
      }
      USFFT_REQUIRE(found, USFFT_EINVAL, "a node lies outside the triangulation");
    }
    P->G_mesh = gm;
  }
  P->d_iidx.ensure(sizeof(int32_t) * idx.size());
  P->d_iw.ensure(sizeof(double) * w.size());
  USFFT_HIP(hipMemcpy(P->d_iidx.p, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice));
  USFFT_HIP(hipMemcpy(P->d_iw.p, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice));
  P->interp = true;
}

static usfft_plan_s* plan_create(const usfft_problem* pb, const usfft_params* par) {
  validate(pb, par);
  std::unique_ptr<usfft_plan_s> P(new usfft_plan_s());
  P->prob = *pb;
  P->par = *par;
  const int d = pb->d;
  P->k_lo.assign(pb->k_lo, pb->k_lo + d);
  P->k_hi.assign(pb->k_hi, pb->k_hi + d);
  P->prob.k_lo = P->k_lo.data();
  P->prob.k_hi = P->k_hi.data();
  if (pb->sampler == USFFT_SAMPLER_PDE) {
    const int n = pb->mesh_n;
    P->G = (int64_t)(n - 1) * (n - 1);
    P->amp.assign(pb->amp, pb->amp + d);
    P->mode1.assign(pb->mode1, pb->mode1 + d);
    P->mode2.assign(pb->mode2, pb->mode2 + d);
    P->prob.amp = P->amp.data();
    P->prob.mode1 = P->mode1.data();
    P->prob.mode2 = P->mode2.data();
    // sin or cos(m pi x) at the centroid abscissae: lower triangle (i+2/3, j+1/3) h,
    // upper triangle (i+1/3, j+2/3) h of cell (i, j)
    const int S = usfft::row_tab_pitch(n);
    std::vector<double> tab((size_t)4 * d * n + (size_t)2 * d * S);
    const double h = 1.0 / n;
    auto b1 = [&](double v) { return pb->basis1 == 1 ? std::cos(v) : std::sin(v); };
    auto b2 = [&](double v) { return pb->basis2 == 1 ? std::cos(v) : std::sin(v); };
    for (int k = 0; k < d; ++k)
      for (int c = 0; c < n; ++c) {
        tab[(size_t)(0 * d + k) * n + c] = b1(P->mode1[k] * M_PI * (c + 2.0 / 3.0) * h);
        tab[(size_t)(1 * d + k) * n + c] = b1(P->mode1[k] * M_PI * (c + 1.0 / 3.0) * h);
        tab[(size_t)(2 * d + k) * n + c] = b2(P->mode2[k] * M_PI * (c + 1.0 / 3.0) * h);
        tab[(size_t)(3 * d + k) * n + c] = b2(P->mode2[k] * M_PI * (c + 2.0 / 3.0) * h);
      }
    for (int q = 0; q < 2; ++q)
      for (int k = 0; k < d; ++k)
        for (int e = 0; e < S; ++e)
          tab[(size_t)4 * d * n + (size_t)(q * d + k) * S + e] =
              tab[(size_t)((2 + q) * d + k) * n + std::min(std::max(e - 1, 0), n - 1)];
    P->d_amp.ensure(sizeof(double) * d);
    P->d_tab.ensure(sizeof(double) * tab.size());
    USFFT_HIP(hipMemcpy(P->d_amp.p, P->amp.data(), sizeof(double) * d, hipMemcpyHostToDevice));
    USFFT_HIP(hipMemcpy(P->d_tab.p, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice));
    P->pde.n = n;
    P->pde.d = d;
    P->pde.a0 = pb->a0;
    P->pde.h2 = h * h;
    P->pde.amp = P->d_amp.as<double>();
    P->pde.tab = P->d_tab.as<double>();
    P->pde.model = pb->model;
    P->pde.alpha = pb->alpha;
    P->pde.beta = pb->beta;
    // Lemma 3.1 for the largest admissible lattice: every lattice and line
    // node (odd sizes <= lattice_mmax) stays at least delta from the poles
    P->pde.delta = pb->delta > 0 ? pb->delta : 1.0 / (4.0 * par->lattice_mmax);
    if (par->precond == USFFT_PRECOND_DST && dst_padded(n) > 0) {
      // fast-Poisson preconditioned PCG on the matrix cores
      P->dst = true;
      P->solver_cfg = -1;
      const int mp = dst_padded(n);
      P->d_sfrag.ensure((size_t)dst_frag_bytes(mp));
      P->d_lam.ensure(sizeof(float) * mp);
      dst_tables_build(n, P->d_sfrag.p, P->d_lam.as<float>(), nullptr);
      USFFT_HIP(hipStreamSynchronize(nullptr));
      // solver_config 0 / 1 / 2 forces the scratch placement: 0 global
      // scratch, 1 LDS-resident (one workgroup per CU), 2 compact float32
      // (float32 edges in LDS, float64 edges in global scratch, two
      // workgroups per CU at h = 1/64).  Defaults: 2 for float32 solves, 1
      // for float64 solves.
      USFFT_REQUIRE(par->solver_config <= 2, USFFT_EINVAL, "solver_config of the DST solver must be <= 2");
      USFFT_REQUIRE(!(par->solver_config == 2 && par->precision == USFFT_FP64), USFFT_EINVAL,
                    "solver_config 2 of the DST solver is float32-only");
      P->dst_variant = par->solver_config >= 0 ? par->solver_config : (par->precision == USFFT_FP64 ? 1 : 2);
      if (par->solver_config < 0) P->dst_variant = autotune_dst_variant(P.get(), P->dst_variant);
      P->wblocks = dst_persistent_blocks(n, par->precision, P->dst_variant);
      P->d_wscr.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, dst_scratch_doubles(n, P->dst_variant,
                                                                                         P->wblocks)));
    } else if (par->precond == USFFT_PRECOND_DST && dst_stream_ok(n)) {
      // per-sample state exceeds one CU, the preconditioner still fits it:
      // streaming float64 PCG with the fast-Poisson preconditioner (MP = 128)
      P->dst_stream = true;
      P->solver_cfg = -1;
      P->d_sfrag.ensure((size_t)dst_frag_bytes(128));
      P->d_lam.ensure(sizeof(float) * 128);
      dst_stream_tables_build(n, P->d_sfrag.p, P->d_lam.as<float>(), nullptr);
      USFFT_HIP(hipStreamSynchronize(nullptr));
      P->wblocks = dst_stream_blocks();
      P->d_stream.ensure(sizeof(double) * (size_t)dst_stream_workspace_doubles(n, P->wblocks));
    } else if (par->precond == USFFT_PRECOND_DST && tl_stream_ok(n)) {
      // the fast-Poisson preconditioner moves to the mesh of width 2h
      // (two-level, additive with scaled Jacobi); its tables are those of n / 2
      P->tl_stream = true;
      P->solver_cfg = -1;
      P->d_sfrag.ensure((size_t)dst_frag_bytes(128));
      P->d_lam.ensure(sizeof(float) * 128);
      dst_stream_tables_build(n / 2, P->d_sfrag.p, P->d_lam.as<float>(), nullptr);
      USFFT_HIP(hipStreamSynchronize(nullptr));
      P->wblocks = tl_stream_blocks();
      P->d_stream.ensure(sizeof(double) * (size_t)tl_stream_workspace_doubles(P->wblocks));
    } else if (n > kMaxMesh) {
      // per-sample state exceeds one CU: streaming float64 solver
      P->streaming = true;
      P->solver_cfg = -1;
      P->d_stream.ensure(sizeof(double) * (size_t)stream_workspace_doubles(n, kStreamBlocks));
    } else if (par->solver_config >= 0) {
      USFFT_REQUIRE(par->solver_config < solver_config_count() && solver_config_fits(par->solver_config, n),
                    USFFT_EINVAL, "solver_config does not fit this mesh");
      P->solver_cfg = par->solver_config;
    } else if (par->solver_config == -2) {
      P->solver_cfg = solver_default_config(n);
    } else {
      P->solver_cfg = autotune_solver(P.get());
    }
    USFFT_REQUIRE(P->dst || P->dst_stream || P->tl_stream || P->streaming || P->solver_cfg >= 0, USFFT_EINVAL,
                  "no solver shape for this mesh");
    if (!P->streaming && !P->dst && !P->dst_stream && !P->tl_stream) {
      P->wblocks = persistent_blocks(P->solver_cfg, n);
      P->d_wscr.ensure(sizeof(double) * (size_t)edge_scratch_doubles(n, P->wblocks));
    }
  } else if (pb->sampler == USFFT_SAMPLER_PDE_MESH) {
    build_mesh(P.get(), pb, par);
  } else {
    P->G = pb->G_poly;
    P->poly_k.assign(pb->poly_k, pb->poly_k + (size_t)pb->n_poly * d);
    P->poly_c.assign(pb->poly_c, pb->poly_c + (size_t)pb->n_poly * pb->G_poly * 2);
    P->d_polyk.ensure(sizeof(int32_t) * P->poly_k.size());
    P->d_polyc.ensure(sizeof(double) * P->poly_c.size());
    USFFT_HIP(hipMemcpy(P->d_polyk.p, P->poly_k.data(), sizeof(int32_t) * P->poly_k.size(), hipMemcpyHostToDevice));
    USFFT_HIP(hipMemcpy(P->d_polyc.p, P->poly_c.data(), sizeof(double) * P->poly_c.size(), hipMemcpyHostToDevice));
    P->prob.poly_k = P->poly_k.data();
    P->prob.poly_c = P->poly_c.data();
  }
  if (pb->n_nodes > 0) {
    build_interp(P.get(), pb);
    P->G = pb->n_nodes;
  }
  P->prob.nodes_xy = nullptr;
  // lattice tables: one slot per admissible size up to lattice_mmax
  {
    size_t off = 0;
    for (int M : admissible_sizes(3, par->lattice_mmax)) {
      P->rader_off[M] = off;
      off += rader_table_bytes(M);
    }
    P->d_rader.ensure(std::max<size_t>(off, 256));
  }
  // pinned staging of small uploads and readbacks
  P->stage_cap = 4u << 20;
  USFFT_HIP(hipHostMalloc(reinterpret_cast<void**>(&P->stage), P->stage_cap, hipHostMallocDefault));
  P->back_cap = 1u << 20;
  USFFT_HIP(hipHostMalloc(reinterpret_cast<void**>(&P->back), P->back_cap, hipHostMallocDefault));
  return P.release();
}

template <typename F>
static usfft_status guarded(F&& f) {
  try {
    f();
    return USFFT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.st;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return USFFT_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return USFFT_EINVAL;
  }
}

}  // namespace usfft

using namespace usfft;

extern "C" {

const char* usfft_last_error(void) { return g_last_error.c_str(); }
const char* usfft_version(void) { return "usfft-gfx950 1.0"; }

usfft_status usfft_plan_create(const usfft_problem* prob, const usfft_params* par, usfft_plan_t* out) {
  return guarded([&] {
    USFFT_REQUIRE(out, USFFT_EINVAL, "null output");
    *out = plan_create(prob, par);
  });
}

void usfft_plan_destroy(usfft_plan_t plan) { delete plan; }

int64_t usfft_plan_nodes(usfft_plan_t plan) { return plan ? plan->G : -1; }

usfft_status usfft_detect(usfft_plan_t plan, uint64_t seed, void* stream, usfft_result_t* out) {
  return guarded([&] {
    USFFT_REQUIRE(plan && out, USFFT_EINVAL, "null plan or output");
    std::lock_guard<std::mutex> lk(plan->mu);
    std::unique_ptr<usfft_result_s> R(new usfft_result_s());
    detect(plan, seed, (hipStream_t)stream, R.get());
    *out = R.release();
  });
}

usfft_status usfft_detect_batch(usfft_plan_t* plans, int32_t n, const uint64_t* seeds, usfft_result_t* out,
                                usfft_status* statuses, int64_t* fuse_stats) {
  return guarded([&] {
    USFFT_REQUIRE(plans && seeds && out && n >= 1 && n <= FuseGroup::kMaxSeg, USFFT_EINVAL,
                  "bad batch arguments (1 <= n <= 64)");
    for (int i = 0; i < n; ++i) {
      USFFT_REQUIRE(plans[i], USFFT_EINVAL, "null plan in batch");
      for (int j = 0; j < i; ++j) USFFT_REQUIRE(plans[j] != plans[i], USFFT_EINVAL, "a plan appears twice in the batch");
      out[i] = nullptr;
    }
    int dev = 0;
    USFFT_HIP(hipGetDevice(&dev));
    FuseGroup F;
    std::vector<int> fused(n, 0);
    for (int i = 0; i < n; ++i) {
      fused[i] = plans[i]->prob.sampler == USFFT_SAMPLER_PDE && plans[i]->dst ? 1 : 0;
      F.active += fused[i];
    }
    std::vector<usfft_status> st(n, USFFT_OK);
    std::vector<std::string> err(n);
    std::vector<std::unique_ptr<usfft_result_s>> res(n);
    std::vector<std::thread> th;
    for (int i = 0; i < n; ++i)
      th.emplace_back([&, i] {
        hipStream_t s = nullptr;
        try {
          USFFT_HIP(hipSetDevice(dev));
          USFFT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
          std::lock_guard<std::mutex> lk(plans[i]->mu);
          plans[i]->fuse = fused[i] ? &F : nullptr;
          res[i].reset(new usfft_result_s());
          detect(plans[i], seeds[i], s, res[i].get());
        } catch (const Error& e) {
          st[i] = e.st;
          err[i] = e.msg;
          res[i].reset();
        } catch (const std::exception& e) {
          st[i] = USFFT_EINVAL;
          err[i] = e.what();
          res[i].reset();
        }
        if (fused[i]) fuse_leave(&F);
        if (s) {
          (void)hipStreamSynchronize(s);
          (void)hipStreamDestroy(s);
        }
      });
    for (auto& t : th) t.join();
    int first_bad = -1;
    for (int i = 0; i < n; ++i) {
      plans[i]->fuse = nullptr;
      if (statuses) statuses[i] = st[i];
      out[i] = res[i].release();
      if (st[i] != USFFT_OK && first_bad < 0) first_bad = i;
    }
    if (fuse_stats) {
      fuse_stats[0] = F.launches;
      fuse_stats[1] = F.fused_launches;
      fuse_stats[2] = F.segments;
    }
    if (first_bad >= 0) throw Error{st[first_bad], "job " + std::to_string(first_bad) + ": " + err[first_bad]};
  });
}

usfft_status usfft_coefficients(usfft_plan_t plan, const int32_t* freqs_host, int64_t n, uint64_t seed,
                                void* stream, usfft_result_t* out) {
  return guarded([&] {
    USFFT_REQUIRE(plan && out && n >= 0 && (n == 0 || freqs_host), USFFT_EINVAL, "bad coefficients arguments");
    const int d = plan->prob.d;
    std::vector<std::vector<int32_t>> rows((size_t)n);
    for (int64_t a = 0; a < n; ++a) rows[a].assign(freqs_host + a * d, freqs_host + (a + 1) * d);
    std::sort(rows.begin(), rows.end());
    USFFT_REQUIRE(std::adjacent_find(rows.begin(), rows.end()) == rows.end(), USFFT_EINVAL,
                  "the frequency set has repeated entries");
    std::lock_guard<std::mutex> lk(plan->mu);
    std::unique_ptr<usfft_result_s> R(new usfft_result_s());
    detect(plan, seed, (hipStream_t)stream, R.get(), true, freqs_host, n);
    *out = R.release();
  });
}

usfft_status usfft_tune_save(const char* path) {
  return guarded([&] {
    USFFT_REQUIRE(path, USFFT_EINVAL, "null path");
    std::ostringstream o;
    o.precision(9);
    o << "{\"version\": 1, \"entries\": [";
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      bool first = true;
      for (const auto& kv : g_tune) {
        o << (first ? "\n  " : ",\n  ") << "{\"key\": \"" << kv.first << "\", \"a\": " << kv.second.a
          << ", \"b\": " << kv.second.b << ", \"time_ms\": " << kv.second.time_ms << "}";
        first = false;
      }
    }
    o << "\n]}\n";
    std::ofstream f(path);
    USFFT_REQUIRE(f.good(), USFFT_EINVAL, std::string("cannot write ") + path);
    f << o.str();
  });
}

usfft_status usfft_tune_load(const char* path) {
  return guarded([&] {
    USFFT_REQUIRE(path, USFFT_EINVAL, "null path");
    std::ifstream f(path);
    USFFT_REQUIRE(f.good(), USFFT_EINVAL, std::string("cannot read ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    // every {...} object that holds a "key": its string and the numbers of
    // "a", "b" and "time_ms" (the file usfft_tune_save writes)
    auto num = [&](const std::string& obj, const char* name, double dflt) {
      const std::string pat = std::string("\"") + name + "\":";
      const size_t p = obj.find(pat);
      if (p == std::string::npos) return dflt;
      return std::strtod(obj.c_str() + p + pat.size(), nullptr);
    };
    std::map<std::string, TuneEntry> got;
    for (size_t p = t.find('{', 1); p != std::string::npos; p = t.find('{', p + 1)) {
      const size_t q = t.find('}', p);
      USFFT_REQUIRE(q != std::string::npos, USFFT_EINVAL, "malformed tuning file");
      const std::string obj = t.substr(p, q - p + 1);
      const size_t k = obj.find("\"key\":");
      if (k == std::string::npos) continue;
      const size_t k0 = obj.find('"', k + 6), k1 = obj.find('"', k0 + 1);
      USFFT_REQUIRE(k0 != std::string::npos && k1 != std::string::npos, USFFT_EINVAL, "malformed tuning key");
      TuneEntry e;
      e.a = (int)num(obj, "a", 0);
      e.b = (int)num(obj, "b", 0);
      e.time_ms = num(obj, "time_ms", 0);
      got[obj.substr(k0 + 1, k1 - k0 - 1)] = e;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : got) g_tune[kv.first] = kv.second;
  });
}

usfft_status usfft_tune_clear(void) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
  });
}

usfft_status usfft_plan_workspace(usfft_plan_t plan, int64_t n_cand_max, int64_t samples_max, size_t* bytes) {
  return guarded([&] {
    USFFT_REQUIRE(plan && bytes && n_cand_max >= 1 && samples_max >= 1, USFFT_EINVAL, "bad workspace arguments");
    std::lock_guard<std::mutex> lk(plan->mu);
    DevBuf C;
    *bytes = ws_total(ws_items(plan, &C, n_cand_max, samples_max));
  });
}

usfft_status usfft_detect_ws(usfft_plan_t plan, uint64_t seed, int64_t n_cand_max, int64_t samples_max, void* ws_dev,
                             size_t ws_bytes, void* stream, usfft_result_t* out) {
  return guarded([&] {
    USFFT_REQUIRE(plan && out, USFFT_EINVAL, "null plan or output");
    std::lock_guard<std::mutex> lk(plan->mu);
    std::unique_ptr<usfft_result_s> R(new usfft_result_s());
    detect_ws(plan, seed, n_cand_max, samples_max, ws_dev, ws_bytes, (hipStream_t)stream, R.get(), false, nullptr,
              0);
    *out = R.release();
  });
}

usfft_status usfft_coefficients_ws(usfft_plan_t plan, const int32_t* freqs_host, int64_t n, uint64_t seed,
                                   int64_t n_cand_max, int64_t samples_max, void* ws_dev, size_t ws_bytes,
                                   void* stream, usfft_result_t* out) {
  return guarded([&] {
    USFFT_REQUIRE(plan && out && n >= 0 && (n == 0 || freqs_host), USFFT_EINVAL, "bad coefficients arguments");
    USFFT_REQUIRE(n <= n_cand_max, USFFT_ENOMEM, "more frequencies than n_cand_max");
    const int d = plan->prob.d;
    std::vector<std::vector<int32_t>> rows((size_t)n);
    for (int64_t a = 0; a < n; ++a) rows[a].assign(freqs_host + a * d, freqs_host + (a + 1) * d);
    std::sort(rows.begin(), rows.end());
    USFFT_REQUIRE(std::adjacent_find(rows.begin(), rows.end()) == rows.end(), USFFT_EINVAL,
                  "the frequency set has repeated entries");
    std::lock_guard<std::mutex> lk(plan->mu);
    std::unique_ptr<usfft_result_s> R(new usfft_result_s());
    detect_ws(plan, seed, n_cand_max, samples_max, ws_dev, ws_bytes, (hipStream_t)stream, R.get(), true, freqs_host,
              n);
    *out = R.release();
  });
}

usfft_status usfft_result_info(usfft_result_t res, int64_t* n_freq, int32_t* d, int64_t* G, usfft_stats* stats) {
  return guarded([&] {
    USFFT_REQUIRE(res, USFFT_EINVAL, "null result");
    if (n_freq) *n_freq = res->d ? (int64_t)res->I.size() / res->d : 0;
    if (d) *d = res->d;
    if (G) *G = res->G;
    if (stats) *stats = res->stats;
  });
}

usfft_status usfft_result_copy(usfft_result_t res, int32_t* freqs_host, double* coeffs_host) {
  return guarded([&] {
    USFFT_REQUIRE(res, USFFT_EINVAL, "null result");
    if (freqs_host && !res->I.empty()) std::memcpy(freqs_host, res->I.data(), sizeof(int32_t) * res->I.size());
    const int64_t n = res->d ? (int64_t)res->I.size() / res->d : 0;
    if (coeffs_host && n > 0)
      USFFT_HIP(hipMemcpy(coeffs_host, res->C.p, sizeof(double) * 2 * n * res->G, hipMemcpyDeviceToHost));
  });
}

usfft_status usfft_result_trace(usfft_result_t res, int32_t stage, int64_t* n, int32_t* width, int64_t* n_cand,
                                int32_t* set_host) {
  return guarded([&] {
    USFFT_REQUIRE(res && n && width && n_cand, USFFT_EINVAL, "bad trace arguments");
    USFFT_REQUIRE(!res->trace_set.empty(), USFFT_EINVAL, "no detection trace was kept (params.trace = 0)");
    USFFT_REQUIRE(stage >= 0 && stage < (int32_t)res->trace_set.size(), USFFT_EINVAL, "trace stage out of range");
    const std::vector<int32_t>& v = res->trace_set[stage];
    *width = res->trace_width[stage];
    *n = (int64_t)v.size() / std::max(1, *width);
    *n_cand = res->trace_cand[stage];
    if (set_host && !v.empty()) std::memcpy(set_host, v.data(), sizeof(int32_t) * v.size());
  });
}

void usfft_result_destroy(usfft_result_t res) {
  if (res) usfft::result_recycle(res);
  delete res;
}

namespace {
// Points per chunk of an evaluation: the phase matrix (2 |I| rows) stays
// within 256 MB and, with FE solutions (G rows), those within 1 GB.
int64_t eval_chunk(int64_t n, int64_t nI, int64_t G, bool with_fe) {
  int64_t nc = (int64_t)(256ll << 20) / std::max<int64_t>(1, 16 * nI);
  if (with_fe) nc = std::min<int64_t>(nc, (int64_t)(1ll << 30) / std::max<int64_t>(1, 8 * G));
  nc = std::max<int64_t>(64, nc / 64 * 64);
  return std::min<int64_t>(nc, std::max<int64_t>(n, 1));
}

// The result's frequency set on the device (null when empty), uploaded on
// the first evaluation call; the caller holds res->emu.
const int32_t* result_set(usfft_result_s* res) {
  if (res->I.empty()) return nullptr;
  if (!res->Iup) {
    res->Idev.ensure(sizeof(int32_t) * res->I.size());
    USFFT_HIP(hipMemcpy(res->Idev.p, res->I.data(), sizeof(int32_t) * res->I.size(), hipMemcpyHostToDevice));
    res->Iup = true;
  }
  return res->Idev.as<int32_t>();
}

// Fixed scratch of usfft_eval_noalloc, for callers that cannot allocate
// device memory.  Each GPU the library runs on holds its own copy of this
// array for the life of the process.  Host code never uses the array's name
// as an address: the device address is looked up once per device with
// hipGetSymbolAddress and kept in g_noalloc_ptr.
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device.
void* noalloc_scratch() {
  int dev = 0;
  USFFT_HIP(hipGetDevice(&dev));
  USFFT_REQUIRE(dev >= 0 && dev < kMaxDevices, USFFT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    USFFT_REQUIRE(e == hipSuccess && p, USFFT_EHIP,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  return g_noalloc_ptr[dev];
}
}  // namespace

usfft_status usfft_eval(usfft_result_t res, const double* y_dev, int64_t n, double* out_dev, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(res && n >= 0 && (n == 0 || (y_dev && out_dev)), USFFT_EINVAL, "bad eval arguments");
    if (n == 0 || res->G == 0) return;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nI = res->d ? (int64_t)res->I.size() / res->d : 0;
    std::lock_guard<std::mutex> lk(res->emu);
    const int32_t* I = result_set(res);
    DevBuf &T = res->ews[0], &B = res->ews[1];
    const int64_t nc = eval_chunk(n, nI, res->G, false);
    T.ensure(sizeof(double) * (size_t)(res->d * nc));
    B.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, 2 * nI * nc));
    for (int64_t c0 = 0; c0 < n; c0 += nc) {
      const int64_t m = std::min(nc, n - c0);
      launch_node_map(y_dev + c0 * res->d, m, res->d, res->model, res->alpha, res->beta, res->delta,
                      T.as<double>(), nc, st);
      launch_phases(I, nI, res->d, T.as<double>(), nc, m, B.as<double>(), nc, st);
      launch_evgemm_values(res->C.as<double>(), res->G, nI, B.as<double>(), nc, m, out_dev + c0 * res->G, res->G,
                           st);
    }
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_eval_noalloc(usfft_result_t res, const double* y_dev, int64_t n, double* out_dev,
                                void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(res && n >= 0 && (n == 0 || (y_dev && out_dev)), USFFT_EINVAL, "bad eval arguments");
    if (n == 0 || res->G == 0) return;
    hipStream_t st = (hipStream_t)stream;
    const int64_t d = res->d;
    const int64_t nI = d ? (int64_t)res->I.size() / d : 0;
    // scratch layout: the frequency set, then per chunk of nc points the
    // mapped nodes (d x nc) and the phase matrix (2 nI x nc)
    const size_t set_bytes = (sizeof(int32_t) * (size_t)(nI * d) + 255) / 256 * 256;
    const size_t per_point = sizeof(double) * (size_t)(d + 2 * nI);
    USFFT_REQUIRE(set_bytes + 64 * per_point <= kNoAllocScratchBytes, USFFT_EINVAL,
                  "the result's frequency set needs " + std::to_string(set_bytes + 64 * per_point) +
                      " bytes of scratch for one 64-point chunk; usfft_eval_noalloc holds " +
                      std::to_string(kNoAllocScratchBytes));
    const int64_t nc = std::min<int64_t>((int64_t)((kNoAllocScratchBytes - set_bytes) / per_point) / 64 * 64,
                                         ceil_div(n, 64) * 64);
    char* base = static_cast<char*>(noalloc_scratch());
    int32_t* I = reinterpret_cast<int32_t*>(base);
    double* T = reinterpret_cast<double*>(base + set_bytes);
    double* B = T + d * nc;
    if (nI > 0)
      USFFT_HIP(hipMemcpyAsync(I, res->I.data(), sizeof(int32_t) * res->I.size(), hipMemcpyHostToDevice, st));
    for (int64_t c0 = 0; c0 < n; c0 += nc) {
      const int64_t m = std::min(nc, n - c0);
      launch_node_map(y_dev + c0 * d, m, (int)d, res->model, res->alpha, res->beta, res->delta, T, nc, st);
      launch_phases(I, nI, (int)d, T, nc, m, B, nc, st);
      launch_evgemm_values(res->C.as<double>(), res->G, nI, B, nc, m, out_dev + c0 * res->G, res->G, st);
    }
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_statistics(usfft_result_t res, double* mean_dev, double* var_dev, double* gsi_dev,
                              void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(res, USFFT_EINVAL, "bad statistics arguments");
    if (res->G == 0 || (!mean_dev && !var_dev && !gsi_dev)) return;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nI = res->d ? (int64_t)res->I.size() / res->d : 0;
    std::lock_guard<std::mutex> lk(res->emu);
    const int32_t* I = result_set(res);
    DevBuf &D = res->ews[0], &ord = res->ews[1];
    D.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, 2 * nI));
    ord.ensure(sizeof(int32_t) * (size_t)std::max<int64_t>(1, nI));
    launch_stats(I, nI, res->d, res->C.as<double>(), res->G, res->model, res->delta, D.as<double>(),
                 ord.as<int32_t>(), mean_dev, var_dev, gsi_dev, st);
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_errors(usfft_plan_t plan, usfft_result_t res, const double* y_dev, int64_t n, double p,
                          double* errp_dev, double* errinf_dev, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(plan && res && n >= 1 && y_dev && errp_dev && errinf_dev, USFFT_EINVAL, "bad errors arguments");
    USFFT_REQUIRE(p >= 1.0 && std::isfinite(p), USFFT_EINVAL, "p must be finite and >= 1");
    USFFT_REQUIRE(res->d == plan->prob.d && res->G == plan->G, USFFT_EINVAL,
                  "the result does not belong to this plan's problem");
    std::lock_guard<std::mutex> lk(plan->mu);
    std::lock_guard<std::mutex> lr(res->emu);
    hipStream_t st = (hipStream_t)stream;
    const int64_t G = res->G, d = res->d;
    const int64_t nI = d ? (int64_t)res->I.size() / d : 0;
    const int64_t nc = eval_chunk(n, nI, G, true);
    const int32_t* I = result_set(res);
    DevBuf &T = res->ews[0], &B = res->ews[1], &U = res->ews[2], &it = res->ews[3], &ps = res->ews[4],
           &pm = res->ews[5], &cnt = res->ews[6];
    T.ensure(sizeof(double) * (size_t)(d * nc));
    B.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, 2 * nI * nc));
    U.ensure(sizeof(double) * (size_t)(G * nc));
    it.ensure(sizeof(int32_t) * (size_t)nc);
    ps.ensure(sizeof(double) * (size_t)(evgemm_tiles_j(nc) * G));
    pm.ensure(sizeof(double) * (size_t)(evgemm_tiles_j(nc) * G));
    cnt.ensure(2 * sizeof(unsigned long long));
    USFFT_HIP(hipMemsetAsync(cnt.p, 0, 2 * sizeof(unsigned long long), st));
    for (int64_t c0 = 0; c0 < n; c0 += nc) {
      const int64_t m = std::min(nc, n - c0);
      const double* Y = y_dev + c0 * d;
      // finite-element solutions at the parameters themselves (Sec. 4)
      run_sampler(plan, Y, m, U.p, 0, nc, 0, it.as<int32_t>(), st, true);
      hipLaunchKernelGGL(iter_stats_kernel, dim3((unsigned)std::min<int64_t>(256, ceil_div(m, 256))), dim3(256), 0,
                         st, it.as<int32_t>(), m, cnt.as<unsigned long long>());
      USFFT_HIP(hipGetLastError());
      launch_node_map(Y, m, (int)d, res->model, res->alpha, res->beta, res->delta, T.as<double>(), nc, st);
      launch_phases(I, nI, (int)d, T.as<double>(), nc, m, B.as<double>(), nc, st);
      launch_evgemm_errors(res->C.as<double>(), G, nI, B.as<double>(), nc, m, U.as<double>(), nc, p, ps.as<double>(),
                           pm.as<double>(), c0 == 0, errp_dev, errinf_dev, st);
    }
    launch_err_final(errp_dev, G, n, p, st);
    unsigned long long h[2];
    USFFT_HIP(hipMemcpyAsync(h, cnt.p, sizeof(h), hipMemcpyDeviceToHost, st));
    USFFT_HIP(hipStreamSynchronize(st));
    USFFT_REQUIRE(h[0] == 0, USFFT_ENOCONV, std::to_string(h[0]) + " test solves missed pcg_rtol within pcg_maxit");
  });
}

usfft_status usfft_sample(usfft_plan_t plan, const double* y_dev, int64_t n, void* u_dev, int32_t out_fp32,
                          int64_t ld, int64_t col0, int32_t* iters_dev, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(plan && (n == 0 || (y_dev && u_dev)), USFFT_EINVAL, "bad sample arguments");
    USFFT_REQUIRE(n >= 0 && col0 >= 0 && ld >= col0 + n, USFFT_EINVAL, "ld < col0 + n");
    std::lock_guard<std::mutex> lk(plan->mu);
    run_sampler(plan, y_dev, n, u_dev, out_fp32 ? 1 : 0, ld, col0, iters_dev, (hipStream_t)stream);
  });
}

usfft_status usfft_nodes(int32_t d, int32_t line, int32_t t, int32_t nlat, const int32_t* M_host,
                         const int32_t* z_host, const double* tail_host, double* y_dev, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(d >= 1 && d <= kMaxD && M_host && tail_host && y_dev, USFFT_EINVAL, "bad nodes arguments");
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> Ms, zs;
    std::vector<int64_t> off = {0};
    std::vector<double> tail(tail_host, tail_host + d);
    if (line >= 0) {
      USFFT_REQUIRE(line < d && M_host[0] >= 1, USFFT_EINVAL, "bad line");
      Ms = {M_host[0]};
      off.push_back(M_host[0]);
    } else {
      USFFT_REQUIRE(nlat >= 1 && t >= 1 && t <= d && z_host, USFFT_EINVAL, "bad lattice list");
      for (int l = 0; l < nlat; ++l) {
        USFFT_REQUIRE(M_host[l] >= 1, USFFT_EINVAL, "bad lattice size");
        Ms.push_back(M_host[l]);
        off.push_back(off.back() + M_host[l]);
      }
      zs.assign(z_host, z_host + (size_t)nlat * t);
    }
    DevBuf dM, dz, doff, dt;
    h2d(dM, Ms, st);
    h2d(dz, zs.empty() ? std::vector<int32_t>{0} : zs, st);
    h2d(doff, off, st);
    h2d(dt, tail, st);
    launch_nodes(d, line, t, (int)Ms.size(), doff.as<int64_t>(), dM.as<int32_t>(), dz.as<int32_t>(), dt.as<double>(),
                 y_dev, off.back(), st);
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_line_dft(const void* u_dev, int32_t u_fp32, int64_t G, int64_t ld, int64_t col0, int32_t K,
                            const int32_t* bins_host, int32_t nb, int32_t out_kind, void* out_dev, int64_t ldo,
                            void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(u_dev && bins_host && out_dev && G >= 1 && nb >= 1 && ld >= col0 + K, USFFT_EINVAL,
                  "bad line DFT arguments");
    USFFT_REQUIRE(out_kind == USFFT_OUT_COMPLEX || ldo >= nb, USFFT_EINVAL, "ldo < nb");
    hipStream_t st = (hipStream_t)stream;
    DevBuf b;
    h2d(b, std::vector<int32_t>(bins_host, bins_host + nb), st);
    launch_line_dft(u_dev, u_fp32, G, ld, col0, K, b.as<int32_t>(), nb, out_kind, out_dev, ldo, st);
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_lattice_dft(const void* u_dev, int32_t u_fp32, int64_t G, int64_t ld, int64_t col0, int32_t M,
                               const int32_t* bins_dev, const int32_t* pos_dev, int32_t nb, int32_t out_kind,
                               void* out_dev, int64_t ldo, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(u_dev && bins_dev && pos_dev && out_dev && G >= 1 && nb >= 0 && ld >= col0 + M, USFFT_EINVAL,
                  "bad lattice DFT arguments");
    USFFT_REQUIRE(lattice_size_ok(M) && M <= lattice_mmax_for(u_fp32), USFFT_EINVAL,
                  "M is not an admissible lattice size for this precision");
    hipStream_t st = (hipStream_t)stream;
    RaderTables T;
    rader_build(T, M, u_fp32 != 0, st);
    try {
      launch_lattice_dft(T, u_dev, u_fp32, G, ld, col0, bins_dev, pos_dev, 0, nb, out_kind, out_dev, ldo, st);
      USFFT_HIP(hipStreamSynchronize(st));
    } catch (...) {
      rader_free(T);
      throw;
    }
    rader_free(T);
  });
}

usfft_status usfft_lattice_coeffs(const void* u_dev, int32_t u_fp32, int64_t G, int64_t ld, int64_t col0, int32_t M,
                                  int32_t t, const int64_t* z_host, const int32_t* J_dev, int64_t n, double* out_dev,
                                  void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(u_dev && z_host && out_dev && G >= 1 && n >= 0 && (n == 0 || J_dev) && ld >= col0 + M && col0 >= 0,
                  USFFT_EINVAL, "bad lattice coefficient arguments");
    USFFT_REQUIRE(t >= 1 && t <= kMaxD, USFFT_EINVAL, "t must be in [1, 64]");
    USFFT_REQUIRE(lattice_size_ok(M) && M <= lattice_mmax_for(u_fp32), USFFT_EINVAL,
                  "M is not an admissible lattice size for this precision");
    USFFT_REQUIRE(n <= INT32_MAX, USFFT_EINVAL, "too many candidates");
    if (n == 0) return;
    hipStream_t st = (hipStream_t)stream;
    GenVec z{};
    for (int j = 0; j < t; ++j) z.z[j] = ((z_host[j] % M) + M) % M;
    DevBuf bins;
    bins.ensure(sizeof(int32_t) * n);
    hipLaunchKernelGGL(lattice_bin_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, J_dev, n, t, z,
                       (int64_t)M, bins.as<int32_t>());
    USFFT_HIP(hipGetLastError());
    RaderTables T;
    rader_build(T, M, u_fp32 != 0, st);
    try {
      launch_lattice_dft(T, u_dev, u_fp32, G, ld, col0, bins.as<int32_t>(), nullptr, 0, (int)n, USFFT_OUT_COMPLEX,
                         out_dev, G, st);
      USFFT_HIP(hipStreamSynchronize(st));
    } catch (...) {
      rader_free(T);
      throw;
    }
    rader_free(T);
  });
}

usfft_status usfft_select(const double* v_dev, int64_t G, int64_t n, int64_t ld, int32_t s_tilde,
                          const double* theta2_dev, double tie_rel, uint32_t* mask_dev, double* thr_dev,
                          void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(v_dev && theta2_dev && mask_dev && G >= 1 && n >= 0 && ld >= n, USFFT_EINVAL,
                  "bad select arguments");
    hipStream_t st = (hipStream_t)stream;
    launch_select(v_dev, G, n, ld, s_tilde, theta2_dev, tie_rel, mask_dev, thr_dev, st);
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_product(const int32_t* parent_dev, int64_t np, int32_t t, const int32_t* child_dev, int64_t nc,
                           int32_t* out_dev, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(np >= 0 && nc >= 0 && t >= 1, USFFT_EINVAL, "bad product arguments");
    hipStream_t st = (hipStream_t)stream;
    launch_product(parent_dev, np, t, child_dev, nc, out_dev, st);
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_compact(const int32_t* J_dev, const uint32_t* mask_dev, int64_t n, int32_t t, int32_t* out_dev,
                           int64_t* count_host, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(n >= 0 && t >= 1 && count_host, USFFT_EINVAL, "bad compact arguments");
    hipStream_t st = (hipStream_t)stream;
    DevBuf c;
    c.ensure(sizeof(int64_t));
    launch_compact(J_dev, mask_dev, n, t, out_dev, c.as<int64_t>(), st);
    USFFT_HIP(hipMemcpyAsync(count_host, c.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    USFFT_HIP(hipStreamSynchronize(st));
  });
}

usfft_status usfft_family(const int32_t* J_dev, int64_t n, int32_t t, double c, int32_t mmax, int32_t tries,
                          int32_t lmax, uint64_t seed, int32_t kind, int32_t tcode, int32_t cap, int32_t* nlat_host,
                          int32_t* M_host, int32_t* z_host, int32_t* assign_dev, int32_t* bins_dev, void* stream) {
  return guarded([&] {
    USFFT_REQUIRE(n >= 0 && t >= 1 && c > 0 && mmax >= 3 && mmax <= kMaxLattice && tries >= 1 && lmax >= 1 &&
                      nlat_host && M_host && z_host,
                  USFFT_EINVAL, "bad family arguments");
    usfft_plan_s P;
    P.par.lattice_c = c;
    P.par.lattice_mmax = mmax;
    P.par.lattice_tries = tries;
    P.par.lattice_max = lmax;
    Family F;
    hipStream_t st = (hipStream_t)stream;
    plan_family(&P, J_dev, n, t, seed, kind, tcode, F, assign_dev, bins_dev, st);
    USFFT_HIP(hipStreamSynchronize(st));
    USFFT_REQUIRE((int)F.M.size() <= cap, USFFT_EINVAL, "family larger than cap");
    *nlat_host = (int32_t)F.M.size();
    for (size_t l = 0; l < F.M.size(); ++l) M_host[l] = F.M[l];
    std::memcpy(z_host, F.z.data(), sizeof(int32_t) * F.z.size());
  });
}

}  // extern "C"

// ---------------------------------------------------------------- serving
namespace usfft {

// Owning copy of a problem + params (the caller's arrays may go away).
struct JobSpec {
  usfft_problem prob{};
  usfft_params par{};
  std::vector<int32_t> k_lo, k_hi, mode1, mode2, poly_k, mesh_tri;
  std::vector<double> amp, poly_c, mesh_xy, nodes_xy;
  std::vector<uint8_t> mesh_boundary;
  void copy(const usfft_problem* pb, const usfft_params* pa) {
    validate(pb, pa);
    prob = *pb;
    par = *pa;
    const int d = pb->d;
    k_lo.assign(pb->k_lo, pb->k_lo + d);
    k_hi.assign(pb->k_hi, pb->k_hi + d);
    prob.k_lo = k_lo.data();
    prob.k_hi = k_hi.data();
    if (pb->sampler != USFFT_SAMPLER_TRIG_POLY) {
      amp.assign(pb->amp, pb->amp + d);
      mode1.assign(pb->mode1, pb->mode1 + d);
      mode2.assign(pb->mode2, pb->mode2 + d);
      prob.amp = amp.data();
      prob.mode1 = mode1.data();
      prob.mode2 = mode2.data();
      if (pb->sampler == USFFT_SAMPLER_PDE_MESH) {
        mesh_xy.assign(pb->mesh_xy, pb->mesh_xy + 2 * (size_t)pb->mesh_nv);
        mesh_tri.assign(pb->mesh_tri, pb->mesh_tri + 3 * (size_t)pb->mesh_nt);
        mesh_boundary.assign(pb->mesh_boundary, pb->mesh_boundary + pb->mesh_nv);
        prob.mesh_xy = mesh_xy.data();
        prob.mesh_tri = mesh_tri.data();
        prob.mesh_boundary = mesh_boundary.data();
      }
      if (pb->n_nodes > 0 && pb->nodes_xy) {
        nodes_xy.assign(pb->nodes_xy, pb->nodes_xy + 2 * (size_t)pb->n_nodes);
        prob.nodes_xy = nodes_xy.data();
      }
    } else {
      poly_k.assign(pb->poly_k, pb->poly_k + (size_t)pb->n_poly * d);
      poly_c.assign(pb->poly_c, pb->poly_c + (size_t)pb->n_poly * pb->G_poly * 2);
      prob.poly_k = poly_k.data();
      prob.poly_c = poly_c.data();
    }
  }
};

// Admission estimate of a job's device footprint (bytes): the largest stage
// holds the sample matrix (G x samples) and the candidate magnitudes
// (G x |J|).  |J| <= |I^(1..t-1)| |I^(t)| is bounded by 3 s_local (detected
// sets grow to a few times s, Remark 4.1) times min(K_t, 17) (1-D projections
// stay small, Sec. 4.2); a lattice family takes about 12 |J| samples.
static uint64_t estimate_footprint(const usfft_problem* pb, const usfft_params* pa) {
  uint64_t G = pb->sampler == USFFT_SAMPLER_PDE ? (uint64_t)(pb->mesh_n - 1) * (pb->mesh_n - 1)
                                                : (uint64_t)pb->G_poly;
  if (pb->sampler == USFFT_SAMPLER_PDE_MESH) {
    G = 0;
    for (int v = 0; v < pb->mesh_nv; ++v) G += pb->mesh_boundary[v] ? 0 : 1;
  }
  const uint64_t ub = pa->precision == USFFT_FP32_REFINE ? 4 : 8;
  int kmax = 1;
  for (int j = 0; j < pb->d; ++j) kmax = std::max(kmax, pb->k_hi[j] - pb->k_lo[j] + 1);
  const uint64_t J = 3ull * (uint64_t)pa->s_local * (uint64_t)std::min(kmax, 17);
  const uint64_t samples = std::min<uint64_t>(12 * J, 64ull * (uint64_t)pa->lattice_mmax) + (uint64_t)kmax;
  const uint64_t lines = G * (uint64_t)pb->d * (uint64_t)pa->r * (uint64_t)kmax * 8;  // step-1 spectra
  // workspace of the streaming solvers (meshes above 65 points per side;
  // 256 workgroups stand in for one per CU of the DST variant)
  uint64_t solver = 0;
  if (pb->sampler == USFFT_SAMPLER_PDE && pb->mesh_n - 1 > 64)
    solver = 8ull * (uint64_t)(pa->precond == USFFT_PRECOND_DST && dst_stream_ok(pb->mesh_n)
                                   ? dst_stream_workspace_doubles(pb->mesh_n, 256)
                                   : pa->precond == USFFT_PRECOND_DST && tl_stream_ok(pb->mesh_n)
                                         ? tl_stream_workspace_doubles(256)
                                         : stream_workspace_doubles(pb->mesh_n, kStreamBlocks));
  return G * samples * ub + G * J * 8 + lines + samples * (uint64_t)pb->d * 8 + solver + (64ull << 20);
}

// Plans are pooled by everything that fixes their device tables: the
// sampler and its coefficient family, mesh and node set, and the parameters
// read at plan creation.  The box, the sparsity parameters, the threshold
// and the lattice-planner and solver knobs that detect() reads per call are
// rebound for every job.
static std::string plan_key(const usfft_problem* pb, const usfft_params* pa) {
  std::string k;
  auto put = [&k](const void* p, size_t n) { k.append(static_cast<const char*>(p), n); };
  auto put_i = [&](int64_t v) { put(&v, sizeof v); };
  auto put_d = [&](double v) { put(&v, sizeof v); };
  put_i(pb->sampler);
  put_i(pb->d);
  put_i(pb->n_nodes);
  if (pb->n_nodes > 0) put(pb->nodes_xy, sizeof(double) * 2 * (size_t)pb->n_nodes);
  if (pb->sampler == USFFT_SAMPLER_TRIG_POLY) {
    put_i(pb->G_poly);
    put_i(pb->n_poly);
    put(pb->poly_k, sizeof(int32_t) * (size_t)pb->n_poly * pb->d);
    put(pb->poly_c, sizeof(double) * 2 * (size_t)pb->n_poly * pb->G_poly);
  } else {
    put_i(pb->mesh_n);
    put_d(pb->a0);
    put(pb->amp, sizeof(double) * pb->d);
    put(pb->mode1, sizeof(int32_t) * pb->d);
    put(pb->mode2, sizeof(int32_t) * pb->d);
    put_i(pb->model);
    put_d(pb->alpha);
    put_d(pb->beta);
    put_d(pb->delta);
    put_i(pb->basis1);
    put_i(pb->basis2);
    if (pb->sampler == USFFT_SAMPLER_PDE_MESH) {
      put_i(pb->mesh_nv);
      put_i(pb->mesh_nt);
      put(pb->mesh_xy, sizeof(double) * 2 * (size_t)pb->mesh_nv);
      put(pb->mesh_tri, sizeof(int32_t) * 3 * (size_t)pb->mesh_nt);
      put(pb->mesh_boundary, (size_t)pb->mesh_nv);
    }
  }
  put_i(pa->precision);
  put_i(pa->lattice_mmax);
  put_i(pa->solver_config);
  put_i(pa->precond);
  put_d(pa->pcg_rtol);
  put_i(pa->pcg_maxit);
  put_d(pa->inner_rtol);
  put_i(pa->refine_every);
  return k;
}

// A pooled plan takes a new job's box and per-call parameters.
static void plan_rebind(usfft_plan_s* P, const usfft_problem* pb, const usfft_params* pa) {
  P->par = *pa;
  P->k_lo.assign(pb->k_lo, pb->k_lo + pb->d);
  P->k_hi.assign(pb->k_hi, pb->k_hi + pb->d);
  P->prob.k_lo = P->k_lo.data();
  P->prob.k_hi = P->k_hi.data();
}

// Device bytes a plan holds (static tables, lattice tables, workspaces).
static uint64_t plan_bytes(const usfft_plan_s* P) {
  uint64_t b = 0;
  for (const DevBuf* x : {&P->d_amp, &P->d_tab, &P->d_polyk, &P->d_polyc, &P->d_stream, &P->d_wscr, &P->d_sfrag,
                          &P->d_lam, &P->m_rowptr, &P->m_col, &P->m_diag, &P->m_cptr, &P->m_ctri, &P->m_cw, &P->m_load,
                          &P->m_psi, &P->d_iidx, &P->d_iw, &P->Umesh, &P->d_rader, &P->famlog, &P->famstate, &P->Y,
                          &P->U, &P->V, &P->iters, &P->cnt, &P->theta2, &P->scratch, &P->J, &P->Jnext, &P->Iprev,
                          &P->mask, &P->gmask, &P->cands, &P->assign, &P->famz, &P->fambins, &P->famcounts,
                          &P->famcov, &P->famscores, &P->lists, &P->latM, &P->latoff, &P->tail,
                          &P->latitems})
    b += x->bytes;
  for (const DevBuf& x : P->I1) b += x.bytes;
  return b;
}

struct Job {
  uint64_t id = 0;
  JobSpec spec;
  uint64_t seed = 0;
  uint64_t footprint = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  usfft_status st = USFFT_OK;
  std::string err;
  usfft_result_s* res = nullptr;
  std::chrono::steady_clock::time_point t_submit, t_start, t_done;
  ~Job() { delete res; }
};

}  // namespace usfft

struct usfft_server_s {
  usfft_server_cfg cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<usfft::Job*> queue;
  std::map<uint64_t, std::unique_ptr<usfft::Job>> jobs;
  uint64_t in_use = 0, next_id = 1;
  int active = 0;
  bool stop = false;
  std::vector<std::thread> workers;
  // idle plans by key, oldest first; their device bytes count against the
  // budget and are released (oldest first) when an admission needs them
  struct Pooled {
    std::string key;
    std::unique_ptr<usfft_plan_s> plan;
    uint64_t bytes;
  };
  std::deque<Pooled> pool;
  uint64_t pooled_bytes = 0;
  int64_t plans_created = 0, plans_reused = 0;
  ~usfft_server_s() {
    pool.clear();
  }
};

namespace usfft {

// Frees pooled plans, oldest first, until `need` more bytes fit the budget
// (called with the server lock held).
static void pool_make_room(usfft_server_s* S, uint64_t need) {
  while (!S->pool.empty() && S->cfg.hbm_budget > 0 && S->in_use + S->pooled_bytes + need > S->cfg.hbm_budget) {
    S->pooled_bytes -= S->pool.front().bytes;
    S->pool.pop_front();
  }
}

static void server_worker(usfft_server_s* S) {
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_work.wait(lk, [&] {
      if (S->stop && S->queue.empty()) return true;
      if (S->queue.empty() || S->active >= S->cfg.max_active) return false;
      const uint64_t fp = S->queue.front()->footprint;
      pool_make_room(S, fp);
      return S->cfg.hbm_budget == 0 || S->active == 0 || S->in_use + S->pooled_bytes + fp <= S->cfg.hbm_budget;
    });
    if (S->queue.empty()) break;
    Job* J = S->queue.front();
    S->queue.pop_front();
    S->active++;
    S->in_use += J->footprint;
    J->state = 1;
    J->t_start = std::chrono::steady_clock::now();
    // an idle plan of the same key, if any (the most recently returned)
    const std::string key = plan_key(&J->spec.prob, &J->spec.par);
    std::unique_ptr<usfft_plan_s> P;
    for (auto it = S->pool.rbegin(); it != S->pool.rend(); ++it)
      if (it->key == key) {
        P = std::move(it->plan);
        S->pooled_bytes -= it->bytes;
        S->pool.erase(std::next(it).base());
        break;
      }
    const bool reused = P != nullptr;
    if (reused) S->plans_reused++; else S->plans_created++;
    lk.unlock();
    usfft_status status = USFFT_OK;
    std::string err;
    std::unique_ptr<usfft_result_s> R(new usfft_result_s());
    try {
      USFFT_REQUIRE(st != nullptr, USFFT_EHIP, "worker stream creation failed");
      if (!P) P.reset(plan_create(&J->spec.prob, &J->spec.par));
      plan_rebind(P.get(), &J->spec.prob, &J->spec.par);
      std::lock_guard<std::mutex> pl(P->mu);
      detect(P.get(), J->seed, st, R.get());
      R->stats.plan_reused = reused ? 1 : 0;
    } catch (const Error& e) {
      status = e.st;
      err = e.msg;
      P.reset();  // a failed job's plan is not pooled
    } catch (const std::exception& e) {
      status = USFFT_EINVAL;
      err = e.what();
      P.reset();
    }
    lk.lock();
    if (P) {
      // keep at most 2 max_active idle plans
      const uint64_t b = plan_bytes(P.get());
      S->pool.push_back({key, std::move(P), b});
      S->pooled_bytes += b;
      while ((int)S->pool.size() > 2 * S->cfg.max_active) {
        S->pooled_bytes -= S->pool.front().bytes;
        S->pool.pop_front();
      }
    }
    J->st = status;
    J->err = err;
    J->res = status == USFFT_OK ? R.release() : nullptr;
    J->t_done = std::chrono::steady_clock::now();
    J->state = 2;
    S->active--;
    S->in_use -= J->footprint;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  lk.unlock();
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace usfft

extern "C" {

usfft_status usfft_server_create(const usfft_server_cfg* cfg, usfft_server_t* out) {
  return guarded([&] {
    USFFT_REQUIRE(cfg && out && cfg->max_active >= 1 && cfg->max_active <= 64, USFFT_EINVAL,
                  "max_active must be in [1, 64]");
    std::unique_ptr<usfft_server_s> S(new usfft_server_s());
    S->cfg = *cfg;
    for (int i = 0; i < cfg->max_active; ++i) S->workers.emplace_back(server_worker, S.get());
    *out = S.release();
  });
}

usfft_status usfft_server_submit(usfft_server_t srv, const usfft_problem* prob, const usfft_params* par,
                                 uint64_t seed, uint64_t* job) {
  return guarded([&] {
    USFFT_REQUIRE(srv && job, USFFT_EINVAL, "null server or job");
    std::unique_ptr<Job> J(new Job());
    J->spec.copy(prob, par);
    J->seed = seed;
    J->footprint = estimate_footprint(&J->spec.prob, &J->spec.par);
    USFFT_REQUIRE(srv->cfg.hbm_budget == 0 || J->footprint <= srv->cfg.hbm_budget, USFFT_EINVAL,
                  "job footprint " + std::to_string(J->footprint) + " B exceeds the server's HBM budget");
    J->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    J->id = srv->next_id++;
    *job = J->id;
    srv->queue.push_back(J.get());
    srv->jobs[J->id] = std::move(J);
    srv->cv_work.notify_all();
  });
}

usfft_status usfft_server_poll(usfft_server_t srv, uint64_t job, int32_t wait, usfft_result_t* out,
                               int32_t* job_status, double* latency_s, double* queue_s) {
  return guarded([&] {
    USFFT_REQUIRE(srv && out, USFFT_EINVAL, "null server or output");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(job);
    USFFT_REQUIRE(it != srv->jobs.end(), USFFT_EINVAL, "unknown or already taken job id");
    Job* J = it->second.get();
    if (wait) srv->cv_done.wait(lk, [&] { return J->state == 2; });
    if (J->state != 2) {
      *out = nullptr;
      if (job_status) *job_status = 1;
      return;
    }
    *out = J->res;
    J->res = nullptr;
    if (job_status) *job_status = J->st;
    if (latency_s) *latency_s = std::chrono::duration<double>(J->t_done - J->t_submit).count();
    if (queue_s) *queue_s = std::chrono::duration<double>(J->t_start - J->t_submit).count();
    if (J->st != USFFT_OK) set_error(J->err);
    srv->jobs.erase(it);
  });
}

void usfft_server_destroy(usfft_server_t srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  for (auto& t : srv->workers) t.join();
  delete srv;
}

}  // extern "C"
