// Device hierarchy, V-cycle, PCG and the C-ABI of the LS-AMG-DD library.
//
// Solve phase (all on the GPU): preconditioned CG in FP64 (sec. 4.1) whose
// preconditioner is one V-cycle per iteration (sec. 3.1.1): RAS pre-smoothing
// (eq:ras), residual b - G^T(G x), restriction with P^T (eq:mg-p), the next
// level's V-cycle or the dense coarsest inverse, prolongation, residual and
// RAS-T post-smoothing (eq:ras-t).  The V-cycle runs in FP64 or, in mixed
// mode, in FP32 under the FP64 CG.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cmath>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "launch_checks.hpp"
#include "kernels.hpp"
#include "kernels_batched.hpp"

using namespace lsamg;

namespace {

thread_local std::string g_last_error;

struct DevError {
  int code;
  std::string msg;
};

#define HIP_OK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw DevError{e_ == hipErrorOutOfMemory ? LSAMG_ENOMEM : LSAMG_EHIP,           \
                     std::string(#expr) + ": " + hipGetErrorString(e_)};              \
  } while (0)

#define LAUNCH_OK() HIP_OK(hipGetLastError())

constexpr int kAtaTile = 16;       // unknowns per tile of k_bata_tile

inline unsigned nblocks(int64_t work) {
  return (unsigned)std::max<int64_t>(1, (work + dev::kBlock - 1) / dev::kBlock);
}

template <typename T>
struct DPrec {            // arrays that exist in both V-cycle precisions
  T* g_val = nullptr;     // G_l values (CSR)
  T* gt_val = nullptr;    // G_l^T values (CSR by unknown)
  T* Zc = nullptr;        // Z_i column-major (RAS)
  T* Zr = nullptr;        // Z_i row-major (RAS-T)
  T* Zh = nullptr;        // Zhat_i row-major (restriction P^T)
  T* ZhT = nullptr;       // Zhat_i column-major (prolongation P)
  T* Ainv = nullptr;      // coarsest inverse, or the dense tail operator
  T* As = nullptr;        // additive cycle: A_i^{-1} per aggregate, padded rows
  T* Spk = nullptr;       // the same operator as packed lower 64x64 tiles (k_sym_gemv)
  T* spart = nullptr;     // k_sym_gemv slots, nT * nT * 64
  T* x = nullptr;         // V-cycle output at this level
  T* b = nullptr;         // V-cycle input at this level
  T* r = nullptr;         // residual
  T* y = nullptr;         // G x (length = rows of G_l)
  T* tb = nullptr;        // RAS-T staging, sum |Omega_i|
  T* stg = nullptr;       // staged G^T G x of the row-group pass (coarse levels)
  T* trv = nullptr;       // tiled one-pass G^T G: row entry values of each tile
  T* tdw = nullptr;       // tiled one-pass G^T G: G^T entry values per unknown
  T* tev = nullptr;       // tiled one-pass G^T G, expanded form: stencil entry values
};

// Launch plan of one batched-GEMV operator on one level.
struct GemvPlan {
  dev::GemvOp op{};
  int64_t nagg = 0;
  int lmax = 0;        // largest input length
  int emax = 0;        // finest level: most G^T entries of one aggregate's inputs (IN_RESG)
  int G = 0;           // narrow form lane-group width (0: wide form)
  int NW = 4;          // wide form: wavefronts per workgroup (default from the task count)
  mutable int nw_t[2] = {0, 0};   // wide form, autotuned per precision (double, float); 0: NW
  mutable int form_t = 0;         // FP32 wide form: 0 one output per lane, 1 four (k_gemv_wide4)
  // residual consumers of the finest level (narrow forms), per precision:
  // 0 untimed, 1 r = b - G^T y in its own pass, 2 formed while staging inputs
  mutable int rsep_t[2] = {0, 0};
  mutable int narrow_t[2] = {1, 1};  // G > 0: the form timed fastest: 0 wide, 1 narrow
                                     // (a wavefront per aggregate), 2 an aggregate per
                                     // lane group, 3 16-byte loads (k_gemv_narrow4)
  int64_t ntask4 = 0;             // tasks (aggregate, 256-wide output slice) of k_gemv_wide4
  int32_t* task4_a = nullptr;
  int32_t* task4_j0 = nullptr;
  int64_t ntask = 0;   // wide form: tasks (aggregate, 64-wide output slice)
  // algorithmic size of one application: matrix entries, distinct input
  // entries, gathered index entries, outputs
  int64_t mat = 0, in_u = 0, idx = 0, out = 0;
  int32_t* task_a = nullptr;
  int32_t* task_j0 = nullptr;
  // per-aggregate output and loop lengths, kept on the host for the task
  // lists of the matrix-core batched form (k_bmm)
  std::vector<int32_t> hlj, hll;
  // tile shape of k_bmm chosen by the autotuner, and its task list
  struct Mm {
    int rt = 0;              // row tiles of 16 per task (0: not tuned, use k_bgemm)
    int u = 2;               // loop steps whose loads are issued together (2 or 8)
    int split = 1;           // loop split of a single-aggregate operator
    bool lds = false;        // 64 columns: the LDS-staged form (k_bmm_lds, 64-row tasks)
    int64_t ntask = 0;
    unsigned grid = 0;       // workgroups of the persistent launch
    dev::MmTasks tk{};
    float* part = nullptr;   // partial sums of a split loop (split > 1)
    int64_t part_cap = 0;    // floats that part holds
  } mm;
  Mm mmd;                    // FP64 on the matrix cores (k_bmmd; rt 0: k_bgemm)
};

struct DLevel {
  GemvPlan ras, rast, rst, pro;
  GemvPlan as;            // additive cycle: A_i^{-1} b(Omega_i) into the staging
  GemvPlan dense;         // coarsest level: A_L^{-1} as one block (batched path)
  int64_t n = 0, nagg = 0, nrows = 0, nnz = 0, ntb = 0;
  bool coarsest = false;
  bool tail = false;      // V-cycle from here down applied as the dense matrix Ainv
  bool fuse_ata = false;  // one-pass FP64 G^T G of the multi-right-hand-side CG (k_bcg_apq1) in use
  bool fuse_ok = false;   // rows of G short enough for it
  int nT = 0;             // 64-row tiles per side of the packed dense operator
  int ata_me = 8;         // k_bcg_apq1: most rows of G per unknown (6, 8 or 16)
  int ata_mf = 4;         // k_bcg_apq1: most entries per row of G (3 or 4)
  dev::AtaTiles at{};     // tiles of the one-pass G^T G on 64 columns (k_bata_tile)
  int at_rmax = 0;        // largest row list of a tile
  bool at_ok = false;     // tiles built
  bool at_on = false;     // ... and in use (LSAMG_OPT_ATA_TILES)
  int at_form = 0;        // 0: per precision (FP32 with the row phase, FP64 expanded
                          // stencils, the faster of each on the benchmark); 2: row phase;
                          // 3: expanded stencils
  dev::AtaTiles at1{};    // tiles of the single-vector CG's k_cg_tile (FP64)
  int at1_rmax = 0;
  double *trv1 = nullptr, *tdw1 = nullptr;
  bool at1_ok = false, at1_on = false;
  int dmm_split = 0;      // dense level, 64 columns: k_dense_mm64 loop ranges (0: bgemm)
  int dmm_kchunk = 0;     // rows per loop range of k_dense_mm64
  int dmm_kc = 64;        // its chunk length (32 or 64)
  float* dmm_M = nullptr; // its padded row-major copy of the FP32 operator (batched buffers)
  int64_t dmm_ld = 0;     // row stride of dmm_M
  double* dmmd_M = nullptr;    // the padded row-major copy of the FP64 operator (batched buffers)
  double* dmmd_part = nullptr; // its partial sums of split loops (batched buffers)
  int64_t dmmd_part_cap = 0;   // doubles that dmmd_part holds
  int dmmd_split = 0;     // dense level, 64 columns, FP64: k_dense_mm64d loop ranges (0: bgemm)
  int dmmd_kchunk = 0, dmmd_kc = 0;
  int lanes_g = 1, lanes_gt = 1;
  int max_nO = 0, max_nw = 0, max_k = 0;
  int64_t* g_ptr = nullptr;
  int32_t* g_col = nullptr;
  int64_t* gt_ptr = nullptr;
  int32_t* gt_col = nullptr;
  int64_t *astart = nullptr, *optr = nullptr,
          *cstart = nullptr, *cptr = nullptr, *cpos = nullptr;
  int32_t* oidx = nullptr;
  int32_t* kk = nullptr;
  // coarse levels: A = G^T G applied by row-group tasks (k_grp_ata) whose
  // staged output the residual's consumer gathers through rc_ptr / rc_pos
  bool grp = false;
  int grp_lw = 0, grp_kc = 0, grp_nw = 0, grp_rw = 0;   // grp_nw > 0: workgroup per task
  int64_t grp_ntask = 0, grp_nstg = 0;
  dev::GrpTasks gtask{};
  int32_t* grp_supp = nullptr;
  int64_t* rc_ptr = nullptr;
  int32_t* rc_pos = nullptr;
  // the same pass on 64 columns (k_bgrp_ata64): one task per group of at
  // most 32 rows, staged rows of 64 values; tuned against the CSR passes
  dev::GrpTasks bgtask{};
  int64_t bg_ntask = 0, bg_nstg = 0;
  int bg_wmax = 0;        // most support columns of a task
  int64_t* bg_cptr = nullptr;
  int64_t* bg_cpos = nullptr;
  bool bg_ok = false;     // tasks built
  bool bg_on = false;     // chosen by the autotuner (FP32, 64 columns)
  DPrec<double> d;
  DPrec<float> f;
};

template <typename T>
DPrec<T>& prec(DLevel& L);
template <>
DPrec<double>& prec<double>(DLevel& L) { return L.d; }
template <>
DPrec<float>& prec<float>(DLevel& L) { return L.f; }

int lanes_for(double avg) {
  int l = 1;
  while (l < 64 && l < avg) l <<= 1;
  return l;
}

// Kernel timing with HIP events (lsamg_profile).
struct Profiler {
  bool on = false;
  bool by_level = false;  // append " @L<level>" to V-cycle kernel names
  std::string only;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    std::string name;
    double bytes;
    hipEvent_t a, b;
    double flops;
  };
  std::vector<Rec> recs;
  // only: a kernel name, or with by_level a name with its " @L<level>"
  bool want(const std::string& nm, const std::string& full) const {
    return on && (only.empty() || nm == only || full == only);
  }
};

thread_local Profiler* g_prof = nullptr;
thread_local int g_level = -1;   // hierarchy level whose kernels are being launched

struct LevelTag {   // sets g_level for the kernels of one V-cycle level
  int old;
  explicit LevelTag(int l) : old(g_level) { g_level = l; }
  ~LevelTag() { g_level = old; }
};

inline Profiler* prof_active() { return (g_prof && g_prof->on) ? g_prof : nullptr; }

struct ProfScope {
  Profiler* p = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope() = default;
  ProfScope(Profiler* pp, const std::string& name, double bytes, hipStream_t, double flops = 0.0) {
    if (!pp) return;
    const std::string full =
        pp->by_level && g_level >= 0 ? name + " @L" + std::to_string(g_level) : name;
    if (!pp->want(name, full) || pp->used + 2 > pp->pool.size()) return;
    p = pp;
    a = pp->pool[pp->used++];
    b = pp->pool[pp->used++];
    pp->recs.push_back(Profiler::Rec{full, bytes, a, b, flops});
  }
};

// Launch kern on stream s; when the launch is being timed, the dispatch packet
// itself stamps the start/stop events (hipExtLaunchKernel), so the recorded
// interval is the kernel's own execution.
// While a GraphRec is active on the calling thread, launches are appended to
// its graph as kernel nodes (each depending on the previous one) instead of
// being enqueued.
struct GraphRec {
  hipGraph_t g = nullptr;
  hipGraphNode_t last = nullptr;
};
thread_local GraphRec* g_rec = nullptr;

template <typename... KArgs, typename... Args>
void klaunch(dim3 grid, dim3 block, size_t lds, hipStream_t s, const ProfScope& ps,
             void (*kern)(KArgs...), Args&&... args) {
  std::tuple<KArgs...> tup(std::forward<Args>(args)...);
  void* argv[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
  std::apply([&](auto&... e) {
    int i = 0;
    ((argv[i++] = (void*)&e), ...);
  }, tup);
  if (g_rec) {
    hipKernelNodeParams kp{};
    kp.func = (void*)kern;
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = (unsigned)lds;
    kp.kernelParams = argv;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, g_rec->g, g_rec->last ? &g_rec->last : nullptr,
                                               g_rec->last ? 1 : 0, &kp);
    if (e != hipSuccess)
      throw DevError{LSAMG_EHIP, std::string("graph kernel node: ") + hipGetErrorString(e)};
    g_rec->last = node;
    return;
  }
  hipError_t e = ps.p ? hipExtLaunchKernel((const void*)kern, grid, block, argv, lds, s, ps.a,
                                           ps.b, 0)
                      : hipLaunchKernel((const void*)kern, grid, block, argv, lds, s);
  if (e != hipSuccess)
    throw DevError{LSAMG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e)};
}

const ProfScope kNoProf{};

// KLAUNCH inside a PROF scope times the launch; KLAUNCH0 never does
#define KLAUNCH(G, B, LDS, S, ...) klaunch(G, B, LDS, S, ps_, __VA_ARGS__)
#define KLAUNCH0(G, B, LDS, S, ...) klaunch(G, B, LDS, S, kNoProf, __VA_ARGS__)

// PROF(name-expression, bytes-expression, stream): the expressions are only
// evaluated while profiling is on.
#define PROF(NAME, BYTES, S)          \
  Profiler* pp_ = prof_active();      \
  ProfScope ps_(pp_, pp_ ? std::string(NAME) : std::string(), pp_ ? (double)(BYTES) : 0.0, S)

// the same with the launch's algorithmic floating-point operations
#define PROF_F(NAME, BYTES, FLOPS, S) \
  Profiler* pp_ = prof_active();      \
  ProfScope ps_(pp_, pp_ ? std::string(NAME) : std::string(), pp_ ? (double)(BYTES) : 0.0, S, \
                pp_ ? (double)(FLOPS) : 0.0)

template <typename T>
const char* tname();
template <>
const char* tname<double>() { return "double"; }
template <>
const char* tname<float>() { return "float"; }

inline std::string kname(const char* base, const std::string& args) {
  return std::string(base) + "<" + args + ">";
}

}  // namespace

struct lsamg_handle {
  Profiler prof;
  Hierarchy H;
  int device = -1;
  int precision = LSAMG_FP64;
  int batch_mode = 1;               // 1: nrhs > 1 solved as batches of <= 64
  bool use_mfma = true;             // FP32 batched V-cycle on the matrix cores (k_bmm)
  int mm_fixed = 0;                 // k_bmm tile shape 100*rt + 10*u + split, 0: autotune
  int dense_split = 0;              // k_dense_mm64 loop ranges: 0 autotune, 1..16 fixed, 17 never
  int bgroup = 0;                   // coarse residual on 64 columns: 0 autotune, 1 row groups, 2 CSR
  bool gv_tuned[2] = {false, false}; // single-vector wide GEMV shapes tuned (double, float)
  // V-cycles replayed from HIP graphs, one per (precision, batch width)
  bool use_graphs = true;
  int krylov = LSAMG_KRYLOV_CG;      // outer iteration: CG or flexible CG
  std::unordered_map<int, hipGraphExec_t> graphs;
  void drop_graphs(bool batched_only) {
    for (auto it = graphs.begin(); it != graphs.end();) {
      if (!batched_only || (it->first & 127) > 1) {
        (void)hipGraphExecDestroy(it->second);
        it = graphs.erase(it);
      } else {
        ++it;
      }
    }
  }
  std::vector<DLevel> L;
  std::vector<void*> allocs;
  size_t bytes = 0;
  int64_t* perm = nullptr;          // internal -> user numbering (finest level)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr,
         *bi = nullptr, *part = nullptr, *sc = nullptr;
  // per-workgroup partial sums of the CG dot products (red_blocks(n) each)
  double *p_pq = nullptr, *p_rr = nullptr, *p_rz[2] = {nullptr, nullptr}, *p_tmp = nullptr;
  // flexible CG: partials of -(z . q) and a copy of the last p . q partials
  double *p_zq = nullptr, *p_pqo = nullptr;
  int red_np = 1;
  // k_cg_tile: the direction update p = z + beta p is applied by the next
  // A-apply, into p2 (then swapped with p); 0 none pending, 1 p = z, 2 p = z + beta p
  double* p2 = nullptr;
  int dir_pending = 0;
  const double *dir_num = nullptr, *dir_den = nullptr;   // partials of beta's terms
  double* sc_host = nullptr;         // pinned
  int nparts = 1024;
  hipEvent_t ev_rr[2] = {nullptr, nullptr};
  // multi-right-hand-side buffers (interleaved n x NB, allocated for NB = 64
  // on the first batched solve; a narrower batch uses a prefix)
  struct BLev {
    double *x = nullptr, *b = nullptr, *r = nullptr, *y = nullptr, *tb = nullptr;
    float *fx = nullptr, *fb = nullptr, *fr = nullptr, *fy = nullptr, *ftb = nullptr;
    float* fstg = nullptr;          // k_bgrp_ata64 staging, bg_nstg x 64
  };
  bool batched_ready = false;
  std::vector<BLev> BL;
  double *BX = nullptr, *BR = nullptr, *BZ = nullptr, *BP = nullptr, *BQ = nullptr,
         *BBi = nullptr, *Bpq = nullptr, *Brr = nullptr, *Brz[2] = {nullptr, nullptr},
         *Btmp = nullptr, *Bzq = nullptr;
  // per-column scalars summed from those partials (k_bsum)
  double *Bpq_s = nullptr, *Brr_s = nullptr, *Brz_s[2] = {nullptr, nullptr}, *Btmp_s = nullptr,
         *Bzq_s = nullptr;
  // block CG (64 columns): Gram partials per workgroup, the summed 64 x 64
  // matrices (G = P^T Q, F = P^T R or E = Q^T Z) and the step matrices C, D
  double *Bg_part = nullptr, *Bg_G = nullptr, *Bg_F = nullptr, *Bg_C = nullptr;
  double* Bg_host = nullptr;         // pinned: G, F and C (3 x 4096)
  int* Bactive = nullptr;            // 64 active, 64 restart, 64 new-direction flags
  int* Bactive_host = nullptr;       // pinned, the same three arrays
  double* Bparts_host = nullptr;     // pinned, 3 slots of kBNP * 64
  // export buffers
  std::vector<int32_t> ex_agg, ex_k, ex_M;
  std::vector<int64_t> ex_optr, ex_oidx, ex_muptr;
  std::vector<double> ex_mu;

  bool dry = false;                  // count bytes only (admission planning)
  bool batch_alloc = false;          // allocations belong to the batched buffers
  std::vector<void*> ballocs;        // batched buffers (freed when the width grows)
  size_t bbytes = 0;
  int bwidth = 0;                    // batch width the buffers were sized for

  template <typename T>
  T* alloc(size_t count) {
    const size_t b = std::max<size_t>(count, 1) * sizeof(T);
    bytes += b;
    if (dry) return nullptr;
    void* ptr = nullptr;
    HIP_OK(hipMalloc(&ptr, b));
    if (batch_alloc) {
      ballocs.push_back(ptr);
      bbytes += b;
    } else {
      allocs.push_back(ptr);
    }
    return (T*)ptr;
  }
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* ptr = alloc<T>(v.size());
    if (!dry && !v.empty())
      HIP_OK(hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return ptr;
  }
  bool mm_tuned = false;             // k_bmm tile shapes chosen for the batched buffers
  bool mm_tuned64 = false;           // and the 64-column forms (dense GEMM split, coarse residual)
  bool dmmd_tuned = false;           // the FP64 matrix-core forms chosen (fp64_tune)
  float* mm_part = nullptr;          // partial sums of split loops, sized for the buffers' width
  int64_t mm_part_cap = 0;
  void free_batched() {
    for (auto& D : L) {
      for (GemvPlan* P : {&D.ras, &D.rast, &D.rst, &D.pro, &D.dense}) P->mm = P->mmd = GemvPlan::Mm{};
      D.dmm_split = D.dmmd_split = 0;
      D.dmm_M = nullptr;                // freed with the batched buffers below
      D.dmmd_M = nullptr;
      D.dmmd_part = nullptr;
      D.dmmd_part_cap = 0;
      D.bg_on = false;                  // its staging goes with them too
    }
    mm_tuned = false;
    mm_tuned64 = false;
    dmmd_tuned = false;
    mm_part = nullptr;                 // freed with the batched buffers below
    mm_part_cap = 0;
    Bg_part = Bg_G = Bg_F = Bg_C = nullptr;
    drop_graphs(true);
    for (void* ptr : ballocs) (void)hipFree(ptr);
    ballocs.clear();
    bytes -= bbytes;
    bbytes = 0;
    bwidth = 0;
  }
  template <typename T>
  T* upload_f(const std::vector<double>& v) {   // FP64 host data in precision T
    if (sizeof(T) == sizeof(double)) return (T*)upload(v);
    std::vector<T> t(v.begin(), v.end());
    return upload(t);
  }
  void free_all() {
    free_batched();
    drop_graphs(false);
    for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
    for (auto& e : ev_rr)
      if (e) (void)hipEventDestroy(e);
    ev_rr[0] = ev_rr[1] = nullptr;
    prof.pool.clear();
    for (void* ptr : allocs) (void)hipFree(ptr);
    allocs.clear();
    if (sc_host) (void)hipHostFree(sc_host);
    sc_host = nullptr;
    if (Bactive_host) (void)hipHostFree(Bactive_host);
    Bactive_host = nullptr;
    if (Bparts_host) (void)hipHostFree(Bparts_host);
    Bparts_host = nullptr;
    if (Bg_host) (void)hipHostFree(Bg_host);
    Bg_host = nullptr;
    bytes = 0;
  }
};

namespace {

// Row-group tasks of a coarse level (k_grp_ata) and the cover lists of the
// staged output.  gp: CSR row pointer of the stored rows of G_l.
// Tasks of the row-group pass on 64 columns (k_bgrp_ata64): a workgroup per
// task of at most 32 rows of one group, covering support columns t0..c-1 (at
// most 128 of them: the staged input rows and the rows' products fit 64 KB
// of LDS in FP32); the staged output of each task and the cover lists of the
// unknowns follow the single-vector layout, with positions in rows of 64.
void build_bgroup_tasks(lsamg_handle* h, const Level& HL, DLevel& D,
                        const std::vector<int64_t>& gp) {
  constexpr int RPT = 32, WMAX = 128;
  const Groups& G = HL.G;
  std::vector<int64_t> vs, s0v, so;
  std::vector<int32_t> nr, t0v, cv;
  std::vector<std::pair<int32_t, int64_t>> cover;
  int64_t row = 0, nstg = 0;
  int wmax = 0;
  for (int64_t g = 0; g < G.ng(); ++g) {
    const int c = (int)(G.sptr[g + 1] - G.sptr[g]);
    const int ntk = (G.nrows[g] + RPT - 1) / RPT;
    const int chunk = (G.nrows[g] + ntk - 1) / ntk;
    for (int t0 = 0; t0 < G.nrows[g]; t0 += chunk) {
      const int w = c - t0, k = std::min(chunk, G.nrows[g] - t0);
      if (w > WMAX) return;
      wmax = std::max(wmax, w);
      vs.push_back(gp[row + t0]);
      nr.push_back(k);
      t0v.push_back(t0);
      cv.push_back(c);
      s0v.push_back(G.sptr[g]);
      so.push_back(nstg);
      for (int j = t0; j < c; ++j) cover.emplace_back(G.supp[G.sptr[g] + j], nstg + (j - t0));
      nstg += w;
    }
    row += G.nrows[g];
  }
  std::vector<int64_t> cp(D.n + 1, 0), cs(cover.size());
  for (auto& e : cover) cp[e.first + 1]++;
  for (int64_t j = 0; j < D.n; ++j) cp[j + 1] += cp[j];
  {
    std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
    for (auto& e : cover) cs[fill[e.first]++] = e.second;   // ascending position
  }
  D.bgtask = dev::GrpTasks{h->upload(vs), h->upload(nr), h->upload(t0v), h->upload(cv),
                           h->upload(s0v), h->upload(so)};
  D.bg_ntask = (int64_t)vs.size();
  D.bg_nstg = nstg;
  D.bg_wmax = wmax;
  D.bg_cptr = h->upload(cp);
  D.bg_cpos = h->upload(cs);
  D.bg_ok = true;
}

void build_group_tasks(lsamg_handle* h, const Level& HL, DLevel& D,
                       const std::vector<int64_t>& gp) {
  const Groups& G = HL.G;
  int cmax = 0;
  for (int64_t g = 0; g < G.ng(); ++g) cmax = std::max<int>(cmax, (int)(G.sptr[g + 1] - G.sptr[g]));
  if (cmax == 0 || cmax > 64 * 16) return;        // keep the two-pass CSR form
  // small supports (c <= 128): a lane group of lw lanes (4 chunks) per task
  // of <= rw rows, rw from the mean rows per group; large supports: a
  // workgroup of nw wavefronts per task of nw * rw rows
  int lw = 64, kc = 1, nw = 0, rw = 4;
  if (cmax <= 128) {
    lw = 4;
    while (lw * 4 < cmax) lw <<= 1;
    while (kc * lw < cmax) kc <<= 1;
    const double mean_rows = (double)G.total_rows() / (double)std::max<int64_t>(1, G.ng());
    while (rw < 16 && rw < mean_rows) rw <<= 1;
  } else {
    while (kc * 64 < cmax) kc <<= 1;
    nw = kc >= 16 ? 4 : 8;       // LDS stays below 64 KiB in FP64
    rw = kc >= 8 ? 4 : 8;
  }
  const int rpt = nw > 0 ? nw * rw : rw;
  std::vector<int64_t> vs, s0v, so;
  std::vector<int32_t> nr, t0v, cv;
  std::vector<std::pair<int32_t, int64_t>> cover;   // (unknown, staging position)
  int64_t row = 0, nstg = 0;
  for (int64_t g = 0; g < G.ng(); ++g) {
    const int c = (int)(G.sptr[g + 1] - G.sptr[g]);
    // split the group's rows evenly into tasks of at most rpt rows
    const int ntk = (G.nrows[g] + rpt - 1) / rpt;
    const int chunk = (G.nrows[g] + ntk - 1) / ntk;
    for (int t0 = 0; t0 < G.nrows[g]; t0 += chunk) {
      vs.push_back(gp[row + t0]);
      nr.push_back(std::min(chunk, G.nrows[g] - t0));
      t0v.push_back(t0);
      cv.push_back(c);
      s0v.push_back(G.sptr[g]);
      so.push_back(nstg);
      for (int j = t0; j < c; ++j) cover.emplace_back(G.supp[G.sptr[g] + j], nstg + (j - t0));
      nstg += c - t0;
    }
    row += G.nrows[g];
  }
  if (nstg >= ((int64_t)1 << 31)) return;         // positions are 32-bit
  std::vector<int64_t> cp(D.n + 1, 0);
  std::vector<int32_t> cs(cover.size());
  for (auto& e : cover) cp[e.first + 1]++;
  for (int64_t j = 0; j < D.n; ++j) cp[j + 1] += cp[j];
  {
    std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
    for (auto& e : cover) cs[fill[e.first]++] = (int32_t)e.second;   // ascending position
  }
  D.grp = true;
  D.grp_lw = lw;
  D.grp_kc = kc;
  D.grp_nw = nw;
  D.grp_rw = rw;
  D.grp_ntask = (int64_t)vs.size();
  D.grp_nstg = nstg;
  D.gtask = dev::GrpTasks{h->upload(vs), h->upload(nr), h->upload(t0v), h->upload(cv),
                          h->upload(s0v), h->upload(so)};
  D.grp_supp = h->upload(G.supp);
  D.rc_ptr = h->upload(cp);
  D.rc_pos = h->upload(cs);
  build_bgroup_tasks(h, HL, D, gp);
  D.d.stg = h->alloc<double>(nstg);
  D.f.stg = h->alloc<float>(nstg);
}

// Packed symmetric copy (k_sym_gemv) of the dense level operator, from the
// FP64 matrix in D.d.Ainv (fill = false: allocate only).
void make_packed(lsamg_handle* h, DLevel& D, bool fill) {
  const int64_t n = D.n;
  D.nT = (int)((n + dev::kTile - 1) / dev::kTile);
  const int64_t nt = (int64_t)D.nT * (D.nT + 1) / 2;
  const size_t tile = (size_t)dev::kTile * dev::kTile;
  D.d.Spk = h->alloc<double>((size_t)nt * tile);
  D.f.Spk = h->alloc<float>((size_t)nt * tile);
  D.d.spart = h->alloc<double>((size_t)D.nT * D.nT * dev::kTile);
  D.f.spart = h->alloc<float>((size_t)D.nT * D.nT * dev::kTile);
  if (h->dry || !fill) return;
  KLAUNCH0((unsigned)nt, dev::kBlock, 0, nullptr, dev::k_sym_pack<double>, n,
           (const double*)D.d.Ainv, D.d.Spk);
  LAUNCH_OK();
  KLAUNCH0((unsigned)nt, dev::kBlock, 0, nullptr, dev::k_sym_pack<float>, n,
           (const double*)D.d.Ainv, D.f.Spk);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(nullptr));
}

// The dense level operator Ainv (n x n) as a one-block operator of the
// multi-right-hand-side GEMM.
void make_dense_plan(lsamg_handle* h, DLevel& D) {
  GemvPlan& P = D.dense;
  std::vector<int64_t> z1(1, 0);
  std::vector<int32_t> n1(1, (int32_t)D.n);
  int32_t* dn = h->upload(n1);
  int64_t* dz = h->upload(z1);
  P.op = dev::GemvOp{dz, dn, dn, dz, dz, 0};
  P.nagg = 1;
  P.hlj = n1;
  P.hll = n1;
  P.lmax = (int)D.n;
  P.mat = D.n * D.n;
  P.in_u = P.out = D.n;
  std::vector<int32_t> ta, tj;
  for (int64_t j = 0; j < D.n; j += 64) {
    ta.push_back(0);
    tj.push_back((int32_t)j);
  }
  P.ntask = (int64_t)ta.size();
  P.task_a = h->upload(ta);
  P.task_j0 = h->upload(tj);
}

// Tiles of the one-pass G^T (G X) (k_bata_tile on 64 columns: TS = 16; the
// single-vector CG's k_cg_tile: TS = 256): TS consecutive unknowns per tile;
// for each tile the unknowns its rows of G reach (U_t) and those rows (R_t),
// both ascending; per row of R_t its entries in row order as (position in
// U_t, value), per unknown its rows in G^T order as (position in R_t, value),
// padded with zero values to the compiled bounds MF and ME.  Fails (false)
// when a tile's two LDS buffers (row_bytes per staged row in FP64) would
// exceed 64 KB, or, with wave_rows, when a wavefront's share of R_t would
// not fit one metadata load.
struct TileHost {
  std::vector<int32_t> uptr{0}, ucol, rptr{0};
  std::vector<uint16_t> rli, drl, eli;
  std::vector<double> rv, dw, ev;
  int umax = 0, rmax = 0;
  int64_t ntile = 0;
};

bool make_tiles(const DLevel& D, const std::vector<int64_t>& gp, const std::vector<int32_t>& gc,
                const std::vector<double>& gv, const std::vector<int64_t>& tp,
                const std::vector<int32_t>& tc, const std::vector<double>& tv, int TS,
                int64_t row_bytes, bool wave_rows, bool expand, TileHost& T) {
  const int ME = D.ata_me, MF = D.ata_mf;
  const int64_t n = D.n;
  T.ntile = (n + TS - 1) / TS;
  T.drl.assign((size_t)n * ME, 0);
  T.dw.assign((size_t)n * ME, 0.0);
  if (expand) {
    T.eli.assign((size_t)n * ME * MF, 0);
    T.ev.assign((size_t)n * ME * MF, 0.0);
  }
  std::vector<int32_t> rows, cols;
  auto pos = [](const std::vector<int32_t>& v, int32_t x) {
    return (uint16_t)(std::lower_bound(v.begin(), v.end(), x) - v.begin());
  };
  for (int64_t t = 0; t < T.ntile; ++t) {
    const int64_t d0 = t * TS, d1 = std::min<int64_t>(n, d0 + TS);
    rows.clear();
    for (int64_t d = d0; d < d1; ++d) rows.insert(rows.end(), tc.begin() + tp[d], tc.begin() + tp[d + 1]);
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    cols.clear();
    for (int32_t r : rows) cols.insert(cols.end(), gc.begin() + gp[r], gc.begin() + gp[r + 1]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    T.umax = std::max(T.umax, (int)cols.size());
    T.rmax = std::max(T.rmax, (int)rows.size());
    if ((int64_t)(T.umax + T.rmax) * row_bytes > 65536) return false;
    if (wave_rows && (T.rmax + 3) / 4 * MF > 64) return false;
    for (int32_t r : rows)
      for (int q = 0; q < MF; ++q) {
        const int64_t f = gp[r] + q;
        const bool ok = f < gp[r + 1];
        T.rli.push_back(ok ? pos(cols, gc[f]) : 0);
        T.rv.push_back(ok ? gv[f] : 0.0);
      }
    for (int64_t d = d0; d < d1; ++d)
      for (int k = 0; k < ME; ++k) {
        const int64_t e = tp[d] + k;
        if (e >= tp[d + 1]) continue;
        T.drl[(size_t)d * ME + k] = pos(rows, tc[e]);
        T.dw[(size_t)d * ME + k] = tv[e];
        // expanded form: the row's entries, in row order
        const int32_t r = tc[e];
        for (int q = 0; expand && q < MF && gp[r] + q < gp[r + 1]; ++q) {
          const size_t x = ((size_t)d * ME + k) * MF + q;
          T.eli[x] = pos(cols, gc[gp[r] + q]);
          T.ev[x] = gv[gp[r] + q];
        }
      }
    T.ucol.insert(T.ucol.end(), cols.begin(), cols.end());
    T.uptr.push_back((int32_t)T.ucol.size());
    T.rptr.push_back(T.rptr.back() + (int32_t)rows.size());
  }
  return true;
}

dev::AtaTiles upload_tiles(lsamg_handle* h, const TileHost& T) {
  return dev::AtaTiles{h->upload(T.uptr), h->upload(T.ucol), h->upload(T.rptr), h->upload(T.rli),
                       h->upload(T.drl), h->upload(T.eli), T.ntile, T.umax};
}

void build_ata_tiles(lsamg_handle* h, DLevel& D, const std::vector<int64_t>& gp,
                     const std::vector<int32_t>& gc, const std::vector<double>& gv,
                     const std::vector<int64_t>& tp, const std::vector<int32_t>& tc,
                     const std::vector<double>& tv) {
  {
    TileHost T;
    if (make_tiles(D, gp, gc, gv, tp, tc, tv, kAtaTile, 64 * 8, true, true, T)) {
      D.at = upload_tiles(h, T);
      D.at_rmax = T.rmax;
      D.d.trv = h->upload_f<double>(T.rv);
      D.f.trv = h->upload_f<float>(T.rv);
      D.d.tdw = h->upload_f<double>(T.dw);
      D.f.tdw = h->upload_f<float>(T.dw);
      D.d.tev = h->upload_f<double>(T.ev);
      D.f.tev = h->upload_f<float>(T.ev);
      D.at_ok = D.at_on = true;
    }
  }
  {
    TileHost T;
    if (make_tiles(D, gp, gc, gv, tp, tc, tv, dev::kBlock, 8, false, false, T)) {
      D.at1 = upload_tiles(h, T);
      D.at1_rmax = T.rmax;
      D.trv1 = h->upload_f<double>(T.rv);
      D.tdw1 = h->upload_f<double>(T.dw);
      D.at1_ok = D.at1_on = true;
    }
  }
}

// Build the device image of one level from the host hierarchy.
void upload_level(lsamg_handle* h, const Level& HL, DLevel& D, bool finest) {
  D.n = HL.n;
  D.coarsest = HL.coarsest;
  // CSR of G_l: finest rows as given; coarse groups store the upper
  // trapezoid of their R factor (row t keeps support columns t..c-1)
  std::vector<int64_t> gp(1, 0);
  std::vector<int32_t> gc;
  std::vector<double> gv;
  const Groups& G = HL.G;
  for (int64_t g = 0; g < G.ng(); ++g) {
    const int64_t s0 = G.sptr[g];
    const int c = (int)(G.sptr[g + 1] - s0);
    const double* R = G.val.data() + G.vptr[g];
    const bool tri = G.nrows[g] > 1;
    for (int t = 0; t < G.nrows[g]; ++t) {
      for (int j = tri ? t : 0; j < c; ++j) {
        gc.push_back(G.supp[s0 + j]);
        gv.push_back(R[(size_t)t * c + j]);
      }
      gp.push_back((int64_t)gc.size());
    }
  }
  D.nrows = (int64_t)gp.size() - 1;
  D.nnz = (int64_t)gc.size();
  // transpose
  std::vector<int64_t> tp(D.n + 1, 0);
  for (int32_t c : gc) tp[c + 1]++;
  for (int64_t j = 0; j < D.n; ++j) tp[j + 1] += tp[j];
  std::vector<int32_t> tc(D.nnz);
  std::vector<double> tv(D.nnz);
  {
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t r = 0; r < D.nrows; ++r)
      for (int64_t e = gp[r]; e < gp[r + 1]; ++e) {
        const int64_t o = fill[gc[e]]++;
        tc[o] = (int32_t)r;
        tv[o] = gv[e];
      }
  }
  {
    int64_t rmax = 0, tmax = 0;
    for (int64_t r = 0; r < D.nrows; ++r) rmax = std::max(rmax, gp[r + 1] - gp[r]);
    for (int64_t j = 0; j < D.n; ++j) tmax = std::max(tmax, tp[j + 1] - tp[j]);
    // recomputing each row of G per touching unknown costs sum_r len(r)^2
    // gathers: worth it only for short rows (finite-difference G)
    D.fuse_ok = finest && rmax <= 4 && tmax <= 16;
    D.fuse_ata = D.fuse_ok;
    // the tightest compiled bounds: every gather beyond them is a wasted load
    D.ata_me = tmax <= 6 ? 6 : tmax <= 8 ? 8 : 16;
    D.ata_mf = rmax <= 3 ? 3 : 4;
  }
  D.lanes_g = lanes_for((double)D.nnz / std::max<int64_t>(1, D.nrows));
  D.lanes_gt = lanes_for((double)D.nnz / std::max<int64_t>(1, D.n));
  // a coarse coarsest level is solved densely and needs no G; the finest
  // level always keeps G (the outer CG applies A = G^T G there)
  if (!HL.coarsest || finest) {
    D.g_ptr = h->upload(gp);
    D.g_col = h->upload(gc);
    D.gt_ptr = h->upload(tp);
    D.gt_col = h->upload(tc);
    D.d.g_val = h->upload_f<double>(gv);
    D.f.g_val = h->upload_f<float>(gv);
    D.d.gt_val = h->upload_f<double>(tv);
    D.f.gt_val = h->upload_f<float>(tv);
  }
  if (finest && D.fuse_ok && !HL.coarsest) build_ata_tiles(h, D, gp, gc, gv, tp, tc, tv);
  if (!finest && !HL.coarsest) build_group_tasks(h, HL, D, gp);
  D.d.x = h->alloc<double>(D.n);
  D.d.b = h->alloc<double>(D.n);
  D.d.r = h->alloc<double>(D.n);
  D.d.y = h->alloc<double>(D.nrows);
  D.f.x = h->alloc<float>(D.n);
  D.f.b = h->alloc<float>(D.n);
  D.f.r = h->alloc<float>(D.n);
  D.f.y = h->alloc<float>(D.nrows);
  if (HL.coarsest) {
    D.d.Ainv = h->upload_f<double>(HL.Ainv);
    D.f.Ainv = h->upload_f<float>(HL.Ainv);
    make_packed(h, D, true);
    make_dense_plan(h, D);
    return;
  }
  D.nagg = HL.nagg;
  D.ntb = HL.optr[HL.nagg];
  for (int64_t a = 0; a < HL.nagg; ++a) {
    D.max_nO = std::max<int>(D.max_nO, (int)(HL.optr[a + 1] - HL.optr[a]));
    D.max_nw = std::max<int>(D.max_nw, (int)(HL.astart[a + 1] - HL.astart[a]));
    D.max_k = std::max<int>(D.max_k, HL.k[a]);
  }
  // device layouts of Z_i (row-major for RAS-T, column-major for RAS) and of
  // Zhat_i (row-major for P^T, column-major for P): every row padded with
  // zeros to a multiple of 4 entries, and every block starting at a multiple
  // of 4 entries, so each row starts 16-byte aligned; an operator with rows
  // longer than 256 entries (the wide forms split them into several output
  // slices) pads its rows to 32 entries instead, so each row starts on a
  // 128-byte line and neighbouring slices share no line
  int64_t max_nw = 1, max_nO = 1, max_k = 1;
  for (int64_t a = 0; a < HL.nagg; ++a) {
    max_nw = std::max<int64_t>(max_nw, HL.astart[a + 1] - HL.astart[a]);
    max_nO = std::max<int64_t>(max_nO, HL.optr[a + 1] - HL.optr[a]);
    max_k = std::max<int64_t>(max_k, HL.k[a]);
  }
  const int64_t pr_ = max_nO > 256 ? 32 : 4, pc_ = max_nw > 256 ? 32 : 4,
                ph_ = max_k > 256 ? 32 : 4;
  auto padto = [](int64_t v, int64_t q) { return (v + q - 1) / q * q; };
  auto padr = [&](int64_t v) { return padto(v, pr_); };   // rows of Omega_i entries
  auto padc = [&](int64_t v) { return padto(v, pc_); };   // rows of omega_i entries
  auto padh = [&](int64_t v) { return padto(v, ph_); };   // rows of k_i entries
  auto opad = [](int64_t q) { return q == 4 ? 1 : (int)q; };
  std::vector<int64_t> offr(HL.nagg), offc(HL.nagg), offh(HL.nagg), offt(HL.nagg);
  int64_t totr = 0, totc = 0, toth = 0, tott = 0;
  for (int64_t a = 0; a < HL.nagg; ++a) {
    const int64_t nw = HL.astart[a + 1] - HL.astart[a], nO = HL.optr[a + 1] - HL.optr[a],
                  k = HL.k[a];
    offr[a] = totr;
    totr += nw * padr(nO);
    offc[a] = totc;
    totc += nO * padc(nw);
    offh[a] = toth;
    toth += nw * padh(k);
    offt[a] = tott;
    tott += k * padc(nw);
  }
  std::vector<double> Zr(totr, 0.0), Zc(totc, 0.0), Zh(toth, 0.0), ZhT(tott, 0.0);
  for (int64_t a = 0; a < HL.nagg; ++a) {
    const int64_t nw = HL.astart[a + 1] - HL.astart[a], nO = HL.optr[a + 1] - HL.optr[a],
                  k = HL.k[a];
    const double* z = HL.Z.data() + HL.zoff[a];        // host: |omega| x |Omega| row-major
    const double* zh = HL.Zhat.data() + HL.poff[a];    // host: |omega| x k row-major
    for (int64_t p = 0; p < nw; ++p) {
      for (int64_t c = 0; c < nO; ++c) {
        Zr[offr[a] + p * padr(nO) + c] = z[p * nO + c];
        Zc[offc[a] + c * padc(nw) + p] = z[p * nO + c];
      }
      for (int64_t t = 0; t < k; ++t) {
        Zh[offh[a] + p * padh(k) + t] = zh[p * k + t];
        ZhT[offt[a] + t * padc(nw) + p] = zh[p * k + t];
      }
    }
  }
  // additive cycle: the whole A_i^{-1} (symmetric), rows padded as above
  std::vector<int64_t> offa(HL.nagg);
  std::vector<double> As;
  const bool additive = !HL.aoff.empty();
  if (additive) {
    int64_t tota = 0;
    for (int64_t a = 0; a < HL.nagg; ++a) {
      offa[a] = tota;
      tota += (HL.optr[a + 1] - HL.optr[a]) * padr(HL.optr[a + 1] - HL.optr[a]);
    }
    As.assign(tota, 0.0);
    for (int64_t a = 0; a < HL.nagg; ++a) {
      const int64_t nO = HL.optr[a + 1] - HL.optr[a];
      const double* z = HL.Ainv_loc.data() + HL.aoff[a];
      for (int64_t l = 0; l < nO; ++l)
        for (int64_t j = 0; j < nO; ++j) As[offa[a] + l * padr(nO) + j] = z[l * nO + j];
    }
  }
  // cover lists for the RAS-T gather: for unknown j, staging positions
  // optr[i] + (index of j in Omega_i), ascending i
  std::vector<int64_t> cp(D.n + 1, 0);
  for (int32_t j : HL.oidx) cp[j + 1]++;
  for (int64_t j = 0; j < D.n; ++j) cp[j + 1] += cp[j];
  std::vector<int64_t> cs(cp[D.n]);
  {
    std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
    for (int64_t a = 0; a < HL.nagg; ++a)
      for (int64_t o = HL.optr[a]; o < HL.optr[a + 1]; ++o) cs[fill[HL.oidx[o]]++] = o;
  }
  D.astart = h->upload(HL.astart);
  D.optr = h->upload(HL.optr);
  D.oidx = h->upload(HL.oidx);
  D.cstart = h->upload(HL.cstart);
  D.kk = h->upload(HL.k);
  D.cptr = h->upload(cp);
  D.cpos = h->upload(cs);
  D.d.Zr = h->upload_f<double>(Zr);
  D.f.Zr = h->upload_f<float>(Zr);
  D.d.Zc = h->upload_f<double>(Zc);
  D.f.Zc = h->upload_f<float>(Zc);
  D.d.Zh = h->upload_f<double>(Zh);
  D.f.Zh = h->upload_f<float>(Zh);
  D.d.ZhT = h->upload_f<double>(ZhT);
  D.f.ZhT = h->upload_f<float>(ZhT);
  std::vector<int32_t> nw(HL.nagg), nO(HL.nagg), kk(HL.k.begin(), HL.k.end());
  std::vector<int64_t> w0(HL.astart.begin(), HL.astart.end() - 1),
      o0(HL.optr.begin(), HL.optr.end() - 1), c0(HL.cstart.begin(), HL.cstart.end() - 1);
  for (int64_t a = 0; a < HL.nagg; ++a) {
    nw[a] = (int32_t)(HL.astart[a + 1] - HL.astart[a]);
    nO[a] = (int32_t)(HL.optr[a + 1] - HL.optr[a]);
  }
  int32_t* d_nw = h->upload(nw);
  int32_t* d_nO = h->upload(nO);
  int32_t* d_k = h->upload(kk);
  int64_t* d_w0 = h->upload(w0);
  int64_t* d_o0 = h->upload(o0);
  int64_t* d_offr = h->upload(offr);
  int64_t* d_offc = h->upload(offc);
  int64_t* d_offh = h->upload(offh);
  int64_t* d_offt = h->upload(offt);
  int64_t* d_c0 = h->upload(c0);
  auto plan = [&](GemvPlan& P, const std::vector<int32_t>& lj, const std::vector<int32_t>& ll,
                  int32_t* dlj, int32_t* dll, int64_t* moff, int64_t* ib, int64_t* ob,
                  int64_t in_unique, bool gathered, int pad) {
    P.op = dev::GemvOp{moff, dlj, dll, ib, ob, pad};
    P.nagg = HL.nagg;
    P.hlj = lj;
    P.hll = ll;
    P.mat = P.out = 0;
    for (int64_t a = 0; a < HL.nagg; ++a) {
      P.mat += (int64_t)lj[a] * ll[a];
      P.out += lj[a];
      if (gathered) P.idx += ll[a];
    }
    P.in_u = in_unique;
    P.lmax = *std::max_element(ll.begin(), ll.end());
    const int ljmax = *std::max_element(lj.begin(), lj.end());
    // tasks (aggregate, 64-wide output slice): the wide single-vector form
    // and the batched form both use them
    std::vector<int32_t> ta, tj;
    for (int64_t a = 0; a < HL.nagg; ++a)
      for (int j = 0; j < lj[a]; j += 64) {
        ta.push_back((int32_t)a);
        tj.push_back(j);
      }
    P.ntask = (int64_t)ta.size();
    P.task_a = h->upload(ta);
    P.task_j0 = h->upload(tj);
    P.G = 0;
    if (ljmax > 64) {
      std::vector<int32_t> ta4, tj4;
      for (int64_t a = 0; a < HL.nagg; ++a)
        for (int j = 0; j < lj[a]; j += 256) {
          ta4.push_back((int32_t)a);
          tj4.push_back(j);
        }
      P.ntask4 = (int64_t)ta4.size();
      P.task4_a = h->upload(ta4);
      P.task4_j0 = h->upload(tj4);
    }
    if (ljmax <= 64) {
      int g = 1;
      while (g < ljmax) g <<= 1;
      P.G = g;
      return;
    }
    P.NW = 4;
    while (P.NW < 16 && P.ntask * P.NW < 4096) P.NW <<= 1;
  };
  const int64_t ncoarse = HL.cstart[HL.nagg];
  plan(D.ras, nw, nO, d_nw, d_nO, d_offc, d_o0, d_w0, D.n, true, opad(pc_));
  plan(D.rast, nO, nw, d_nO, d_nw, d_offr, d_w0, d_o0, D.n, false, opad(pr_));
  plan(D.rst, kk, nw, d_k, d_nw, d_offh, d_w0, d_c0, D.n, false, opad(ph_));
  plan(D.pro, nw, kk, d_nw, d_k, d_offt, d_c0, d_w0, ncoarse, false, opad(pc_));
  if (additive) {
    D.d.As = h->upload_f<double>(As);
    D.f.As = h->upload_f<float>(As);
    plan(D.as, nO, nO, d_nO, d_nO, h->upload(offa), d_o0, d_o0, D.n, true, opad(pr_));
  }
  if (finest) {      // inputs of P^T and RAS-T are residual rows omega_a formed on the fly
    int64_t em = 0;
    for (int64_t a = 0; a < HL.nagg; ++a) em = std::max(em, tp[HL.astart[a + 1]] - tp[HL.astart[a]]);
    D.rst.emax = D.rast.emax = (int)em;
  }
  D.d.tb = h->alloc<double>(D.ntb);
  D.f.tb = h->alloc<float>(D.ntb);
}

void build_tail(lsamg_handle* h, size_t lc);

// Staging of the allocation-free entry point (lsamg_apply_op_noalloc): one
// array per GPU for the whole process.  Host code never passes `scratch`
// itself to a kernel (on the host it is only a stand-in symbol); it uses the
// device address that hipGetSymbolAddress returns, resolved once per device
// with that device current and kept in g_scratch_dev.
constexpr int64_t kScratchDoubles = LSAMG_NOALLOC_SCRATCH_BYTES / sizeof(double);
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
double* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices)
    throw DevError{LSAMG_EINVAL, "device index beyond the allocation-free staging table"};
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      throw DevError{LSAMG_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e)};
    g_scratch_dev[device] = (double*)ptr;
  }
  return g_scratch_dev[device];
}

void upload(lsamg_handle* h) {
  if (!h->dry) HIP_OK(hipSetDevice(h->device));
  if (!h->dry) (void)scratch_on(h->device);   // resolve the staging address at set-up
  h->L.resize(h->H.levels.size());
  for (size_t l = 0; l < h->H.levels.size(); ++l) upload_level(h, h->H.levels[l], h->L[l], l == 0);
  const Level& L0 = h->H.levels[0];
  h->perm = h->upload(L0.canon);
  const int64_t n = L0.n;
  h->x = h->alloc<double>(n);
  h->r = h->alloc<double>(n);
  h->z = h->alloc<double>(n);
  h->p = h->alloc<double>(n);
  h->p2 = h->alloc<double>(n);
  h->q = h->alloc<double>(n);
  h->bi = h->alloc<double>(n);
  h->part = h->alloc<double>(h->nparts);
  h->sc = h->alloc<double>(8);
  h->red_np = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + dev::kBlock - 1) / dev::kBlock));
  h->p_pq = h->alloc<double>(h->red_np);
  h->p_rr = h->alloc<double>(h->red_np);
  h->p_rz[0] = h->alloc<double>(h->red_np);
  h->p_rz[1] = h->alloc<double>(h->red_np);
  h->p_tmp = h->alloc<double>(h->red_np);
  h->p_zq = h->alloc<double>(h->red_np);
  h->p_pqo = h->alloc<double>(h->red_np);
  // dense tail: the first level below the finest that is small enough
  size_t lc = 0;
  if (h->H.params.dense_tail > 0 && h->H.params.cycle == LSAMG_CYCLE_V)
    for (size_t l = 1; l < h->L.size() && !h->L[l].coarsest; ++l)
      if (h->L[l].n <= h->H.params.dense_tail) {
        lc = l;
        break;
      }
  if (lc > 0) build_tail(h, lc);
  if (h->dry) return;
  HIP_OK(hipHostMalloc((void**)&h->sc_host, 3 * 1024 * sizeof(double), hipHostMallocDefault));
  for (auto& e : h->ev_rr) HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

// Device bytes the upload of h's hierarchy will allocate (no GPU call).
size_t planned_device_bytes(lsamg_handle* h) {
  lsamg_handle t;
  std::swap(t.H, h->H);   // the dry upload reads only the host hierarchy
  t.dry = true;
  t.device = h->device;
  try {
    upload(&t);
  } catch (...) {
    std::swap(t.H, h->H);
    throw;
  }
  std::swap(t.H, h->H);
  return t.bytes;
}

// --------------------------------------------------------------------------
// kernel launch helpers
// --------------------------------------------------------------------------
template <typename T>
void spmv_csr(int64_t rows, int lanes, const int64_t* ptr, const int32_t* col, const T* val,
              const T* x, T* y, hipStream_t s, int64_t nnz, int64_t ncols) {
  const unsigned g = nblocks((rows + 1) / 2 * lanes);
  PROF(kname("k_spmv", std::string(tname<T>()) + ", " + std::to_string(lanes)),
       nnz * (sizeof(T) + 4) + 8 * (rows + 1) + sizeof(T) * (ncols + rows), s);
  switch (lanes) {
#define CASE(L) \
  case L: KLAUNCH(g, dev::kBlock, 0, s, dev::k_spmv<T, L>, rows, ptr, col, val, x, y); break;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
  }
  LAUNCH_OK();
}

template <typename T>
void resid_csr(int64_t rows, int lanes, const int64_t* ptr, const int32_t* col, const T* val,
               const T* y, const T* b, T* r, hipStream_t s, int64_t nnz, int64_t ny) {
  const unsigned g = nblocks((rows + 1) / 2 * lanes);
  PROF(kname("k_resid_t", std::string(tname<T>()) + ", " + std::to_string(lanes)),
       nnz * (sizeof(T) + 4) + 8 * (rows + 1) + sizeof(T) * (ny + 2 * rows), s);
  switch (lanes) {
#define CASE(L) \
  case L: KLAUNCH(g, dev::kBlock, 0, s, dev::k_resid_t<T, L>, rows, ptr, col, val, y, b, r); break;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
  }
  LAUNCH_OK();
}

// Autotuning of the single-vector wide GEMV (wavefronts per task): while a
// GvTune is active on the calling thread (one eager V-cycle on the first
// solve of each precision), every wide GEMV whose shape is not tuned yet times
// each candidate on its real inputs, writing to a scratch output (so that
// accumulating operators are not applied twice), and keeps the fastest.
struct GvTune {
  void* scratch = nullptr;      // >= the longest GEMV output, in doubles
  hipEvent_t e0 = nullptr, e1 = nullptr;
};
thread_local GvTune* g_gvtune = nullptr;

template <typename T, int MODE, bool ADD, int NW>
void gemv_wide_launch(const GemvPlan& P, const dev::InSpec<T>& sp, const T* M, const T* in,
                      T* out, hipStream_t s, const ProfScope& ps_) {
  const int emax = MODE == dev::IN_RESG ? P.emax : 0;
  const size_t lds = ((size_t)P.lmax + emax + (size_t)NW * 64) * sizeof(T);
  KLAUNCH((unsigned)P.ntask, NW * 64, lds, s, dev::k_gemv_wide<T, MODE, ADD, NW>, P.task_a,
          P.task_j0, P.op, P.lmax, emax, sp, M, in, out);
}

template <int MODE, bool ADD, int NW>
void gemv_wide4_launch(const GemvPlan& P, const dev::InSpec<float>& sp, const float* M,
                       const float* in, float* out, hipStream_t s, const ProfScope& ps_) {
  const int emax = MODE == dev::IN_RESG ? P.emax : 0;
  const size_t lds = ((((size_t)P.lmax + emax + 3) & ~(size_t)3) + (size_t)NW * 256) * sizeof(float);
  KLAUNCH((unsigned)P.ntask4, NW * 64, lds, s, dev::k_gemv_wide4<MODE, ADD, NW>, P.task4_a,
          P.task4_j0, P.op, P.lmax, emax, sp, M, in, out);
}

// wide GEMV with nw wavefronts per task; form 1 (FP32 only): four outputs per lane
template <typename T, int MODE, bool ADD>
void gemv_wide_nw(int nw, int form, const GemvPlan& P, const dev::InSpec<T>& sp, const T* M,
                  const T* in, T* out, hipStream_t s, const ProfScope& ps) {
  if constexpr (std::is_same<T, float>::value) {
    if (form == 1) {
      if (nw == 4)
        gemv_wide4_launch<MODE, ADD, 4>(P, sp, M, in, out, s, ps);
      else if (nw == 8)
        gemv_wide4_launch<MODE, ADD, 8>(P, sp, M, in, out, s, ps);
      else
        gemv_wide4_launch<MODE, ADD, 16>(P, sp, M, in, out, s, ps);
      return;
    }
  }
  if (nw == 4)
    gemv_wide_launch<T, MODE, ADD, 4>(P, sp, M, in, out, s, ps);
  else if (nw == 8)
    gemv_wide_launch<T, MODE, ADD, 8>(P, sp, M, in, out, s, ps);
  else
    gemv_wide_launch<T, MODE, ADD, 16>(P, sp, M, in, out, s, ps);
}

// narrow form: a wavefront per four aggregates, lane groups of G
template <typename T, int MODE, bool ADD>
void gemv_narrow_launch(const GemvPlan& P, const dev::InSpec<T>& sp, const T* M, const T* in,
                        T* out, hipStream_t s, const ProfScope& ps_) {
  const unsigned g = (unsigned)((P.nagg + 3) / 4);
  const int emax = MODE == dev::IN_RESG ? P.emax : 0;
  const size_t lds = (size_t)4 * (P.lmax + emax) * sizeof(T);
  switch (P.G) {
#define CASE(GG)                                                                            \
  case GG:                                                                                  \
    KLAUNCH(g, dev::kBlock, lds, s, dev::k_gemv_narrow<T, MODE, ADD, GG>, P.nagg, P.op, P.lmax,  \
            emax, sp, M, in, out);                                                          \
    break;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
  }
}

// narrow form, an aggregate per lane group of G < 64 lanes
template <typename T, int MODE, bool ADD>
void gemv_narrow_m_launch(const GemvPlan& P, const dev::InSpec<T>& sp, const T* M, const T* in,
                          T* out, hipStream_t s, const ProfScope& ps_) {
  const int S = 64 / P.G;
  const unsigned g = (unsigned)((P.nagg + 4 * S - 1) / (4 * S));
  const int emax = MODE == dev::IN_RESG ? P.emax : 0;
  const size_t lds = (size_t)4 * S * (P.lmax + emax) * sizeof(T);
  switch (P.G) {
#define CASE(GG)                                                                              \
  case GG:                                                                                    \
    KLAUNCH(g, dev::kBlock, lds, s, dev::k_gemv_narrow_m<T, MODE, ADD, GG>, P.nagg, P.op, P.lmax, \
            emax, sp, M, in, out);                                                            \
    break;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32)
#undef CASE
  }
}

// narrow form with 16-byte loads, a wavefront per aggregate
template <typename T, int MODE, bool ADD>
void gemv_narrow4_launch(const GemvPlan& P, const dev::InSpec<T>& sp, const T* M, const T* in,
                         T* out, hipStream_t s, const ProfScope& ps_) {
  const unsigned g = (unsigned)((P.nagg + 3) / 4);
  const int emax = MODE == dev::IN_RESG ? P.emax : 0;
  const size_t lds = (size_t)4 * (((P.lmax + emax + 3) & ~3) + 64 * (16 / sizeof(T))) * sizeof(T);
  KLAUNCH(g, dev::kBlock, lds, s, dev::k_gemv_narrow4<T, MODE, ADD>, P.nagg, P.op, P.lmax, emax,
          sp, M, in, out);
}

template <typename T, int MODE, bool ADD>
void gemv(const GemvPlan& P, const dev::InSpec<T>& sp, const T* M, const T* in, T* out,
          hipStream_t s, int64_t extra_bytes = 0) {
  const int pi = sizeof(T) == sizeof(float) ? 1 : 0;
  // operators of <= 64 outputs per aggregate: the tuner times the narrow
  // form (a wavefront per aggregate), the narrow form with an aggregate per
  // lane group, and, when aggregates are few, the wide form (the loop split
  // over waves)
  const bool try_wide = P.G == 0 || P.nagg < 4096;
  if (P.nw_t[pi] == 0 && g_gvtune && !g_rec && (try_wide || P.G < 64)) {
    float best = 1e30f;
    int pick = P.NW, pick_form = 0, pick_narrow = 0;
    for (int nf = 1; nf <= 3 && P.G > 0; ++nf) {
      if (nf == 2 && P.G >= 64) continue;
      auto run = [&]() {
        if (nf == 1)
          gemv_narrow_launch<T, MODE, ADD>(P, sp, M, in, (T*)g_gvtune->scratch, s, kNoProf);
        else if (nf == 2)
          gemv_narrow_m_launch<T, MODE, ADD>(P, sp, M, in, (T*)g_gvtune->scratch, s, kNoProf);
        else
          gemv_narrow4_launch<T, MODE, ADD>(P, sp, M, in, (T*)g_gvtune->scratch, s, kNoProf);
      };
      run();
      for (int round = 0; round < 2; ++round) {
        HIP_OK(hipEventRecord(g_gvtune->e0, s));
        for (int r = 0; r < 3; ++r) run();
        HIP_OK(hipEventRecord(g_gvtune->e1, s));
        HIP_OK(hipEventSynchronize(g_gvtune->e1));
        float t = 0.f;
        HIP_OK(hipEventElapsedTime(&t, g_gvtune->e0, g_gvtune->e1));
        if (t < best) {
          best = t;
          pick_narrow = nf;
        }
      }
    }
    for (int form : {0, 1}) {
      if (!try_wide) break;
      if (form == 1 && (pi == 0 || P.ntask4 == 0)) continue;   // four outputs per lane: FP32, > 64 outputs
      for (int nw : {4, 8, 16}) {
        gemv_wide_nw<T, MODE, ADD>(nw, form, P, sp, M, in, (T*)g_gvtune->scratch, s, kNoProf);
        float ms = 1e30f;
        for (int round = 0; round < 2; ++round) {   // best of two rounds of three launches
          HIP_OK(hipEventRecord(g_gvtune->e0, s));
          for (int r = 0; r < 3; ++r)
            gemv_wide_nw<T, MODE, ADD>(nw, form, P, sp, M, in, (T*)g_gvtune->scratch, s, kNoProf);
          HIP_OK(hipEventRecord(g_gvtune->e1, s));
          HIP_OK(hipEventSynchronize(g_gvtune->e1));
          float t = 0.f;
          HIP_OK(hipEventElapsedTime(&t, g_gvtune->e0, g_gvtune->e1));
          ms = std::min(ms, t);
        }
        if (ms < best) {
          best = ms;
          pick = nw;
          pick_form = form;
          pick_narrow = 0;
        }
      }
    }
    P.nw_t[pi] = pick;
    P.narrow_t[pi] = pick_narrow;
    if (pi == 1) P.form_t = pick_form;
  }
  const int nform = P.G == 0 ? 0 : P.nw_t[pi] == 0 ? 1 : P.narrow_t[pi];
  const bool narrow = nform > 0;
  const int NWsel = P.nw_t[pi] ? P.nw_t[pi] : P.NW;
  const int form = pi == 1 ? P.form_t : 0;
  // the names are those of the kernel symbols (k_gemv_wide4 has no type parameter)
  PROF(kname(narrow ? (nform == 2 ? "k_gemv_narrow_m" : nform == 3 ? "k_gemv_narrow4" : "k_gemv_narrow")
                    : (form == 1 ? "k_gemv_wide4" : "k_gemv_wide"),
             (form == 1 && !narrow ? std::string() : std::string(tname<T>()) + ", ") +
                 std::to_string(MODE) + ", " + (ADD ? "true" : "false") +
                 (nform == 3 ? std::string()
                             : ", " + std::to_string(narrow ? P.G : NWsel))),
       sizeof(T) * (P.mat + P.in_u + P.out * (ADD ? 2 : 1)) + 4 * P.idx + 32 * P.nagg + extra_bytes,
       s);
  if (nform == 3) {
    gemv_narrow4_launch<T, MODE, ADD>(P, sp, M, in, out, s, ps_);
  } else if (nform == 2) {
    gemv_narrow_m_launch<T, MODE, ADD>(P, sp, M, in, out, s, ps_);
  } else if (narrow) {
    gemv_narrow_launch<T, MODE, ADD>(P, sp, M, in, out, s, ps_);
  } else {
    gemv_wide_nw<T, MODE, ADD>(NWsel, form, P, sp, M, in, out, s, ps_);
  }
  LAUNCH_OK();
}

template <typename T>
dev::InSpec<T> no_spec() {
  return dev::InSpec<T>{nullptr, nullptr, nullptr, nullptr, nullptr};
}

// x = RAS(b) from a zero initial guess (eq:ras)
template <typename T>
void ras(DLevel& L, const T* b, T* x, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  dev::InSpec<T> sp = no_spec<T>();
  sp.idx = L.oidx;
  gemv<T, dev::IN_GATHER, false>(L.ras, sp, P.Zc, b, x, s);
}

// staged RAS-T(r) (eq:ras-t) into tb; gather_add folds it into x
template <typename T>
void ras_t_stage(DLevel& L, const T* r, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  gemv<T, dev::IN_DIRECT, false>(L.rast, no_spec<T>(), P.Zr, r, P.tb, s);
}

template <typename T>
void gather_add(DLevel& L, T* x, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  PROF(kname("k_gather_add", tname<T>()),
       (sizeof(T) + 8) * L.ntb + 8 * (L.n + 1) + 2 * sizeof(T) * L.n, s);
  KLAUNCH(nblocks(L.n), dev::kBlock, 0, s, dev::k_gather_add<T>, L.n, L.cptr, L.cpos, P.tb, x);
  LAUNCH_OK();
}

// First pass of the residual b - A x of level L for a consumer that forms
// r(omega_i) on the fly: the row-group pass (coarse levels, staged output) or
// y = G x (finest level, G^T applied by the consumer).
template <typename T>
void resid_first(DLevel& L, const T* x, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  if (!L.grp) {
    if (!L.g_ptr || !L.gt_ptr) throw DevError{LSAMG_EINVAL, "G missing on the device"};
    spmv_csr<T>(L.nrows, L.lanes_g, L.g_ptr, L.g_col, P.g_val, x, P.y, s, L.nnz, L.n);
    return;
  }
  const int lw = L.grp_lw, kc = L.grp_kc, nw = L.grp_nw, rw = L.grp_rw;
  const double bytes = sizeof(T) * (L.nnz + L.n + L.grp_nstg) + 4 * L.grp_nstg + 36 * L.grp_ntask;
  if (nw > 0) {
    PROF(kname("k_grp_ata_wg", std::string(tname<T>()) + ", " + std::to_string(kc) + ", " +
                                   std::to_string(nw) + ", " + std::to_string(rw)),
         bytes, s);
    const size_t lds = (size_t)(nw * kc * 64) * sizeof(T);
    switch (kc * 10000 + nw * 100 + rw) {
#define CASE(KC, NW, RW)                                                                   \
  case KC * 10000 + NW * 100 + RW:                                                         \
    KLAUNCH((unsigned)L.grp_ntask, NW * 64, lds, s, dev::k_grp_ata_wg<T, KC, NW, RW>,      \
            L.gtask, P.g_val, L.grp_supp, x, P.stg);                                       \
    break;
      CASE(2, 8, 8) CASE(4, 8, 8) CASE(8, 8, 4) CASE(16, 4, 4)
#undef CASE
      default:
        throw DevError{LSAMG_EINVAL, "row-group pass: unsupported shape"};
    }
  } else {
    PROF(kname("k_grp_ata", std::string(tname<T>()) + ", " + std::to_string(lw) + ", " +
                                std::to_string(kc) + ", " + std::to_string(rw)),
         bytes, s);
    const unsigned g = nblocks(L.grp_ntask * lw);
    switch (lw * 10000 + kc * 100 + rw) {
#define CASE(LW, KC, RW)                                                                   \
  case LW * 10000 + KC * 100 + RW:                                                         \
    KLAUNCH(g, dev::kBlock, 0, s, dev::k_grp_ata<T, LW, KC, RW>, L.grp_ntask, L.gtask,     \
            P.g_val, L.grp_supp, x, P.stg);                                                \
    break;
#define CASES(LW, KC) CASE(LW, KC, 4) CASE(LW, KC, 8) CASE(LW, KC, 16)
      CASES(4, 1) CASES(4, 2) CASES(4, 4) CASES(8, 4) CASES(16, 4) CASES(32, 4)
#undef CASES
#undef CASE
      default:
        throw DevError{LSAMG_EINVAL, "row-group pass: unsupported shape"};
    }
  }
  LAUNCH_OK();
}

// out (=|+=) op(r) where r = b - A x is formed by the consumer from the first
// pass of resid_first
template <typename T, bool ADD>
void gemv_resid(DLevel& L, const GemvPlan& Pl, const T* M, const T* b, T* out, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  dev::InSpec<T> sp = no_spec<T>();
  if (L.grp) {
    // r = b - (staged row-group output), formed once for the level
    {
      PROF(kname("k_resid_stg", tname<T>()),
           (sizeof(T) + 4) * L.grp_nstg + 8 * (L.n + 1) + 2 * sizeof(T) * L.n, s);
      KLAUNCH(nblocks(L.n * 8), dev::kBlock, 0, s, dev::k_resid_stg<T>, L.n, L.rc_ptr, L.rc_pos,
              P.stg, b, P.r);
      LAUNCH_OK();
    }
    gemv<T, dev::IN_DIRECT, ADD>(Pl, sp, M, P.r, out, s);
  } else if (Pl.G == 0) {
    // the wide form has several output slices per aggregate, each of which
    // would re-form r(omega_i): form r once
    resid_csr<T>(L.n, L.lanes_gt, L.gt_ptr, L.gt_col, P.gt_val, P.y, b, P.r, s, L.nnz, L.nrows);
    gemv<T, dev::IN_DIRECT, ADD>(Pl, sp, M, P.r, out, s);
  } else {
    // the narrow forms can form r(omega_i) while staging their inputs, or
    // read r from its own pass: the first solve of each precision times both
    const int pi = sizeof(T) == sizeof(float) ? 1 : 0;
    sp.idx = L.gt_col;
    sp.ptr = L.gt_ptr;
    sp.v1 = P.gt_val;
    sp.v2 = P.y;
    auto on_the_fly = [&]() {
      gemv<T, dev::IN_RESG, ADD>(Pl, sp, M, b, out, s,
                                 (int64_t)(sizeof(T) + 4) * L.nnz + 8 * (L.n + 1) +
                                     sizeof(T) * L.nrows);
    };
    auto separate = [&]() {
      resid_csr<T>(L.n, L.lanes_gt, L.gt_ptr, L.gt_col, P.gt_val, P.y, b, P.r, s, L.nnz, L.nrows);
      gemv<T, dev::IN_DIRECT, ADD>(Pl, no_spec<T>(), M, P.r, out, s);
    };
    if (Pl.rsep_t[pi] == 0 && g_gvtune && !g_rec) {
      on_the_fly();                     // fixes the GEMV form first
      float best[2] = {1e30f, 1e30f};
      for (int f = 0; f < 2; ++f)
        for (int round = 0; round < 2; ++round) {
          HIP_OK(hipEventRecord(g_gvtune->e0, s));
          for (int r = 0; r < 3; ++r) f == 0 ? on_the_fly() : separate();
          HIP_OK(hipEventRecord(g_gvtune->e1, s));
          HIP_OK(hipEventSynchronize(g_gvtune->e1));
          float t = 0.f;
          HIP_OK(hipEventElapsedTime(&t, g_gvtune->e0, g_gvtune->e1));
          best[f] = std::min(best[f], t);
        }
      Pl.rsep_t[pi] = best[1] < best[0] ? 1 : 2;
    }
    if (Pl.rsep_t[pi] == 1)
      separate();
    else
      on_the_fly();
  }
}

// x = S b with the dense symmetric operator of level L (the coarsest
// inverse, or the dense tail)
template <typename T>
void dense_apply(DLevel& L, const T* b, T* x, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  {
    {
      // algorithmic: the stored half of the symmetric operator, x and y once
      PROF(kname("k_sym_gemv", tname<T>()), sizeof(T) * (L.n * (L.n + 1) / 2 + 2 * L.n), s);
      KLAUNCH((unsigned)((int64_t)L.nT * (L.nT + 1) / 2), dev::kBlock, 0, s, dev::k_sym_gemv<T>,
              L.n, L.nT, (const T*)P.Spk, b, P.spart);
      LAUNCH_OK();
    }
    PROF(kname("k_sym_reduce", tname<T>()),
         sizeof(T) * ((int64_t)L.nT * L.nT * dev::kTile + L.n), s);
    KLAUNCH((unsigned)L.nT * (dev::kTile / 16), dev::kBlock, 0, s, dev::k_sym_reduce<T>, L.n, L.nT,
            (const T*)P.spart, x);
    LAUNCH_OK();
  }
}

// x = B b on level l from a zero initial guess.  With finalize = false the
// RAS-T contributions of this level are left staged in tb: the caller (the
// finer level's prolongation) adds them when it reads x.
template <typename T>
void vcycle(lsamg_handle* h, size_t l, const T* b, T* x, hipStream_t s, bool finalize) {
  LevelTag tag_((int)l);
  DLevel& L = h->L[l];
  DPrec<T>& P = prec<T>(L);
  if (L.coarsest || L.tail) {
    dense_apply<T>(L, b, x, s);
    return;
  }
  DLevel& C = h->L[l + 1];
  DPrec<T>& PC = prec<T>(C);
  ras<T>(L, b, x, s);                                                        // eq:ras
  resid_first<T>(L, x, s);
  gemv_resid<T, false>(L, L.rst, P.Zh, b, PC.b, s);                          // P^T (b - A x)
  vcycle<T>(h, l + 1, PC.b, PC.x, s, false);
  if (C.coarsest || C.tail) {
    gemv<T, dev::IN_DIRECT, true>(L.pro, no_spec<T>(), P.ZhT, PC.x, x, s);
  } else {
    dev::InSpec<T> sp = no_spec<T>();
    sp.ptr = C.cptr;
    sp.pos = C.cpos;
    sp.v1 = PC.tb;
    gemv<T, dev::IN_TB, true>(L.pro, sp, P.ZhT, PC.x, x, s,
                              (int64_t)(sizeof(T) + 8) * C.ntb + 8 * (C.n + 1));
  }
  resid_first<T>(L, x, s);
  gemv_resid<T, false>(L, L.rast, P.Zr, b, P.tb, s);                         // eq:ras-t
  if (finalize) gather_add<T>(L, x, s);
}

// x = B b on level l by the additive method of sec. 3.1.1 made multilevel:
// the additive Schwarz smoother sum_i R_i^T A_i^{-1} R_i b (eq:ras without
// the partition of unity; its local results staged in tb, as RAS-T's are)
// plus P applied to the same cycle of P^T b on the next level, exact on the
// coarsest.  No residual is formed.  finalize as in vcycle.
template <typename T>
void acycle(lsamg_handle* h, size_t l, const T* b, T* x, hipStream_t s, bool finalize) {
  LevelTag tag_((int)l);
  DLevel& L = h->L[l];
  DPrec<T>& P = prec<T>(L);
  if (L.coarsest || L.tail) {
    dense_apply<T>(L, b, x, s);
    return;
  }
  if (!P.As) throw DevError{LSAMG_EINVAL, "the hierarchy was set up for the V-cycle"};
  DLevel& C = h->L[l + 1];
  DPrec<T>& PC = prec<T>(C);
  dev::InSpec<T> sg = no_spec<T>();
  sg.idx = L.oidx;
  gemv<T, dev::IN_GATHER, false>(L.as, sg, P.As, b, P.tb, s);                // A_i^{-1} b(Omega_i)
  gemv<T, dev::IN_DIRECT, false>(L.rst, no_spec<T>(), P.Zh, b, PC.b, s);     // P^T b
  acycle<T>(h, l + 1, PC.b, PC.x, s, false);
  if (C.coarsest || C.tail) {
    gemv<T, dev::IN_DIRECT, false>(L.pro, no_spec<T>(), P.ZhT, PC.x, x, s);  // x = P e
  } else {
    dev::InSpec<T> sp = no_spec<T>();
    sp.ptr = C.cptr;
    sp.pos = C.cpos;
    sp.v1 = PC.tb;
    gemv<T, dev::IN_TB, false>(L.pro, sp, P.ZhT, PC.x, x, s,
                               (int64_t)(sizeof(T) + 8) * C.ntb + 8 * (C.n + 1));
  }
  if (finalize) gather_add<T>(L, x, s);
}

// the handle's cycle (V or additive) on level 0
template <typename T>
void cycle(lsamg_handle* h, const T* b, T* x, hipStream_t s, bool finalize) {
  if (h->H.params.cycle == LSAMG_CYCLE_ADDITIVE)
    acycle<T>(h, 0, b, x, s, finalize);
  else
    vcycle<T>(h, 0, b, x, s, finalize);
}

// Run fn (which launches a fixed sequence of kernels on a stream: one
// V-cycle) on s.  With graphs on and no kernel timing active, the sequence is
// recorded once per key as a chain of kernel nodes of a HIP graph (no stream
// capture, so other threads' allocations and copies are unaffected) and
// replayed on s.  The launches' arguments are device addresses that stay
// fixed while the graph lives (batched graphs are dropped with the batched
// buffers); only kernels are recorded, no memset or copy.
template <typename F>
void run_graph(lsamg_handle* h, int key, hipStream_t s, F&& fn) {
  if (!h->use_graphs || prof_active()) {
    fn(s);
    return;
  }
  auto it = h->graphs.find(key);
  if (it == h->graphs.end()) {
    GraphRec rec;
    HIP_OK(hipGraphCreate(&rec.g, 0));
    struct Stop {
      GraphRec* r;
      ~Stop() {
        g_rec = nullptr;
        if (r->g) (void)hipGraphDestroy(r->g);
      }
    } stop{&rec};
    g_rec = &rec;
    fn(s);
    g_rec = nullptr;
    hipGraphExec_t ex = nullptr;
    HIP_OK(hipGraphInstantiate(&ex, rec.g, nullptr, nullptr, 0));
    it = h->graphs.emplace(key, ex).first;
  }
  HIP_OK(hipGraphLaunch(it->second, s));
}

// z = B r (FP64 in and out), in the handle's precision.
void precondition(lsamg_handle* h, const double* r, double* z, hipStream_t s) {
  DLevel& L0 = h->L[0];
  if (h->precision == LSAMG_MIXED) {
    {
      PROF("k_convert<double, float>", 12 * L0.n, s);
      KLAUNCH(nblocks(L0.n), dev::kBlock, 0, s, dev::k_convert<double, float>, L0.n, r, L0.f.b);
      LAUNCH_OK();
    }
    cycle<float>(h, L0.f.b, L0.f.x, s, true);
    {
      PROF("k_convert<float, double>", 12 * L0.n, s);
      KLAUNCH(nblocks(L0.n), dev::kBlock, 0, s, dev::k_convert<float, double>, L0.n, L0.f.x, z);
      LAUNCH_OK();
    }
  } else {
    cycle<double>(h, r, z, s, true);
  }
}

// y = A x = G^T (G x), FP64, finest level
void apply_A(lsamg_handle* h, const double* x, double* y, hipStream_t s) {
  DLevel& L = h->L[0];
  if (!L.g_ptr || !L.gt_ptr) throw DevError{LSAMG_EINVAL, "finest-level G missing on the device"};
  spmv_csr<double>(L.nrows, L.lanes_g, L.g_ptr, L.g_col, L.d.g_val, x, L.d.y, s, L.nnz, L.n);
  spmv_csr<double>(L.n, L.lanes_gt, L.gt_ptr, L.gt_col, L.d.gt_val, L.d.y, y, s, L.nnz,
                   L.nrows);
}

inline unsigned red_blocks(int64_t n) {
  return (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (n + dev::kBlock - 1) / dev::kBlock));
}

// partials of a . b into part (red_np of them)
void dot_parts(lsamg_handle* h, int64_t n, const double* a, const double* b, double* part,
               hipStream_t s) {
  PROF("k_dot", 16 * n + 8 * h->red_np, s);
  KLAUNCH(h->red_np, dev::kBlock, 0, s, dev::k_dot, n, a, b, part);
  LAUNCH_OK();
}

// queue a copy of red_np partials into pinned host slot (1024 doubles each)
void parts_to_host(lsamg_handle* h, const double* part, int slot, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(h->sc_host + (size_t)slot * 1024, part, h->red_np * sizeof(double),
                        hipMemcpyDeviceToHost, s));
}

double host_sum(const lsamg_handle* h, int slot) {
  double t = 0;
  for (int i = 0; i < h->red_np; ++i) t += h->sc_host[(size_t)slot * 1024 + i];
  return t;
}

struct ProfGuard {
  explicit ProfGuard(Profiler* p) { g_prof = p; }
  ~ProfGuard() { g_prof = nullptr; }
};

struct DeviceGuard {
  int old = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    HIP_OK(hipSetDevice(dev));
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

// q = A p (finest level, FP64) with sc[CG_PQ] = p . q fused into the G^T pass
void cg_apply(lsamg_handle* h, hipStream_t s) {
  DLevel& L = h->L[0];
  if (!L.g_ptr || !L.gt_ptr) throw DevError{LSAMG_EINVAL, "finest-level G missing on the device"};
  const int64_t n = L.n;
  if (h->dir_pending) {                 // p = z (+ beta p) and q = A p in one pass
    const double* rz_old = h->dir_pending == 2 ? h->dir_den : nullptr;
    PROF(kname("k_cg_tile", std::to_string(L.ata_me) + ", " + std::to_string(L.ata_mf)),
         8.0 * (3 * n + (h->dir_pending == 2 ? n : 0)) + 12.0 * L.nnz + 8.0 * L.nrows + 16 * h->red_np,
         s);
    const size_t lds = (size_t)(L.at1.umax + L.at1_rmax) * sizeof(double);
    auto launch = [&](auto kern) {
      KLAUNCH(h->red_np, dev::kBlock, lds, s, kern, n, L.at1, (const double*)L.trv1,
              (const double*)L.tdw1, h->dir_num, rz_old, (const double*)h->z,
              (const double*)h->p, h->p2, h->q, h->p_pq);
    };
    const int me = L.ata_me, mf = L.ata_mf;
    if (me == 6 && mf == 3)
      launch(dev::k_cg_tile<6, 3>);
    else if (me == 6)
      launch(dev::k_cg_tile<6, 4>);
    else if (me == 8 && mf == 3)
      launch(dev::k_cg_tile<8, 3>);
    else if (me == 8)
      launch(dev::k_cg_tile<8, 4>);
    else if (mf == 3)
      launch(dev::k_cg_tile<16, 3>);
    else
      launch(dev::k_cg_tile<16, 4>);
    LAUNCH_OK();
    std::swap(h->p, h->p2);
    h->dir_pending = 0;
    return;
  }
  spmv_csr<double>(L.nrows, L.lanes_g, L.g_ptr, L.g_col, L.d.g_val, h->p, L.d.y, s, L.nnz, n);
  const unsigned g = h->red_np;
  PROF(kname("k_cg_apq", std::to_string(L.lanes_gt)),
       12 * L.nnz + 8 * (n + 1) + 8 * L.nrows + 24 * n + 8 * g, s);
  switch (L.lanes_gt) {
#define CASE(LN)                                                                          \
  case LN:                                                                                \
    KLAUNCH(g, dev::kBlock, 0, s, dev::k_cg_apq<LN>, n, L.gt_ptr, L.gt_col, L.d.gt_val, L.d.y, \
                                                h->p, h->q, h->p_pq);                     \
    break;
    CASE(1) CASE(2) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64)
#undef CASE
  }
  LAUNCH_OK();
}

// z = B r from the residual h->r (and its FP32 copy in mixed mode), the
// partials of r . z into p_rz[cur], and p = z + beta p (p = z when first):
// beta = rho_new / rho_old from p_rz[cur] over p_rz[1-cur], or in flexible
// CG beta = -(z . q) / (p . q) with q = A p of the direction just used.
void cg_precondition(lsamg_handle* h, hipStream_t s, bool first, int cur) {
  DLevel& L0 = h->L[0];
  const int64_t n = L0.n;
  const unsigned g = h->red_np;
  const bool stage = !L0.coarsest;
  const bool fcg = h->krylov == LSAMG_KRYLOV_FCG;
  const double* qv = fcg && !first ? h->q : nullptr;
  h->dir_num = fcg ? h->p_zq : h->p_rz[cur];
  h->dir_den = fcg ? h->p_pqo : h->p_rz[1 - cur];
  if (h->precision == LSAMG_MIXED) {
    run_graph(h, 128 + 1, s, [&](hipStream_t gs) { cycle<float>(h, L0.f.b, L0.f.x, gs, false); });
    PROF("k_cg_z<float>",
         4 * n + (stage ? 12 * L0.ntb + 8 * (n + 1) : 0) + (qv ? 24 : 16) * n + 8 * g, s);
    KLAUNCH(g, dev::kBlock, 0, s, dev::k_cg_z<float>, n, L0.f.x, stage ? L0.cptr : nullptr, L0.cpos,
                                                 L0.f.tb, h->r, h->z, h->p_rz[cur], qv, h->p_zq);
  } else {
    run_graph(h, 1, s, [&](hipStream_t gs) { cycle<double>(h, h->r, L0.d.x, gs, false); });
    PROF("k_cg_z<double>",
         8 * n + (stage ? 16 * L0.ntb + 8 * (n + 1) : 0) + (qv ? 24 : 16) * n + 8 * g, s);
    KLAUNCH(g, dev::kBlock, 0, s, dev::k_cg_z<double>, n, L0.d.x, stage ? L0.cptr : nullptr, L0.cpos,
                                                  L0.d.tb, h->r, h->z, h->p_rz[cur], qv, h->p_zq);
  }
  LAUNCH_OK();
  if (L0.at1_on) {                      // applied by the next cg_apply (k_cg_tile)
    h->dir_pending = first ? 1 : 2;
    return;
  }
  PROF("k_cg_dir", 24 * n + 16 * g, s);
  KLAUNCH(g, dev::kBlock, 0, s, dev::k_cg_dir, n, h->dir_num, first ? nullptr : h->dir_den, h->z,
                                          h->p);
  LAUNCH_OK();
}

// One PCG solve of a single right-hand side (device vectors in user
// numbering).  The host learns ||r_k|| through a pinned copy recorded after
// the update of iteration k; while it waits, the V-cycle of iteration k is
// already queued, so the GPU never idles on the stop test.  Only when the
// residual history predicts convergence within the next iteration does the
// host wait before queueing the V-cycle (which would otherwise be wasted).
// One eager V-cycle on the current level-0 input with GEMV autotuning on
// (first solve of each precision); its output is overwritten by the solve.
void gv_tune(lsamg_handle* h, hipStream_t s) {
  const bool mixed = h->precision == LSAMG_MIXED;
  const int pi = mixed ? 1 : 0;
  if (h->gv_tuned[pi] || h->L.empty()) return;
  int64_t mx = 1;
  for (auto& D : h->L)
    for (const GemvPlan* P : {&D.ras, &D.rast, &D.rst, &D.pro, &D.as}) mx = std::max(mx, P->out);
  struct Ctx {
    GvTune t;
    Profiler* saved = g_prof;
    ~Ctx() {
      g_gvtune = nullptr;
      g_prof = saved;
      if (t.scratch) (void)hipFree(t.scratch);
      if (t.e0) (void)hipEventDestroy(t.e0);
      if (t.e1) (void)hipEventDestroy(t.e1);
    }
  } c;
  HIP_OK(hipMalloc(&c.t.scratch, (size_t)mx * sizeof(double)));
  HIP_OK(hipEventCreate(&c.t.e0));
  HIP_OK(hipEventCreate(&c.t.e1));
  g_prof = nullptr;                     // tuning launches are not profiled
  g_gvtune = &c.t;
  DLevel& L0 = h->L[0];
  if (mixed)
    cycle<float>(h, L0.f.b, L0.f.x, s, false);
  else
    cycle<double>(h, h->r, L0.d.x, s, false);
  HIP_OK(hipStreamSynchronize(s));
  h->gv_tuned[pi] = true;
}

// ||b - A x||_2 in FP64 (the true residual, left in h->z; q is overwritten)
double true_residual(lsamg_handle* h, hipStream_t s) {
  const int64_t n = h->L[0].n;
  const unsigned gb = nblocks(n);
  apply_A(h, h->x, h->q, s);
  KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_sub, n, h->bi, h->q, h->z);
  LAUNCH_OK();
  dot_parts(h, n, h->z, h->z, h->p_tmp, s);
  parts_to_host(h, h->p_tmp, 0, s);
  HIP_OK(hipStreamSynchronize(s));
  return std::sqrt(host_sum(h, 0));
}

// Stop test: the recurrence residual ||r_k|| <= tol ||b|| and then the true
// residual ||b - A x_k|| <= tol ||b||, both in FP64.  When only the first
// holds, r is replaced by the true residual and CG restarts from x_k with
// p = z (in FP32 V-cycle mode the two residuals part by the preconditioner's
// rounding, so a reported convergence is always one of b - A x).
int pcg_one(lsamg_handle* h, const double* b, double* x, double tol, int maxit, hipStream_t s,
            lsamg_stats* st) {
  auto t0 = std::chrono::steady_clock::now();
  DLevel& L0 = h->L[0];
  const int64_t n = L0.n;
  const unsigned gb = nblocks(n);
  KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_perm_in, n, h->perm, b, h->bi);
  LAUNCH_OK();
  KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_fill, n, 0.0, h->x);
  LAUNCH_OK();
  KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_copy, n, h->bi, h->r);
  LAUNCH_OK();
  dot_parts(h, n, h->bi, h->bi, h->p_tmp, s);
  parts_to_host(h, h->p_tmp, 0, s);
  HIP_OK(hipStreamSynchronize(s));
  const double nb2 = host_sum(h, 0);
  if (!std::isfinite(nb2)) throw DevError{LSAMG_EBADINPUT, "non-finite entry in the right-hand side"};
  const double nb = std::sqrt(nb2);
  const bool mixed = h->precision == LSAMG_MIXED;
  int its = 0, restarts = 0;
  double rn = nb, rprev = nb, fac = 0.5, tr = -1.0;
  bool conv = (nb == 0.0);
  if (!conv && maxit > 0) {
    if (mixed) {
      KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_convert<double, float>, n, h->r, L0.f.b);
      LAUNCH_OK();
    }
    gv_tune(h, s);
    h->dir_pending = 0;
    int cur = 0;                        // p_rz[cur] holds rho of the current direction
    cg_precondition(h, s, true, cur);
    const double target = tol * nb;
    while (its < maxit) {
      cg_apply(h, s);
      {
        PROF("k_cg_update", (mixed ? 60 : 56) * n + 24 * h->red_np, s);
        KLAUNCH(h->red_np, dev::kBlock, 0, s, dev::k_cg_update, n, h->p_rz[cur], h->p_pq, h->p, h->q,
                                                          h->x, h->r, mixed ? L0.f.b : nullptr,
                                                          h->p_rr,
                                                          h->krylov == LSAMG_KRYLOV_FCG ? h->p_pqo
                                                                                        : nullptr);
        LAUNCH_OK();
      }
      const int slot = 1 + (its & 1);
      parts_to_host(h, h->p_rr, slot, s);
      HIP_OK(hipEventRecord(h->ev_rr[its & 1], s));
      ++its;
      // predicted residual after this update, from the average reduction so far
      const bool near = rprev * fac <= 2.0 * target || its >= maxit;
      if (!near) cg_precondition(h, s, false, 1 - cur);
      HIP_OK(hipEventSynchronize(h->ev_rr[(its - 1) & 1]));
      rn = std::sqrt(host_sum(h, slot));
      if (!std::isfinite(rn)) throw DevError{LSAMG_ENOTSPD, "CG breakdown (non-finite residual)"};
      fac = std::pow(rn / nb, 1.0 / its);
      rprev = rn;
      bool restart = false;
      if (rn <= target) {
        tr = true_residual(h, s);
        if (tr <= target) {
          conv = true;
          break;
        }
        // replace r by b - A x (left in z) and restart with p = z
        KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_copy, n, h->z, h->r);
        LAUNCH_OK();
        if (mixed) {
          KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_convert<double, float>, n, h->r, L0.f.b);
          LAUNCH_OK();
        }
        rn = rprev = tr;
        tr = -1.0;
        restart = true;
        ++restarts;
      }
      if (its >= maxit) break;
      if (near || restart) cg_precondition(h, s, restart, 1 - cur);
      cur = 1 - cur;
    }
  }
  if (tr < 0.0) tr = true_residual(h, s);
  KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_perm_out, n, h->perm, h->x, x);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  if (st) {
    st->iters = its;
    st->converged = conv ? 1 : 0;
    st->rel_res = nb > 0 ? rn / nb : 0.0;
    st->true_rel_res = nb > 0 ? tr / nb : 0.0;
    st->rho = (its > 0 && nb > 0) ? std::pow(rn / nb, 1.0 / its) : 0.0;
    st->restarts = restarts;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return conv ? LSAMG_OK : LSAMG_ENOCONV;
}

// ===========================================================================
// Multi-right-hand-side path
// ===========================================================================
constexpr int kBNP = 8192;     // workgroups (and partials per column) of the batched CG kernels
constexpr int kBMax = 64;      // widest batch

void ensure_batched(lsamg_handle* h, int NB) {
  if (h->batched_ready && h->bwidth >= NB) return;
  h->free_batched();
  h->batched_ready = false;
  h->batch_alloc = true;
  struct Reset {
    lsamg_handle* h;
    ~Reset() { h->batch_alloc = false; }
  } reset{h};
  for (auto& L : h->L)            // the batched kernels index rows with 32-bit wave-uniform values
    if (L.n >= ((int64_t)1 << 31) || L.nrows >= ((int64_t)1 << 31))
      throw DevError{LSAMG_EINVAL, "level too large for the multi-right-hand-side path"};
  h->bwidth = NB;
  const int W = NB;                // buffers sized for this width
  h->BL.assign(h->L.size(), lsamg_handle::BLev{});
  for (size_t l = 0; l < h->L.size(); ++l) {
    DLevel& L = h->L[l];
    auto& B = h->BL[l];
    const size_t n = (size_t)L.n * W, ny = (size_t)std::max<int64_t>(L.nrows, 1) * W,
                 nt = (size_t)std::max<int64_t>(L.ntb, 1) * W;
    B.x = h->alloc<double>(n);
    B.b = h->alloc<double>(n);
    B.r = h->alloc<double>(n);
    B.y = h->alloc<double>(ny);
    B.tb = h->alloc<double>(nt);
    B.fx = h->alloc<float>(n);
    B.fb = h->alloc<float>(n);
    B.fr = h->alloc<float>(n);
    B.fy = h->alloc<float>(ny);
    B.ftb = h->alloc<float>(nt);
    if (L.bg_ok) B.fstg = h->alloc<float>((size_t)L.bg_nstg * W);
  }
  const size_t n0 = (size_t)h->L[0].n * W;
  h->BX = h->alloc<double>(n0);
  h->BR = h->alloc<double>(n0);
  h->BZ = h->alloc<double>(n0);
  h->BP = h->alloc<double>(n0);
  h->BQ = h->alloc<double>(n0);
  h->BBi = h->alloc<double>(n0);
  h->Bpq = h->alloc<double>(kBNP * W);
  h->Brr = h->alloc<double>(kBNP * W);
  h->Brz[0] = h->alloc<double>(kBNP * W);
  h->Brz[1] = h->alloc<double>(kBNP * W);
  h->Btmp = h->alloc<double>(kBNP * W);
  h->Bzq = h->alloc<double>(kBNP * W);
  h->Bpq_s = h->alloc<double>(W);
  h->Brr_s = h->alloc<double>(W);
  h->Brz_s[0] = h->alloc<double>(W);
  h->Brz_s[1] = h->alloc<double>(W);
  h->Btmp_s = h->alloc<double>(W);
  h->Bzq_s = h->alloc<double>(W);
  h->Bactive = h->alloc<int>(3 * 64);   // active, restart and new-direction flags, 64 columns
  if (!h->Bactive_host)
    HIP_OK(hipHostMalloc((void**)&h->Bactive_host, 3 * 64 * sizeof(int), hipHostMallocDefault));
  if (!h->Bparts_host)
    HIP_OK(hipHostMalloc((void**)&h->Bparts_host, 3 * 64 * sizeof(double),
                         hipHostMallocDefault));
  h->batched_ready = true;
}

template <typename T>
struct BVec {
  T *x, *b, *r, *y, *tb;
  T* stg;                 // k_bgrp_ata64 staging (FP32 only)
};
template <typename T>
BVec<T> bvec(lsamg_handle::BLev& B);
template <>
BVec<double> bvec<double>(lsamg_handle::BLev& B) { return {B.x, B.b, B.r, B.y, B.tb, nullptr}; }
template <>
BVec<float> bvec<float>(lsamg_handle::BLev& B) { return {B.fx, B.fb, B.fr, B.fy, B.ftb, B.fstg}; }

// Task list of k_bmm for RT row tiles per task and a loop split S (single-
// aggregate operators only).  Tasks are ordered by loop length, longest
// first, in power-of-two size buckets (aggregate order inside a bucket), so
// the persistent launch starts the longest tasks first.  tmp: allocate with
// hipMalloc (a tuning candidate, freed by mm_free) instead of the handle.
GemvPlan::Mm mm_build(lsamg_handle* h, const GemvPlan& P, int RT, int S, bool tmp) {
  struct Task {
    int32_t a, j0, k0, k1, slot, bucket;
  };
  std::vector<Task> ts;
  // a split cuts every aggregate's loop into S ranges of a multiple of 8
  // (trailing ranges may be empty): slot q of every output row is written by
  // exactly one task
  const int sn = std::max(1, S);
  int used_split = 1;
  if (sn > 1 && P.nagg == 1) {        // a single aggregate: no empty ranges
    const int K = P.hll[0];
    const int kc = std::max(8, ((K + sn - 1) / sn + 7) / 8 * 8);
    used_split = std::max(1, (K + kc - 1) / kc);
  } else if (sn > 1) {
    used_split = sn;
  }
  for (int64_t a = 0; a < P.nagg; ++a) {
    const int nj = P.hlj[a], K = P.hll[a];
    const int kc = std::max(8, ((K + used_split - 1) / used_split + 7) / 8 * 8);
    const int ns = used_split;
    for (int j0 = 0; j0 < nj; j0 += 16 * RT)
      for (int q = 0; q < ns; ++q) {
        const int k0 = ns > 1 ? std::min(K, q * kc) : 0, k1 = ns > 1 ? std::min(K, (q + 1) * kc) : K;
        int b = 0;
        while ((1 << b) < k1 - k0) ++b;
        ts.push_back(Task{(int32_t)a, j0, k0, k1, ns > 1 ? q : -1, b});
      }
  }
  std::stable_sort(ts.begin(), ts.end(),
                   [](const Task& x, const Task& y) { return x.bucket > y.bucket; });
  std::vector<int32_t> v[5];
  for (auto& t : ts) {
    v[0].push_back(t.a);
    v[1].push_back(t.j0);
    v[2].push_back(t.k0);
    v[3].push_back(t.k1);
    v[4].push_back(t.slot);
  }
  GemvPlan::Mm mm;
  mm.rt = RT;
  mm.split = used_split;
  mm.ntask = (int64_t)ts.size();
  // persistent launch: at most 8 workgroups of 4 wavefronts per compute unit
  mm.grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((mm.ntask + 3) / 4, 256 * 8));
  int32_t* d[5];
  for (int c = 0; c < 5; ++c) {
    if (tmp) {
      HIP_OK(hipMalloc((void**)&d[c], std::max<size_t>(1, v[c].size()) * sizeof(int32_t)));
      if (!v[c].empty())
        HIP_OK(hipMemcpy(d[c], v[c].data(), v[c].size() * sizeof(int32_t), hipMemcpyHostToDevice));
    } else {
      d[c] = h->upload(v[c]);
    }
  }
  mm.tk = dev::MmTasks{d[0], d[1], d[2], d[3], d[4]};
  return mm;
}

void mm_free(GemvPlan::Mm& mm) {
  for (const int32_t* p : {mm.tk.a, mm.tk.j0, mm.tk.k0, mm.tk.k1, mm.tk.slot})
    if (p) (void)hipFree((void*)p);
  mm.tk = dev::MmTasks{};
}

template <int MODE, bool ADD, int NB>
void bmm_launch(const GemvPlan& P, const GemvPlan::Mm& mm, const int32_t* gidx,
                const int64_t* cptr, const int64_t* cpos, const float* tb, const float* M,
                const float* in, float* out, hipStream_t s, double bytes) {
  const bool split = mm.split > 1;
  if (!split_fits(mm.split, P.out, NB, mm.part, mm.part_cap))
    throw DevError{LSAMG_EINVAL, "matrix-core launch: the loop split's partial sums (" +
                                     std::to_string(mm.split) + " x " + std::to_string(P.out) +
                                     " x " + std::to_string(NB) + ") exceed their buffer"};
  bool done = false;
  if constexpr (NB == 64) {
    if (mm.lds) {
      PROF_F(kname("k_bmm_lds", std::to_string(MODE) + ", " + (ADD ? "true" : "false")),
             split ? bytes - sizeof(float) * (double)P.out * NB : bytes, 2.0 * (double)P.mat * NB,
             s);
      KLAUNCH((unsigned)mm.ntask, dev::kBlock, 0, s, dev::k_bmm_lds<MODE, ADD>, mm.tk, P.op, gidx,
              cptr, cpos, tb, M, in, split ? mm.part : out, mm.part, (int64_t)P.out);
      LAUNCH_OK();
      done = true;
    }
  }
  if (!done) {
    PROF_F(kname("k_bmm", std::to_string(MODE) + ", " + (ADD ? "true" : "false") + ", " +
                              std::to_string(mm.rt) + ", " + std::to_string(mm.u) + ", " +
                              std::to_string(NB)),
           split ? bytes - sizeof(float) * (double)P.out * NB : bytes, 2.0 * (double)P.mat * NB,
           s);
    auto launch = [&](auto kern) {
      KLAUNCH(mm.grid, dev::kBlock, 0, s, kern, mm.tk, (int)mm.ntask, P.op, gidx, cptr, cpos, tb, M,
              in, split ? mm.part : out, mm.part, (int64_t)P.out);
    };
    if (mm.u == 2) {
      if (mm.rt == 1)
        launch(dev::k_bmm<MODE, ADD, 1, 2, NB>);
      else if (mm.rt == 2)
        launch(dev::k_bmm<MODE, ADD, 2, 2, NB>);
      else
        launch(dev::k_bmm<MODE, ADD, 4, 2, NB>);
    } else {
      if (mm.rt == 1)
        launch(dev::k_bmm<MODE, ADD, 1, 8, NB>);
      else if (mm.rt == 2)
        launch(dev::k_bmm<MODE, ADD, 2, 8, NB>);
      else
        launch(dev::k_bmm<MODE, ADD, 4, 8, NB>);
    }
    LAUNCH_OK();
  }
  if (split) {
    PROF(kname("k_bmm_reduce", std::string(ADD ? "true" : "false") + ", " + std::to_string(NB)),
         sizeof(float) * (double)P.out * NB * (mm.split + (ADD ? 2 : 1)), s);
    KLAUNCH(nblocks(P.out * NB), dev::kBlock, 0, s, dev::k_bmm_reduce<ADD, NB>, (int64_t)P.out,
            mm.split, (const float*)mm.part, out);
    LAUNCH_OK();
  }
}

template <typename T, int MODE, bool ADD, int NB>
void bgemm(const GemvPlan& P, const int32_t* gidx, const int64_t* cptr, const int64_t* cpos,
           const T* tb, const T* M, const T* in, T* out, hipStream_t s, int64_t tb_extra = 0) {
  const double bytes = sizeof(T) * (P.mat + (P.in_u + P.out * (ADD ? 2 : 1)) * NB) + 4 * P.idx +
                       32 * P.nagg + tb_extra * NB;
  if constexpr (std::is_same<T, float>::value && NB >= 16) {
    if (P.mm.rt > 0) {
      bmm_launch<MODE, ADD, NB>(P, P.mm, gidx, cptr, cpos, tb, M, in, out, s, bytes);
      return;
    }
  }
  if constexpr (std::is_same<T, double>::value && NB >= 16) {
    if (NB == 64 && P.mmd.rt > 0 && P.mmd.lds) {
      const GemvPlan::Mm& mm = P.mmd;
      PROF_F(kname("k_bmmd_lds", std::to_string(MODE) + ", " + (ADD ? "true" : "false")), bytes,
             2.0 * (double)P.mat * NB, s);
      KLAUNCH((unsigned)mm.ntask, dev::kBlock, 0, s, dev::k_bmmd_lds<MODE, ADD>, mm.tk, P.op, gidx,
              cptr, cpos, tb, M, in, out);
      LAUNCH_OK();
      return;
    }
    if (P.mmd.rt > 0) {
      const GemvPlan::Mm& mm = P.mmd;
      PROF_F(kname("k_bmmd", std::to_string(MODE) + ", " + (ADD ? "true" : "false") + ", " +
                                 std::to_string(mm.rt) + ", " + std::to_string(mm.u) + ", " +
                                 std::to_string(NB)),
             bytes, 2.0 * (double)P.mat * NB, s);
      auto launch = [&](auto kern) {
        KLAUNCH(mm.grid, dev::kBlock, 0, s, kern, mm.tk, (int)mm.ntask, P.op, gidx, cptr, cpos,
                tb, M, in, out);
      };
      if (mm.rt == 4)
        launch(dev::k_bmmd<MODE, ADD, 4, 2, NB>);
      else if (mm.rt == 2 && mm.u == 8)
        launch(dev::k_bmmd<MODE, ADD, 2, 8, NB>);
      else if (mm.rt == 2)
        launch(dev::k_bmmd<MODE, ADD, 2, 2, NB>);
      else if (mm.u == 8)
        launch(dev::k_bmmd<MODE, ADD, 1, 8, NB>);
      else
        launch(dev::k_bmmd<MODE, ADD, 1, 2, NB>);
      LAUNCH_OK();
      return;
    }
  }
  PROF_F(kname("k_bgemm", std::string(tname<T>()) + ", " + std::to_string(MODE) + ", " +
                              (ADD ? "true" : "false") + ", " + std::to_string(NB)),
         bytes, 2.0 * (double)P.mat * NB, s);
  KLAUNCH((unsigned)P.ntask, dev::kBlock, 0, s, dev::k_bgemm<T, MODE, ADD, NB>, P.task_a,
          P.task_j0, P.op, gidx, cptr, cpos, tb, M, in, out);
  LAUNCH_OK();
}

// Autotuner of the matrix-core batched GEMM: every candidate tile shape (row
// tiles per task, loads in flight, loop split, and on 64 columns the
// LDS-staged form) is timed on the operator's own matrices and buffers (one
// warm-up and three timed launches, each after evicting the last-level
// cache), and the fastest is kept.
template <int MODE, bool ADD, int NB>
float mm_tune(lsamg_handle* h, GemvPlan& P, const int32_t* gidx, const int64_t* cptr,
             const int64_t* cpos, const float* tb, const float* M, const float* in, float* out,
             float* part, int64_t part_cap, hipStream_t s, double* flush, int64_t flush_n) {
  if (P.nagg == 0 || P.hlj.empty()) return 0.f;
  const int ljmax = *std::max_element(P.hlj.begin(), P.hlj.end());
  const int llmax = *std::max_element(P.hll.begin(), P.hll.end());
  struct Cand {
    int rt, u, sp;
    bool lds;
  };
  std::vector<Cand> cand;
  if (h->mm_fixed > 0) {               // a fixed tile shape (LSAMG_OPT_MFMA_TILE)
    const int rt = h->mm_fixed / 100;
    int u = (h->mm_fixed / 10) % 10;
    int sp = h->mm_fixed % 10;
    if ((int64_t)sp * P.out * std::max<int64_t>(NB, h->bwidth) > part_cap) sp = 1;
    const bool lds = u == 0 && NB == 64;  // u = 0: the LDS-staged form (64 columns)
    if (u == 0) u = 2;
    cand.push_back(Cand{rt, u, sp, lds});
  }
  const bool fixed = !cand.empty();
  for (int rt : {1, 2, 4}) {
    if (fixed) break;                                     // the shape is given
    if (rt > 1 && 16 * (rt / 2) >= ljmax) continue;      // the tile would be mostly empty
    for (int u : {2, 8}) {
      if (u == 8 && llmax <= 32) continue;                // a few steps cover the loop
      for (int sp : {1, 2, 4, 8, 16}) {
        if (sp > 1 && (llmax / sp < (P.nagg == 1 ? 256 : 64) || (P.nagg > 1 && sp > 4))) continue;
        if ((int64_t)sp * P.out * std::max<int64_t>(NB, h->bwidth) > part_cap) continue;
        cand.push_back(Cand{rt, u, sp, false});
        // the LDS-staged form on 64 columns: 64-row tasks, same loop splits
        if (NB == 64 && rt == 4 && u == 2) cand.push_back(Cand{4, 2, sp, true});
      }
    }
  }
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float best = 1e30f;
  Cand pick{1, 2, 1, false};
  for (auto c : cand) {
    GemvPlan::Mm mm = mm_build(h, P, c.rt, c.sp, true);
    mm.u = c.u;
    mm.lds = c.lds;
    mm.part = part;
    mm.part_cap = part_cap;
    float ms = 1e30f;
    try {
      bmm_launch<MODE, ADD, NB>(P, mm, gidx, cptr, cpos, tb, M, in, out, s, 0.0);
      for (int round = 0; round < 1; ++round) {   // three launches after the warm-up
        float tot = 0.f;
        for (int r = 0; r < 3; ++r) {
          // in a V-cycle the operator's matrix arrives from HBM, not from the
          // last-level cache: evict it first when a flush buffer is given
          if (flush)
            KLAUNCH0(nblocks(flush_n), dev::kBlock, 0, s, dev::k_fill, flush_n, 0.0, flush);
          HIP_OK(hipEventRecord(e0, s));
          bmm_launch<MODE, ADD, NB>(P, mm, gidx, cptr, cpos, tb, M, in, out, s, 0.0);
          HIP_OK(hipEventRecord(e1, s));
          HIP_OK(hipEventSynchronize(e1));
          float t = 0.f;
          HIP_OK(hipEventElapsedTime(&t, e0, e1));
          tot += t;
        }
        ms = std::min(ms, tot);
      }
    } catch (...) {
      mm_free(mm);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    mm_free(mm);
    if (ms < best) {
      best = ms;
      pick = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P.mm = mm_build(h, P, pick.rt, pick.sp, false);
  P.mm.u = pick.u;
  P.mm.lds = pick.lds;
  P.mm.part = part;
  P.mm.part_cap = part_cap;
  return best;
}

// The dense level operator on 64 columns as the LDS-staged GEMM
// k_dense_mm64<KC> on the padded row-major copy L.dmm_M, with S loop ranges
// of kchunk rows (S > 1: partial sums in part, then k_bmm_reduce in slot
// order).
void dense_mm_launch(const DLevel& L, int S, int kchunk, int KC, const float* in, float* out,
                     float* part, int64_t part_cap, hipStream_t s) {
  const int64_t n = L.n;
  if (!split_fits(S, n, 64, part, part_cap))
    throw DevError{LSAMG_EINVAL, "dense-level launch: " + std::to_string(S) +
                                     " loop ranges exceed the partial-sum buffer"};
  {
    PROF_F("k_dense_mm64",
           sizeof(float) * ((double)n * n + (double)n * 64 * (1 + (S > 1 ? S : 1))),
           2.0 * (double)n * n * 64, s);
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)S);
    if (KC == 64)
      KLAUNCH(grid, dev::kBlock, 0, s, dev::k_dense_mm64<64>, n, L.dmm_ld, kchunk,
              (const float*)L.dmm_M, in, out, part);
    else
      KLAUNCH(grid, dev::kBlock, 0, s, dev::k_dense_mm64<32>, n, L.dmm_ld, kchunk,
              (const float*)L.dmm_M, in, out, part);
    LAUNCH_OK();
  }
  if (S > 1) {
    PROF(kname("k_bmm_reduce", "false, 64"), sizeof(float) * (double)n * 64 * (S + 1), s);
    KLAUNCH(nblocks(n * 64), dev::kBlock, 0, s, dev::k_bmm_reduce<false, 64>, n, S,
            (const float*)part, out);
    LAUNCH_OK();
  }
}

// Loop ranges of k_dense_mm64: kchunk rows (a multiple of its KC-row chunk)
// per range, and the number of ranges that covers n rows.
void dense_split_shape(int64_t n, int want, int KC, int* S, int* kchunk) {
  int64_t kc = (n + want - 1) / want;
  kc = (kc + KC - 1) / KC * KC;
  *kchunk = (int)std::max<int64_t>(KC, kc);
  *S = (int)((n + *kchunk - 1) / *kchunk);
}

// Autotuner of the dense level on 64 columns: k_dense_mm64 for both chunk
// lengths and each loop split that fits the partial-sum buffer, timed as
// mm_tune times k_bmm; kept if faster than the k_bmm tile shape already
// chosen (time bmm_ms), or always when the split is fixed.  Makes the padded
// row-major copy of the operator (with the multi-right-hand-side buffers).
void dense_tune(lsamg_handle* h, DLevel& L, const float* M, const float* in, float* out,
                float* part, int64_t part_cap, hipStream_t s, double* flush, int64_t flush_n,
                float bmm_ms) {
  L.dmm_split = 0;
  if (h->dense_split > 16 || (h->dense_split == 0 && h->mm_fixed > 0)) return;
  const int64_t n = L.n;
  if (!L.dmm_M) {
    L.dmm_ld = (n + 3) / 4 * 4;
    L.dmm_M = h->alloc<float>((size_t)(n * L.dmm_ld));
    KLAUNCH0(nblocks(n * L.dmm_ld), dev::kBlock, 0, s, dev::k_pad_rows<float>, n, L.dmm_ld, M, L.dmm_M);
    LAUNCH_OK();
  }
  std::vector<int> want;
  if (h->dense_split > 0)
    want.push_back(h->dense_split);
  else
    want = {1, 2, 3, 4, 6, 8, 9, 12, 16};
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float best = h->dense_split > 0 ? 1e30f : bmm_ms;
  try {
    for (int KC : {32, 64}) {
      for (int w : want) {
        int S = 1, kc = 0;
        dense_split_shape(n, w, KC, &S, &kc);
        while (S > 1 && (int64_t)S * n * 64 > part_cap) dense_split_shape(n, S - 1, KC, &S, &kc);
        if (S > 1 && !part) dense_split_shape(n, 1, KC, &S, &kc);
        dense_mm_launch(L, S, kc, KC, in, out, part, part_cap, s);
        float ms = 1e30f;
        for (int round = 0; round < 1; ++round) {   // three launches after the warm-up
          float tot = 0.f;
          for (int r = 0; r < 3; ++r) {
            if (flush)
              KLAUNCH0(nblocks(flush_n), dev::kBlock, 0, s, dev::k_fill, flush_n, 0.0, flush);
            HIP_OK(hipEventRecord(e0, s));
            dense_mm_launch(L, S, kc, KC, in, out, part, part_cap, s);
            HIP_OK(hipEventRecord(e1, s));
            HIP_OK(hipEventSynchronize(e1));
            float t = 0.f;
            HIP_OK(hipEventElapsedTime(&t, e0, e1));
            tot += t;
          }
          ms = std::min(ms, tot);
        }
        if (ms < best) {
          best = ms;
          L.dmm_split = S;
          L.dmm_kchunk = kc;
          L.dmm_kc = KC;
        }
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// The FP64 dense level operator on 64 columns as k_dense_mm64d<KC> on the
// padded row-major copy L.dmmd_M, with S loop ranges of kchunk rows (S > 1:
// partial sums in L.dmmd_part, then k_dense_reduce64d in slot order).
void dense_mm_launch_d(const DLevel& L, int S, int kchunk, int KC, const double* in, double* out,
                       hipStream_t s) {
  const int64_t n = L.n;
  if (!split_fits(S, n, 64, L.dmmd_part, L.dmmd_part_cap))
    throw DevError{LSAMG_EINVAL, "FP64 dense-level launch: " + std::to_string(S) +
                                     " loop ranges exceed the partial-sum buffer"};
  {
    PROF_F("k_dense_mm64d",
           sizeof(double) * ((double)n * n + (double)n * 64 * (1 + (S > 1 ? S : 1))),
           2.0 * (double)n * n * 64, s);
    const dim3 grid((unsigned)((n + 63) / 64), (unsigned)S);
    if (KC == 32)
      KLAUNCH(grid, dev::kBlock, 0, s, dev::k_dense_mm64d<32>, n, L.dmm_ld, kchunk,
              (const double*)L.dmmd_M, in, out, L.dmmd_part);
    else
      KLAUNCH(grid, dev::kBlock, 0, s, dev::k_dense_mm64d<16>, n, L.dmm_ld, kchunk,
              (const double*)L.dmmd_M, in, out, L.dmmd_part);
    LAUNCH_OK();
  }
  if (S > 1) {
    PROF("k_dense_reduce64d", sizeof(double) * (double)n * 64 * (S + 1), s);
    KLAUNCH(nblocks(n * 64), dev::kBlock, 0, s, dev::k_dense_reduce64d, n, S,
            (const double*)L.dmmd_part, out);
    LAUNCH_OK();
  }
}

// Time run() (a fixed sequence of launches on s): one warm-up, then three
// runs between two events; milliseconds for the three.
template <typename F>
float time_runs(hipStream_t s, F&& run) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  float t = 0.f;
  try {
    run();
    HIP_OK(hipEventRecord(e0, s));
    for (int r = 0; r < 3; ++r) run();
    HIP_OK(hipEventRecord(e1, s));
    HIP_OK(hipEventSynchronize(e1));
    HIP_OK(hipEventElapsedTime(&t, e0, e1));
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return t;
}

// One FP64 aggregate-block operator on the matrix cores: the FMA k_bgemm
// against k_bmmd (tasks of 1, 2 or 4 row tiles of 16; 2 or 8 loop steps'
// loads together, 2 with 4 row tiles) and the LDS-staged k_bmmd_lds (64-row
// tasks), timed on the level's own matrices and buffers; the fastest is kept
// in P.mmd (task lists live with the batched buffers).
template <int MODE, bool ADD>
void mmd_tune(lsamg_handle* h, GemvPlan& P, const int32_t* gidx, const int64_t* cptr,
              const int64_t* cpos, const double* tb, const double* M, const double* in,
              double* out, hipStream_t s) {
  P.mmd = GemvPlan::Mm{};
  if (P.nagg == 0 || P.hlj.empty()) return;
  if (h->mm_fixed > 0) {              // a fixed tile shape: its row tiles and loads in flight
    const int rt = h->mm_fixed / 100, u = (h->mm_fixed / 10) % 10;
    const bool lds = u == 0;           // u = 0: the LDS-staged form, 64-row tasks
    P.mmd = mm_build(h, P, lds ? 4 : rt, 1, false);
    P.mmd.u = u == 8 && rt < 4 ? 8 : 2;
    P.mmd.lds = lds;
    return;
  }
  auto run = [&] { bgemm<double, MODE, ADD, 64>(P, gidx, cptr, cpos, tb, M, in, out, s); };
  float best = time_runs(s, run);
  const int llmax = *std::max_element(P.hll.begin(), P.hll.end());
  GemvPlan::Mm pick{};                 // rt 0: k_bgemm
  for (int rt : {1, 2, 4}) {
    const GemvPlan::Mm mm = mm_build(h, P, rt, 1, false);
    for (int u : {2, 8}) {
      if (u == 8 && (llmax <= 32 || rt == 4)) continue;
      P.mmd = mm;
      P.mmd.u = u;
      const float t = time_runs(s, run);
      if (t < best) {
        best = t;
        pick = P.mmd;
      }
    }
    if (rt == 4) {                     // the same tasks, staged through LDS
      P.mmd = mm;
      P.mmd.lds = true;
      const float t = time_runs(s, run);
      if (t < best) {
        best = t;
        pick = P.mmd;
      }
    }
  }
  P.mmd = pick;
}

// FP64 forms on the matrix cores, chosen by the first FP64 batch of 64: each
// level's aggregate-block operators (mmd_tune) and the dense level
// (k_dense_mm64d for both chunk lengths and loop splits 1..16, or the split
// LSAMG_OPT_DENSE_SPLIT fixes, against the FMA k_bgemm), each timed on the
// level's own buffers (one warm-up and three timed launches; the FP64
// dense matrix exceeds the last-level cache, so nothing is evicted between
// them); the fastest is kept.  Makes the dense level's padded row-major FP64
// copy and partial-sum buffer with the batched buffers.
void fp64_tune(lsamg_handle* h, hipStream_t s) {
  if (h->dmmd_tuned || h->dry) return;
  struct Quiet {                       // tuning launches are not profiled
    Profiler* p;
    lsamg_handle* h;
    ~Quiet() {
      g_prof = p;
      h->batch_alloc = false;
    }
  } quiet{g_prof, h};
  g_prof = nullptr;
  h->batch_alloc = true;
  for (size_t l = 0; l < h->L.size(); ++l) {
    DLevel& L = h->L[l];
    auto& B = h->BL[l];
    if (!(L.coarsest || L.tail)) {
      DLevel& C = h->L[l + 1];
      auto& BC = h->BL[l + 1];
      mmd_tune<dev::IN_GATHER, false>(h, L.ras, L.oidx, nullptr, nullptr, nullptr, L.d.Zc, B.b,
                                      B.x, s);
      mmd_tune<dev::IN_DIRECT, false>(h, L.rst, nullptr, nullptr, nullptr, nullptr, L.d.Zh, B.r,
                                      BC.b, s);
      if (C.coarsest || C.tail)
        mmd_tune<dev::IN_DIRECT, true>(h, L.pro, nullptr, nullptr, nullptr, nullptr, L.d.ZhT,
                                       BC.x, B.x, s);
      else
        mmd_tune<dev::IN_TB, true>(h, L.pro, nullptr, C.cptr, C.cpos, BC.tb, L.d.ZhT, BC.x, B.x,
                                   s);
      mmd_tune<dev::IN_DIRECT, false>(h, L.rast, nullptr, nullptr, nullptr, nullptr, L.d.Zr, B.r,
                                      B.tb, s);
      continue;
    }
    L.dmmd_split = 0;
    if (h->dense_split > 16) break;
    const int64_t n = L.n;
    const double* in = B.b;
    double* out = B.x;
    if (!L.dmmd_M) {
      L.dmm_ld = (n + 3) / 4 * 4;
      L.dmmd_M = h->alloc<double>((size_t)(n * L.dmm_ld));
      KLAUNCH0(nblocks(n * L.dmm_ld), dev::kBlock, 0, s, dev::k_pad_rows<double>, n, L.dmm_ld,
               L.d.Ainv, L.dmmd_M);
      LAUNCH_OK();
      L.dmmd_part = h->alloc<double>((size_t)(16 * n * 64));
      L.dmmd_part_cap = 16 * n * 64;
    }
    float best = 1e30f;
    if (h->dense_split == 0)
      best = time_runs(s, [&] {
        bgemm<double, dev::IN_DIRECT, false, 64>(L.dense, nullptr, nullptr, nullptr, nullptr,
                                                 L.d.Ainv, in, out, s);
      });
    std::vector<int> want;
    if (h->dense_split > 0)
      want.push_back(h->dense_split);
    else
      want = {1, 2, 3, 4, 6, 8, 12, 16};
    for (int KC : {16, 32})
      for (int w : want) {
        int S = 1, kc = 0;
        dense_split_shape(n, w, KC, &S, &kc);
        const float ms = time_runs(s, [&] { dense_mm_launch_d(L, S, kc, KC, in, out, s); });
        if (ms < best) {
          best = ms;
          L.dmmd_split = S;
          L.dmmd_kchunk = kc;
          L.dmmd_kc = KC;
        }
      }
    break;
  }
  HIP_OK(hipStreamSynchronize(s));
  h->dmmd_tuned = true;
}

// Rows per wavefront of k_bspmm64: about 48 entries per wave; 0 when the
// rows are long enough for one row per wave (k_bspmv / k_bresid_t).
int rows_per_wave(int64_t nnz, int64_t rows) {
  const int64_t avg = std::max<int64_t>(1, nnz / std::max<int64_t>(1, rows));
  const int rpw = (int)std::min<int64_t>(16, std::max<int64_t>(1, 48 / avg));
  return rpw >= 2 ? rpw : 0;
}

// k_bata_tile on 64 columns: EPI 0 R = B - G^T G X; EPI 1 R = G^T G X and
// partials of B . R (kBNP workgroups, as k_bsum expects)
template <typename T, int EPI>
void bata_tile(const DLevel& L, const T* X, const T* B, T* R, double* part, hipStream_t s) {
  const DPrec<T>& P = prec<T>(const_cast<DLevel&>(L));
  const size_t lds = (size_t)(L.at.umax + L.at_rmax) * 64 * sizeof(T);
  const unsigned grid = EPI == 1 ? (unsigned)kBNP : (unsigned)L.at.ntile;
  const bool rows = L.at_form == 2 || (L.at_form == 0 && sizeof(T) == sizeof(float));
  PROF(kname(rows ? "k_bata_tile" : "k_bata_tilex",
             std::string(tname<T>()) + ", " + std::to_string(kAtaTile) + ", " +
                                std::to_string(L.ata_me) + ", " + std::to_string(L.ata_mf) + ", " +
                                std::to_string(EPI)),
       (double)sizeof(T) * L.n * 64 * 3 + (double)L.nnz * (sizeof(T) + 4) + 8.0 * (L.n + L.nrows),
       s);
  if (!rows) {
    auto launchx = [&](auto kern) {
      KLAUNCH(grid, dev::kBlock, (size_t)L.at.umax * 64 * sizeof(T), s, kern, L.n, L.at,
              (const T*)P.tev, (const T*)P.tdw, X, B, R, part);
    };
    const int me = L.ata_me, mf = L.ata_mf;
    if (me == 6 && mf == 3)
      launchx(dev::k_bata_tilex<T, kAtaTile, 6, 3, EPI>);
    else if (me == 6)
      launchx(dev::k_bata_tilex<T, kAtaTile, 6, 4, EPI>);
    else if (me == 8 && mf == 3)
      launchx(dev::k_bata_tilex<T, kAtaTile, 8, 3, EPI>);
    else if (me == 8)
      launchx(dev::k_bata_tilex<T, kAtaTile, 8, 4, EPI>);
    else if (mf == 3)
      launchx(dev::k_bata_tilex<T, kAtaTile, 16, 3, EPI>);
    else
      launchx(dev::k_bata_tilex<T, kAtaTile, 16, 4, EPI>);
    LAUNCH_OK();
    return;
  }
  auto launch = [&](auto kern) {
    KLAUNCH(grid, dev::kBlock, lds, s, kern, L.n, L.at, (const T*)P.trv, (const T*)P.tdw, X, B, R,
            part);
  };
  const int me = L.ata_me, mf = L.ata_mf;
  if (me == 6 && mf == 3)
    launch(dev::k_bata_tile<T, kAtaTile, 6, 3, EPI>);
  else if (me == 6)
    launch(dev::k_bata_tile<T, kAtaTile, 6, 4, EPI>);
  else if (me == 8 && mf == 3)
    launch(dev::k_bata_tile<T, kAtaTile, 8, 3, EPI>);
  else if (me == 8)
    launch(dev::k_bata_tile<T, kAtaTile, 8, 4, EPI>);
  else if (mf == 3)
    launch(dev::k_bata_tile<T, kAtaTile, 16, 3, EPI>);
  else
    launch(dev::k_bata_tile<T, kAtaTile, 16, 4, EPI>);
  LAUNCH_OK();
}

// coarse-level residual on 64 columns by row groups: k_bgrp_ata64 stages
// R_g^T R_g X(supp_g) per task, k_bresid_stg64 gathers R = B - staged
void bgrp_resid(const DLevel& L, const float* X, const float* B, float* R, float* stg,
                hipStream_t s) {
  {
    PROF("k_bgrp_ata64",
         4.0 * (L.nnz + 2.0 * L.bg_nstg * 64) + 36.0 * L.bg_ntask, s);
    const size_t lds = ((size_t)(L.bg_wmax + 32) * 64 + 32 * (size_t)(L.bg_wmax + 1)) * sizeof(float);
    KLAUNCH((unsigned)L.bg_ntask, dev::kBlock, lds, s, dev::k_bgrp_ata64, L.bgtask,
            L.bg_wmax, (const float*)L.f.g_val, L.grp_supp, X, stg);
    LAUNCH_OK();
  }
  PROF("k_bresid_stg64<float>", 4.0 * (L.bg_nstg + 2.0 * L.n) * 64 + 8.0 * (L.bg_nstg + L.n), s);
  KLAUNCH(nblocks(L.n * 64), dev::kBlock, 0, s, dev::k_bresid_stg64<float>, L.n, L.bg_cptr,
          L.bg_cpos, (const float*)stg, B, R);
  LAUNCH_OK();
}

template <typename T, int NB>
void bresidual(DLevel& L, BVec<T>& V, const T* X, const T* B, T* R, hipStream_t s) {
  DPrec<T>& P = prec<T>(L);
  if (!L.g_ptr || !L.gt_ptr) throw DevError{LSAMG_EINVAL, "G missing on the device"};
  if constexpr (NB == 64) {
    if (L.at_on) {                      // one pass, X rows staged per tile
      bata_tile<T, 0>(L, X, B, R, nullptr, s);
      return;
    }
    if constexpr (std::is_same<T, float>::value) {
      if (L.bg_on) {                    // row groups, staged
        bgrp_resid(L, X, B, R, V.stg, s);
        return;
      }
    }
  }
  // two CSR passes: on 64 columns a 16-lane group per row, four columns per
  // lane (k_bspmv4); narrower batches one row per wavefront slice
  if (NB == 64) {
    {
      PROF(kname("k_bspmv4", std::string(tname<T>()) + ", false"),
           L.nnz * (sizeof(T) + 4) + 8 * (L.nrows + 1) + sizeof(T) * (L.n + L.nrows) * NB, s);
      KLAUNCH(nblocks(L.nrows * 16), dev::kBlock, 0, s, dev::k_bspmv4<T, false>, L.nrows,
              L.g_ptr, L.g_col, P.g_val, X, (const T*)nullptr, V.y);
      LAUNCH_OK();
    }
    PROF(kname("k_bspmv4", std::string(tname<T>()) + ", true"),
         L.nnz * (sizeof(T) + 4) + 8 * (L.n + 1) + sizeof(T) * (L.nrows + 2 * L.n) * NB, s);
    KLAUNCH(nblocks(L.n * 16), dev::kBlock, 0, s, dev::k_bspmv4<T, true>, L.n, L.gt_ptr,
            L.gt_col, P.gt_val, (const T*)V.y, B, R);
    LAUNCH_OK();
    return;
  }
  {
    PROF(kname("k_bspmv", std::string(tname<T>()) + ", " + std::to_string(NB)),
         L.nnz * (sizeof(T) + 4) + 8 * (L.nrows + 1) + sizeof(T) * (L.n + L.nrows) * NB, s);
    KLAUNCH(nblocks(L.nrows * NB), dev::kBlock, 0, s, dev::k_bspmv<T, NB>, L.nrows, L.g_ptr,
            L.g_col, P.g_val, X, V.y);
    LAUNCH_OK();
  }
  PROF(kname("k_bresid_t", std::string(tname<T>()) + ", " + std::to_string(NB)),
       L.nnz * (sizeof(T) + 4) + 8 * (L.n + 1) + sizeof(T) * (L.nrows + 2 * L.n) * NB, s);
  KLAUNCH(nblocks(L.n * NB), dev::kBlock, 0, s, dev::k_bresid_t<T, NB>, L.n, L.gt_ptr, L.gt_col,
          P.gt_val, (const T*)V.y, B, R);
  LAUNCH_OK();
}

// X = B_l(B) for NB interleaved right-hand sides (see vcycle)
template <typename T, int NB>
void bvcycle(lsamg_handle* h, size_t l, const T* B, T* X, hipStream_t s, bool finalize) {
  LevelTag tag_((int)l);
  DLevel& L = h->L[l];
  DPrec<T>& P = prec<T>(L);
  BVec<T> V = bvec<T>(h->BL[l]);
  if (L.coarsest || L.tail) {
    if constexpr (std::is_same<T, float>::value && NB == 64) {
      if (L.dmm_split > 0) {
        dense_mm_launch(L, L.dmm_split, L.dmm_kchunk, L.dmm_kc, B, X, L.dense.mm.part,
                        L.dense.mm.part_cap, s);
        return;
      }
    }
    if constexpr (std::is_same<T, double>::value && NB == 64) {
      if (L.dmmd_split > 0) {
        dense_mm_launch_d(L, L.dmmd_split, L.dmmd_kchunk, L.dmmd_kc, B, X, s);
        return;
      }
    }
    bgemm<T, dev::IN_DIRECT, false, NB>(L.dense, nullptr, nullptr, nullptr, nullptr, P.Ainv, B, X,
                                        s);
    return;
  }
  DLevel& C = h->L[l + 1];
  BVec<T> VC = bvec<T>(h->BL[l + 1]);
  bgemm<T, dev::IN_GATHER, false, NB>(L.ras, L.oidx, nullptr, nullptr, nullptr, P.Zc, B, X, s);
  bresidual<T, NB>(L, V, X, B, V.r, s);
  bgemm<T, dev::IN_DIRECT, false, NB>(L.rst, nullptr, nullptr, nullptr, nullptr, P.Zh, V.r, VC.b,
                                      s);
  bvcycle<T, NB>(h, l + 1, VC.b, VC.x, s, false);
  if (C.coarsest || C.tail)
    bgemm<T, dev::IN_DIRECT, true, NB>(L.pro, nullptr, nullptr, nullptr, nullptr, P.ZhT, VC.x, X,
                                       s);
  else
    bgemm<T, dev::IN_TB, true, NB>(L.pro, nullptr, C.cptr, C.cpos, VC.tb, P.ZhT, VC.x, X, s,
                                   (int64_t)(sizeof(T)) * C.ntb + 8 * (C.ntb + C.n + 1) / NB);
  bresidual<T, NB>(L, V, X, B, V.r, s);
  bgemm<T, dev::IN_DIRECT, false, NB>(L.rast, nullptr, nullptr, nullptr, nullptr, P.Zr, V.r, V.tb,
                                      s);
  if (finalize) {
    PROF(kname("k_bgather_add", std::string(tname<T>()) + ", " + std::to_string(NB)),
         8 * (L.ntb + L.n + 1) + sizeof(T) * (L.ntb + 2 * L.n) * NB, s);
    KLAUNCH(nblocks(L.n * NB), dev::kBlock, 0, s, dev::k_bgather_add<T, NB>, L.n, L.cptr, L.cpos,
            (const T*)V.tb, X);
    LAUNCH_OK();
  }
}

// Choose the k_bmm tile shapes of every operator the FP32 multi-right-hand-
// side V-cycle applies (once per allocation of the batched buffers).
void bgroup_tune(lsamg_handle* h, hipStream_t s);

template <int NB>
void mm_tune_all(lsamg_handle* h, hipStream_t s) {
  if constexpr (NB >= 16) {
    // the k_bmm shapes are chosen by the first batch (of any width >= 16);
    // the 64-column forms (dense-level GEMM, coarse residual) by the first
    // batch of 64, which also re-times the dense level's k_bmm shape at 64
    const bool need_mm = !h->mm_tuned, need64 = NB == 64 && !h->mm_tuned64;
    if ((!need_mm && !need64) || h->dry) return;
    struct Quiet {                       // tuning launches are not profiled
      Profiler* p;
      lsamg_handle* h;
      ~Quiet() {
        g_prof = p;
        h->batch_alloc = false;
      }
    } quiet{g_prof, h};
    g_prof = nullptr;
    h->batch_alloc = true;               // task lists live with the batched buffers
    // partial sums of split loops: 16 slots of the dense level, or 4 slots
    // of a coarse level's output (RAS/P^T/P: n unknowns; RAS-T: staging).
    // The shapes chosen now serve every later batch up to the buffers' width
    // (bwidth >= NB), so the buffer and the split limits are sized for it.
    const int64_t W = std::max<int64_t>(NB, h->bwidth);
    int64_t cap = 0;
    for (size_t l = 0; l < h->L.size(); ++l) {
      DLevel& L = h->L[l];
      if (L.coarsest || L.tail) {
        cap = std::max<int64_t>(cap, 16 * L.n * W);
        break;
      }
      if (l > 0) cap = std::max<int64_t>(cap, 4 * std::max(L.n, L.ntb) * W);
    }
    if (!h->mm_part && cap > 0) {
      h->mm_part = h->alloc<float>((size_t)cap);
      h->mm_part_cap = cap;
    }
    float* part = h->mm_part;
    cap = h->mm_part_cap;
    // 512 MiB written between timed launches evicts the 256 MiB last-level cache
    struct Flush {
      double* p = nullptr;
      ~Flush() {
        if (p) (void)hipFree(p);
      }
    } fl;
    const int64_t flush_n = (int64_t)64 << 20;
    if (hipMalloc((void**)&fl.p, (size_t)flush_n * sizeof(double)) != hipSuccess) {
      fl.p = nullptr;                      // no room: time without evicting
      (void)hipGetLastError();
    }
    for (size_t l = 0; l < h->L.size(); ++l) {
      DLevel& L = h->L[l];
      auto& B = h->BL[l];
      if (L.coarsest || L.tail) {
        const float bmm_ms =
            mm_tune<dev::IN_DIRECT, false, NB>(h, L.dense, nullptr, nullptr, nullptr, nullptr,
                                               L.f.Ainv, B.fb, B.fx, part, cap, s, fl.p, flush_n);
        if (NB == 64)
          dense_tune(h, L, L.f.Ainv, B.fb, B.fx, part, cap, s, fl.p, flush_n, bmm_ms);
        break;
      }
      if (!need_mm) continue;
      DLevel& C = h->L[l + 1];
      auto& BC = h->BL[l + 1];
      mm_tune<dev::IN_GATHER, false, NB>(h, L.ras, L.oidx, nullptr, nullptr, nullptr, L.f.Zc,
                                         B.fb, B.fx, part, cap, s, fl.p, flush_n);
      mm_tune<dev::IN_DIRECT, false, NB>(h, L.rst, nullptr, nullptr, nullptr, nullptr, L.f.Zh,
                                         B.fr, BC.fb, part, cap, s, fl.p, flush_n);
      if (C.coarsest || C.tail)
        mm_tune<dev::IN_DIRECT, true, NB>(h, L.pro, nullptr, nullptr, nullptr, nullptr, L.f.ZhT,
                                          BC.fx, B.fx, part, cap, s, fl.p, flush_n);
      else
        mm_tune<dev::IN_TB, true, NB>(h, L.pro, nullptr, C.cptr, C.cpos, BC.ftb, L.f.ZhT, BC.fx,
                                      B.fx, part, cap, s, fl.p, flush_n);
      mm_tune<dev::IN_DIRECT, false, NB>(h, L.rast, nullptr, nullptr, nullptr, nullptr, L.f.Zr,
                                         B.fr, B.ftb, part, cap, s, fl.p, flush_n);
    }
    if (NB == 64) bgroup_tune(h, s);
    HIP_OK(hipStreamSynchronize(s));
    h->mm_tuned = true;
    if (NB == 64) h->mm_tuned64 = true;
  }
}

// Coarse-level residual on 64 columns, FP32: the row-group pass against the
// two CSR passes, each timed on the level's own buffers (one warm-up and
// three timed applications), unless LSAMG_OPT_BGROUP fixes the form.
void bgroup_tune(lsamg_handle* h, hipStream_t s) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  try {
    for (size_t l = 1; l < h->L.size(); ++l) {
      DLevel& L = h->L[l];
      if (L.coarsest || L.tail) break;
      L.bg_on = false;
      if (!L.bg_ok || h->bgroup == 2) continue;
      if (h->bgroup == 1) {
        L.bg_on = true;
        continue;
      }
      BVec<float> V = bvec<float>(h->BL[l]);
      float t[2] = {1e30f, 1e30f};
      for (int form = 0; form < 2; ++form) {
        L.bg_on = form == 1;
        bresidual<float, 64>(L, V, V.x, V.b, V.r, s);
        for (int round = 0; round < 1; ++round) {   // three launches after the warm-up
          HIP_OK(hipEventRecord(e0, s));
          for (int r = 0; r < 3; ++r) bresidual<float, 64>(L, V, V.x, V.b, V.r, s);
          HIP_OK(hipEventRecord(e1, s));
          HIP_OK(hipEventSynchronize(e1));
          float ms = 0.f;
          HIP_OK(hipEventElapsedTime(&ms, e0, e1));
          t[form] = std::min(t[form], ms);
        }
      }
      L.bg_on = t[1] < t[0];
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Dense tail: the V-cycle of levels >= lc is a fixed symmetric linear map
// B_lc.  It is formed once, in FP64, by applying the multi-right-hand-side
// V-cycle to the columns of the identity (64 at a time), symmetrized, and
// stored in both precisions as the level's dense operator; later V-cycles
// apply it with one dense GEMV (or GEMM) instead of recursing.  Temporary
// multi-right-hand-side buffers for levels >= lc are freed afterwards.
void build_tail(lsamg_handle* h, size_t lc) {
  DLevel& T = h->L[lc];
  const int64_t n = T.n;
  T.d.Ainv = h->alloc<double>((size_t)n * n);
  T.f.Ainv = h->alloc<float>((size_t)n * n);
  make_dense_plan(h, T);
  if (h->dry) {
    make_packed(h, T, false);
    T.tail = true;
    return;
  }
  constexpr int NB = 64;
  struct Tmp {
    std::vector<void*> v;
    lsamg_handle* h;
    ~Tmp() {
      for (void* p : v) (void)hipFree(p);
      h->BL.clear();
    }
    double* get(size_t count) {
      void* p = nullptr;
      HIP_OK(hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(double)));
      v.push_back(p);
      return (double*)p;
    }
  } tmp{{}, h};
  h->BL.assign(h->L.size(), lsamg_handle::BLev{});
  for (size_t l = lc; l < h->L.size(); ++l) {
    DLevel& L = h->L[l];
    auto& B = h->BL[l];
    const size_t nn = (size_t)L.n * NB, ny = (size_t)std::max<int64_t>(L.nrows, 1) * NB,
                 nt = (size_t)std::max<int64_t>(L.ntb, 1) * NB;
    B.x = tmp.get(nn);
    B.b = tmp.get(nn);
    B.r = tmp.get(nn);
    B.y = tmp.get(ny);
    B.tb = tmp.get(nt);
  }
  double* E = tmp.get((size_t)n * NB);
  double* X = tmp.get((size_t)n * NB);
  hipStream_t s = nullptr;
  const unsigned g = nblocks(n * NB);
  for (int64_t j0 = 0; j0 < n; j0 += NB) {
    KLAUNCH0(g, dev::kBlock, 0, s, dev::k_unit_block<NB>, n, j0, E);
    LAUNCH_OK();
    bvcycle<double, NB>(h, lc, E, X, s, true);
    KLAUNCH0(g, dev::kBlock, 0, s, dev::k_scatter_cols<NB>, n, j0, (const double*)X, T.d.Ainv);
    LAUNCH_OK();
  }
  KLAUNCH0(nblocks(n * n), dev::kBlock, 0, s, dev::k_symmetrize, n, T.d.Ainv);
  LAUNCH_OK();
  KLAUNCH0(nblocks(n * n), dev::kBlock, 0, s, dev::k_convert<double, float>, n * n,
           (const double*)T.d.Ainv, T.f.Ainv);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  make_packed(h, T, true);
  T.tail = true;
}

template <int NB>
void bsum(const double* part, double* out, hipStream_t s);

template <int NB>
void bcg_apply(lsamg_handle* h, const double* Pv, double* Qv, double* pq_part, double* pq,
               hipStream_t s) {
  DLevel& L = h->L[0];
  BVec<double> V = bvec<double>(h->BL[0]);
  if (!L.g_ptr || !L.gt_ptr) throw DevError{LSAMG_EINVAL, "finest-level G missing on the device"};
  if constexpr (NB == 64) {
    if (L.fuse_ata && L.at_on) {
      bata_tile<double, 1>(L, Pv, Pv, Qv, pq_part, s);
      bsum<NB>(pq_part, pq, s);
      return;
    }
  }
  if (L.fuse_ata) {
    {
      PROF(kname("k_bcg_apq1", std::to_string(NB) + ", " + std::to_string(L.ata_me) + ", " +
                                   std::to_string(L.ata_mf)),
           2 * L.nnz * 12 + 8 * (L.n + L.nrows + 2) + 8 * 3 * L.n * NB, s);
      auto launch = [&](auto kern) {
        KLAUNCH(kBNP, dev::kBlock, 0, s, kern, L.n, L.gt_ptr, L.gt_col, L.d.gt_val, L.g_ptr,
                L.g_col, L.d.g_val, Pv, Qv, pq_part);
      };
      const int me = L.ata_me, mf = L.ata_mf;
      if (me == 6 && mf == 3)
        launch(dev::k_bcg_apq1<NB, 6, 3>);
      else if (me == 6)
        launch(dev::k_bcg_apq1<NB, 6, 4>);
      else if (me == 8 && mf == 3)
        launch(dev::k_bcg_apq1<NB, 8, 3>);
      else if (me == 8)
        launch(dev::k_bcg_apq1<NB, 8, 4>);
      else if (mf == 3)
        launch(dev::k_bcg_apq1<NB, 16, 3>);
      else
        launch(dev::k_bcg_apq1<NB, 16, 4>);
      LAUNCH_OK();
    }
    bsum<NB>(pq_part, pq, s);
    return;
  }
  const int rpw_g = NB == 64 ? rows_per_wave(L.nnz, L.nrows) : 0;
  if (rpw_g > 0) {
    PROF(kname("k_bspmm64", "double"), L.nnz * 12 + 8 * (L.nrows + 1) + 8 * (L.n + L.nrows) * NB,
         s);
    KLAUNCH((unsigned)((L.nrows + 4 * rpw_g - 1) / (4 * rpw_g)), dev::kBlock, 0, s,
            dev::k_bspmm64<double>, L.nrows, rpw_g, L.g_ptr, L.g_col, L.d.g_val, Pv,
            (const double*)nullptr, V.y);
    LAUNCH_OK();
  } else {
    PROF(kname("k_bspmv", std::string("double, ") + std::to_string(NB)),
         L.nnz * 12 + 8 * (L.nrows + 1) + 8 * (L.n + L.nrows) * NB, s);
    KLAUNCH(nblocks(L.nrows * NB), dev::kBlock, 0, s, dev::k_bspmv<double, NB>, L.nrows, L.g_ptr,
            L.g_col, L.d.g_val, Pv, V.y);
    LAUNCH_OK();
  }
  PROF(kname("k_bcg_apq", std::to_string(NB)),
       L.nnz * 12 + 8 * (L.n + 1) + 8 * (L.nrows + 2 * L.n) * NB, s);
  KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_apq<NB>, L.n, L.gt_ptr, L.gt_col, L.d.gt_val,
          (const double*)V.y, Pv, Qv, pq_part);
  LAUNCH_OK();
  bsum<NB>(pq_part, pq, s);
}

// Z = B R (one batched V-cycle) and the rho partials of R . Z into Brz[cur];
// with Qv given also the partials of -(Z . Qv) into Bzq
template <int NB>
void bcg_z(lsamg_handle* h, hipStream_t s, int cur, const double* Qv) {
  DLevel& L0 = h->L[0];
  const int64_t n = L0.n;
  auto& B0 = h->BL[0];
  const bool stage = !L0.coarsest;
  if (h->precision == LSAMG_MIXED) {
    run_graph(h, 128 + NB, s,
              [&](hipStream_t gs) { bvcycle<float, NB>(h, 0, B0.fb, B0.fx, gs, false); });
    if (NB == 64) {
      PROF("k_bcg_z64<float>", (Qv ? 28 : 20) * n * NB, s);
      KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_z64<float>, n, (const float*)B0.fx,
              stage ? L0.cptr : nullptr, L0.cpos, (const float*)B0.ftb, (const double*)h->BR,
              h->BZ, h->Brz[cur], Qv, h->Bzq);
    } else {
      PROF(kname("k_bcg_z", std::string("float, ") + std::to_string(NB)), (Qv ? 28 : 20) * n * NB,
           s);
      KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_z<float, NB>, n, (const float*)B0.fx,
              stage ? L0.cptr : nullptr, L0.cpos, (const float*)B0.ftb, (const double*)h->BR, h->BZ,
              h->Brz[cur], Qv, h->Bzq);
    }
  } else {
    run_graph(h, NB, s, [&](hipStream_t gs) { bvcycle<double, NB>(h, 0, h->BR, B0.x, gs, false); });
    if (NB == 64) {
      PROF("k_bcg_z64<double>", (Qv ? 32 : 24) * n * NB, s);
      KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_z64<double>, n, (const double*)B0.x,
              stage ? L0.cptr : nullptr, L0.cpos, (const double*)B0.tb, (const double*)h->BR,
              h->BZ, h->Brz[cur], Qv, h->Bzq);
    } else {
      PROF(kname("k_bcg_z", std::string("double, ") + std::to_string(NB)), (Qv ? 32 : 24) * n * NB,
           s);
      KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_z<double, NB>, n, (const double*)B0.x,
              stage ? L0.cptr : nullptr, L0.cpos, (const double*)B0.tb, (const double*)h->BR,
              h->BZ, h->Brz[cur], Qv, h->Bzq);
    }
  }
  LAUNCH_OK();
}

// Z = B R, rho per column into Brz_s[cur], and the next direction P = Z +
// beta P (P = Z when first); with restart_mask given, only the masked
// columns take P = Z and the others keep P (their direction was already
// formed from the same Z)
template <int NB>
void bcg_precondition(lsamg_handle* h, hipStream_t s, bool first, int cur,
                      const int* restart_mask = nullptr) {
  const int64_t n = h->L[0].n;
  // flexible CG: beta_j = -(Z_j . Q_j) / (P_j . Q_j) with Q = A P of the
  // directions just used (Bpq_s still holds P . Q from that A-apply)
  const bool fcg = h->krylov == LSAMG_KRYLOV_FCG;
  const double* Qv = fcg && !first ? (const double*)h->BQ : nullptr;
  bcg_z<NB>(h, s, cur, Qv);
  bsum<NB>(h->Brz[cur], h->Brz_s[cur], s);
  if (Qv) bsum<NB>(h->Bzq, h->Bzq_s, s);
  if (restart_mask) {
    PROF(kname("k_bcg_dir_mask", std::to_string(NB)), 16 * n * NB, s);
    KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_dir_mask<NB>, n, restart_mask,
            (const double*)h->BZ, h->BP);
    LAUNCH_OK();
    return;
  }
  PROF(kname("k_bcg_dir", std::to_string(NB)), 24 * n * NB, s);
  const double* num = fcg ? h->Bzq_s : h->Brz_s[cur];
  const double* den = fcg ? h->Bpq_s : h->Brz_s[1 - cur];
  KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_dir<NB>, n, num, first ? (const double*)nullptr : den,
          (const double*)h->BZ, h->BP);
  LAUNCH_OK();
}

// per-column scalars out[j] = sum of the kBNP partials of column j
template <int NB>
void bsum(const double* part, double* out, hipStream_t s) {
  PROF(kname("k_bsum", std::to_string(NB)), 8.0 * (kBNP + 1) * NB, s);
  KLAUNCH(NB, dev::kBlock, 0, s, dev::k_bsum<NB>, kBNP, part, out);
  LAUNCH_OK();
}

// NB per-column scalars copied to pinned slot
void bparts_to_host(lsamg_handle* h, const double* scal, int NB, int slot, hipStream_t s) {
  HIP_OK(hipMemcpyAsync(h->Bparts_host + (size_t)slot * 64, scal, (size_t)NB * sizeof(double),
                        hipMemcpyDeviceToHost, s));
}

void bhost_sums(const lsamg_handle* h, int NB, int slot, double* out) {
  for (int j = 0; j < NB; ++j) out[j] = h->Bparts_host[(size_t)slot * 64 + j];
}

// Host-side state of one column of the multi-right-hand-side PCG.
struct BCol {
  int active = 0;        // iterating
  int its = 0, maxit = 0, restarts = 0, conv = 0, done = 0, bad = 0;
  double tol = 0, nb = 0, rn = 0, tr = 0;   // tr: ||b - A x|| when done
};

// Multi-right-hand-side PCG on up to NB interleaved columns: one FP64 CG per
// column (own scalars, stop test and iteration count) sharing every matrix
// read of the V-cycle and of A.  Columns can be loaded whenever the engine
// is between iterations and retire as soon as they finish, so a solve can
// take new right-hand sides at any iteration boundary (the request server
// does; pcg_batched loads all columns at once).
//
// Cycle: load columns -> norms() -> prepare() [Z = B R, next directions]
// -> step() [q = A p, x, r update; stop tests on the recurrence residual,
// then on the true residual] -> retire / load -> norms() -> prepare() ...
// A column that enters (fresh) or whose recurrence residual passed while
// its true residual did not (restart: r = b - A x) takes p = z as its next
// direction.
template <int NB>
struct BatchCG {
  lsamg_handle* h;
  hipStream_t s;
  bool mixed;
  int cur = 0;               // Brz_s[cur]: rho of the current directions
  bool pre_queued = false;   // the next preconditioner step is already queued
  double fac = 0.5;          // slowest average reduction per iteration so far
  BCol c[NB];
  // flags of the device copy (h->Bactive): active, restart, new direction;
  // copied to the pinned staging only inside prepare(), right before the
  // upload (the step that follows synchronises past that copy)
  int flg[192] = {};
  int* act = flg;
  int* rst = flg + 64;
  int* ndir = flg + 128;

  BatchCG(lsamg_handle* h_, hipStream_t s_) : h(h_), s(s_) {
    ensure_batched(h, NB);
    if (h->precision == LSAMG_MIXED && h->use_mfma) mm_tune_all<NB>(h, s);
    if (h->precision == LSAMG_FP64 && h->use_mfma && NB == 64) fp64_tune(h, s);
    mixed = h->precision == LSAMG_MIXED;
    const int64_t n0 = h->L[0].n * NB;
    // every column starts from zeros, so unused columns stay finite
    for (double* v : {h->BX, h->BR, h->BZ, h->BP, h->BQ, h->BBi}) {
      KLAUNCH0(nblocks(n0), dev::kBlock, 0, s, dev::k_fill, n0, 0.0, v);
      LAUNCH_OK();
    }
    for (double* v : {h->Brz_s[0], h->Brz_s[1], h->Bpq_s, h->Bzq_s}) {
      KLAUNCH0(1, dev::kBlock, 0, s, dev::k_fill, (int64_t)NB, 0.0, v);
      LAUNCH_OK();
    }
    if (mixed) {
      KLAUNCH0(nblocks(n0), dev::kBlock, 0, s, dev::k_fill_f32, n0, 0.0f, h->BL[0].fb);
      LAUNCH_OK();
    }
  }

  int64_t n() const { return h->L[0].n; }
  int nactive() const {
    int k = 0;
    for (int j = 0; j < NB; ++j) k += c[j].active;
    return k;
  }

  // columns j0 .. j0+ncols-1 from the user's device columns b (leading
  // dimension ld); they become fresh (norms() then decides what runs)
  void load(int j0, int ncols, const double* b, int64_t ld, double tol, int maxit) {
    const int64_t nn = n() * ncols;
    KLAUNCH0(nblocks(nn), dev::kBlock, 0, s, dev::k_bload<NB>, n(), j0, ncols, ld,
             (const int64_t*)h->perm, b, h->BBi, h->BR, h->BX, h->BP,
             mixed ? h->BL[0].fb : (float*)nullptr);
    LAUNCH_OK();
    for (int j = j0; j < j0 + ncols; ++j) {
      c[j] = BCol{};
      c[j].tol = tol;
      c[j].maxit = maxit;
      c[j].nb = -1.0;            // norm pending
      ndir[j] = 1;
    }
  }

  // ||b|| of the freshly loaded columns; a zero column is done at once
  // (x = 0), a non-finite one is marked bad, maxit 0 leaves x = 0 unconverged
  void norms() {
    bool any = false;
    for (int j = 0; j < NB; ++j) any = any || c[j].nb < 0;
    if (!any) return;
    KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bdot<NB>, n(), (const double*)h->BBi,
             (const double*)h->BBi, h->Btmp);
    LAUNCH_OK();
    bsum<NB>(h->Btmp, h->Btmp_s, s);
    bparts_to_host(h, h->Btmp_s, NB, 0, s);
    HIP_OK(hipStreamSynchronize(s));
    double nb2[NB];
    bhost_sums(h, NB, 0, nb2);
    for (int j = 0; j < NB; ++j) {
      if (!(c[j].nb < 0)) continue;
      BCol& q = c[j];
      if (!std::isfinite(nb2[j])) {
        q.bad = q.done = 1;
        q.nb = 0;
        continue;
      }
      q.nb = q.rn = q.tr = std::sqrt(nb2[j]);
      if (q.nb == 0.0) {
        q.conv = q.done = 1;
      } else if (q.maxit <= 0) {
        q.done = 1;
      } else {
        q.active = 1;
      }
    }
  }

  // Z = B R and the next directions (P = Z on fresh and restarted columns)
  void prepare() {
    int nnew = 0;
    for (int j = 0; j < NB; ++j) {
      act[j] = c[j].active;
      if (!c[j].active) ndir[j] = rst[j] = 0;
      nnew += ndir[j];
    }
    const int nact = nactive();
    if (nact == 0) {
      pre_queued = false;
      return;
    }
    std::memcpy(h->Bactive_host, flg, sizeof(flg));
    HIP_OK(hipMemcpyAsync(h->Bactive, h->Bactive_host, sizeof(flg), hipMemcpyHostToDevice, s));
    int nrst = 0;
    for (int j = 0; j < NB; ++j) nrst += rst[j];
    if (nrst > 0) {
      // r = b - A x on the restarted columns (A x is in BZ from the true-residual
      // test of the last step); rho_old = 0 there
      KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bcg_restart<NB>, n(), (const int*)(h->Bactive + 64),
               (const double*)h->BBi, (const double*)h->BZ, h->BR,
               mixed ? h->BL[0].fb : (float*)nullptr, h->Brz_s[cur]);
      LAUNCH_OK();
    }
    if (pre_queued) {
      // the other columns' next direction is formed; redo Z for the new ones
      if (nnew > 0) bcg_precondition<NB>(h, s, false, 1 - cur, h->Bactive + 128);
    } else {
      if (nnew > 0) {           // beta = 0 there: zero rho_old (CG) or p . q (flexible CG)
        KLAUNCH0(1, dev::kBlock, 0, s, dev::k_bzero_masked<NB>, (const int*)(h->Bactive + 128),
                 h->krylov == LSAMG_KRYLOV_FCG ? h->Bpq_s : h->Brz_s[cur]);
        LAUNCH_OK();
      }
      bcg_precondition<NB>(h, s, false, 1 - cur);
    }
    for (int j = 0; j < NB; ++j) ndir[j] = rst[j] = 0;
    pre_queued = false;
    cur = 1 - cur;
  }

  // one iteration of every active column; columns that finish in it get
  // done = 1 (converged or at maxit, with their true residual) and leave the
  // active set.  expect_more: the caller will load columns after this step,
  // so the next preconditioner step waits for that instead of being queued
  // early.  Returns the number of columns that finished.
  int step(bool expect_more) {
    if (nactive() == 0) return 0;
    const int64_t nn = n();
    bcg_apply<NB>(h, h->BP, h->BQ, h->Bpq, h->Bpq_s, s);
    {
      PROF(kname("k_bcg_update", std::to_string(NB)), (mixed ? 60 : 56) * nn * NB, s);
      KLAUNCH(kBNP, dev::kBlock, 0, s, dev::k_bcg_update<NB>, nn, (const double*)h->Brz_s[cur],
              (const double*)h->Bpq_s, (const int*)h->Bactive, (const double*)h->BP,
              (const double*)h->BQ, h->BX, h->BR, mixed ? h->BL[0].fb : (float*)nullptr, h->Brr);
      LAUNCH_OK();
    }
    bsum<NB>(h->Brr, h->Brr_s, s);
    bparts_to_host(h, h->Brr_s, NB, 1, s);
    HIP_OK(hipEventRecord(h->ev_rr[0], s));
    // the most advanced column predicts whether this update converges one
    bool near = expect_more;
    for (int j = 0; j < NB; ++j) {
      if (!c[j].active) continue;
      ++c[j].its;
      near = near || c[j].rn / c[j].nb * fac <= 2.0 * c[j].tol || c[j].its >= c[j].maxit;
    }
    if (!near) {
      bcg_precondition<NB>(h, s, false, 1 - cur);
      pre_queued = true;
    }
    HIP_OK(hipEventSynchronize(h->ev_rr[0]));
    double rr[NB];
    bhost_sums(h, NB, 1, rr);
    int ntest = 0;
    for (int j = 0; j < NB; ++j) {
      if (!c[j].active) continue;
      c[j].rn = std::sqrt(rr[j]);
      if (!std::isfinite(c[j].rn)) throw DevError{LSAMG_ENOTSPD, "CG breakdown (non-finite residual)"};
      ntest += c[j].rn <= c[j].tol * c[j].nb || c[j].its >= c[j].maxit;
    }
    int nfin = 0;
    if (ntest > 0) {
      // true residuals b - A x of the whole block (one batched A-apply into
      // BZ: Z is spent once the directions are formed, and BQ = A P stays
      // for flexible CG's next beta)
      bcg_apply<NB>(h, h->BX, h->BZ, h->Btmp, h->Btmp_s, s);
      KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bres_parts<NB>, nn, (const double*)h->BBi,
               (const double*)h->BZ, h->Btmp);
      LAUNCH_OK();
      bsum<NB>(h->Btmp, h->Btmp_s, s);
      bparts_to_host(h, h->Btmp_s, NB, 0, s);
      HIP_OK(hipStreamSynchronize(s));
      double t2[NB];
      bhost_sums(h, NB, 0, t2);
      for (int j = 0; j < NB; ++j) {
        BCol& q = c[j];
        if (!q.active) continue;
        const bool pass = q.rn <= q.tol * q.nb;
        if (!pass && q.its < q.maxit) continue;
        q.tr = std::sqrt(t2[j]);
        if (pass && q.tr <= q.tol * q.nb) {
          q.conv = 1;
        } else if (q.its < q.maxit) {      // replace r by b - A x, restart
          rst[j] = ndir[j] = 1;
          q.rn = q.tr;
          ++q.restarts;
          continue;
        }
        q.active = 0;
        q.done = 1;
        ++nfin;
      }
    }
    double worst = 0;
    for (int j = 0; j < NB; ++j)
      if (c[j].active) worst = std::max(worst, std::pow(c[j].rn / c[j].nb, 1.0 / c[j].its));
    if (worst > 0) fac = worst;
    return nfin;
  }

  // columns j0 .. j0+ncols-1 of X to the user's device columns x
  void store(int j0, int ncols, double* x, int64_t ld) {
    const int64_t nn = n() * ncols;
    KLAUNCH0(nblocks(nn), dev::kBlock, 0, s, dev::k_bstore<NB>, n(), j0, ncols, ld,
             (const int64_t*)h->perm, (const double*)h->BX, x);
    LAUNCH_OK();
  }

  void stats(int j, lsamg_stats* st, double secs) const {
    const BCol& q = c[j];
    st->iters = q.its;
    st->converged = q.conv;
    st->rel_res = q.nb > 0 ? q.rn / q.nb : 0.0;
    st->true_rel_res = q.nb > 0 ? q.tr / q.nb : 0.0;
    st->rho = (q.its > 0 && q.nb > 0) ? std::pow(q.rn / q.nb, 1.0 / q.its) : 0.0;
    st->restarts = q.restarts;
    st->reserved = 0;
    st->seconds = secs;
  }
};

// PCG on nr <= NB right-hand sides at once (all loaded before the first
// iteration).
template <int NB>
int pcg_batched(lsamg_handle* h, const double* b, double* x, int nr, int64_t ld, double tol,
                int maxit, hipStream_t s, lsamg_stats* st) {
  auto t0 = std::chrono::steady_clock::now();
  BatchCG<NB> E(h, s);
  E.load(0, nr, b, ld, tol, maxit);
  E.norms();
  for (int j = 0; j < nr; ++j)
    if (E.c[j].bad) throw DevError{LSAMG_EBADINPUT, "non-finite entry in a right-hand side"};
  while (E.nactive() > 0) {
    E.prepare();
    E.step(false);
  }
  E.store(0, nr, x, ld);
  HIP_OK(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all = true;
  for (int j = 0; j < nr; ++j) {
    all = all && E.c[j].conv;
    if (st) E.stats(j, st + j, secs);
  }
  return all ? LSAMG_OK : LSAMG_ENOCONV;
}

// Block PCG (O'Leary) on nr <= 64 columns: the A-orthogonalised form
//   Q = A P, G = P^T Q, C = G^+ P^T R, X += P C, R -= Q C,
//   Z = B R, D = -G^+ Q^T Z, P = Z + P D,
// from P = Z = B R0; the 64 x 64 Gram matrices are summed on the device and
// their pseudo-inverse step (eigenvalues at or below 1e-12 of the largest
// dropped, so dependent directions leave the block) runs on the host.  All
// columns iterate together; the stop test and the true-residual restart are
// those of pcg_batched, taken when every nonzero column passes.  Unused
// columns of the 64 are zero and drop out of the Gram matrices.
constexpr int kBgBlocks = 512;         // workgroups of the Gram and update kernels

int pcg_block(lsamg_handle* h, const double* b, double* x, int nr, int64_t ld, double tol,
              int maxit, hipStream_t s, lsamg_stats* st) {
  constexpr int NB = 64;
  auto t0 = std::chrono::steady_clock::now();
  ensure_batched(h, NB);
  if (h->precision == LSAMG_MIXED && h->use_mfma) mm_tune_all<NB>(h, s);
  if (h->precision == LSAMG_FP64 && h->use_mfma) fp64_tune(h, s);
  if (!h->Bg_part) {
    h->batch_alloc = true;
    struct Reset {
      lsamg_handle* h;
      ~Reset() { h->batch_alloc = false; }
    } reset{h};
    h->Bg_part = h->alloc<double>((size_t)kBgBlocks * 4096);
    h->Bg_G = h->alloc<double>(4096);
    h->Bg_F = h->alloc<double>(4096);
    h->Bg_C = h->alloc<double>(4096);
  }
  if (!h->Bg_host)
    HIP_OK(hipHostMalloc((void**)&h->Bg_host, 3 * 4096 * sizeof(double), hipHostMallocDefault));
  double* Gh = h->Bg_host;
  double* Fh = Gh + 4096;
  double* Ch = Fh + 4096;
  const int64_t n = h->L[0].n, nn = n * NB;
  const unsigned ge = nblocks(nn);
  const bool mixed = h->precision == LSAMG_MIXED;
  float* R32 = mixed ? h->BL[0].fb : nullptr;
  auto gram = [&](const double* A, const double* B, double* out) {
    {
      PROF("k_bgram64", 16.0 * nn + 8.0 * kBgBlocks * 4096, s);
      KLAUNCH(kBgBlocks, dev::kBlock, 0, s, dev::k_bgram64, n, A, B, h->Bg_part);
      LAUNCH_OK();
    }
    KLAUNCH0(16, dev::kBlock, 0, s, dev::k_bgram_sum, kBgBlocks, (const double*)h->Bg_part, out);
    LAUNCH_OK();
  };
  auto fetch = [&](const double* dsrc, double* hdst) {
    HIP_OK(hipMemcpyAsync(hdst, dsrc, 4096 * sizeof(double), hipMemcpyDeviceToHost, s));
  };
  auto step_matrix = [&](const double* F, double sign) {   // Ch = sign G^+ F, uploaded
    if (gram_pinv_apply(NB, Gh, F, Ch, 1e-12) < 0)
      throw DevError{LSAMG_ENOTSPD, "block CG: Gram eigen-decomposition did not converge"};
    if (sign < 0)
      for (int e = 0; e < 4096; ++e) Ch[e] = -Ch[e];
    HIP_OK(hipMemcpyAsync(h->Bg_C, Ch, 4096 * sizeof(double), hipMemcpyHostToDevice, s));
  };
  // B (internal numbering, zero beyond nr), X = 0, R = B
  KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_bperm_in<NB>, n, nr, ld, (const int64_t*)h->perm, b,
           h->BBi);
  LAUNCH_OK();
  KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_fill, nn, 0.0, h->BX);
  LAUNCH_OK();
  KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_copy, nn, (const double*)h->BBi, h->BR);
  LAUNCH_OK();
  if (mixed) {
    KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_convert<double, float>, nn, (const double*)h->BR, R32);
    LAUNCH_OK();
  }
  auto col_sums = [&](double* out) {   // per-column sums of h->Btmp partials (kBNP each)
    bsum<NB>(h->Btmp, h->Btmp_s, s);
    bparts_to_host(h, h->Btmp_s, NB, 0, s);
    HIP_OK(hipStreamSynchronize(s));
    bhost_sums(h, NB, 0, out);
  };
  double nb2[NB], nb[NB];
  KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bdot<NB>, n, (const double*)h->BBi,
           (const double*)h->BBi, h->Btmp);
  LAUNCH_OK();
  col_sums(nb2);
  bool any = false;
  for (int j = 0; j < NB; ++j) {
    if (!std::isfinite(nb2[j])) throw DevError{LSAMG_EBADINPUT, "non-finite entry in a right-hand side"};
    nb[j] = std::sqrt(nb2[j]);
    any = any || (j < nr && nb[j] > 0.0);
  }
  auto precondition_into_p = [&]() {   // Z = B R, P = Z
    bcg_z<NB>(h, s, 0, nullptr);
    KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_copy, nn, (const double*)h->BZ, h->BP);
    LAUNCH_OK();
  };
  int its = 0, restarts = 0;
  bool conv = !any;
  double rn[NB], tr[NB];
  for (int j = 0; j < NB; ++j) rn[j] = tr[j] = nb[j];
  if (!conv && maxit > 0) precondition_into_p();
  while (!conv && its < maxit) {
    bcg_apply<NB>(h, h->BP, h->BQ, h->Bpq, h->Bpq_s, s);            // Q = A P
    gram(h->BP, h->BQ, h->Bg_G);
    gram(h->BP, h->BR, h->Bg_F);
    fetch(h->Bg_G, Gh);
    fetch(h->Bg_F, Fh);
    HIP_OK(hipStreamSynchronize(s));
    step_matrix(Fh, 1.0);                                             // C = G^+ P^T R
    {
      PROF("k_bupd64", 8.0 * nn * (mixed ? 6.5 : 6.0) + 8.0 * 4096, s);
      KLAUNCH(kBgBlocks, dev::kBlock, 0, s, dev::k_bupd64, n, (const double*)h->BP,
              (const double*)h->BQ, (const double*)h->Bg_C, h->BX, h->BR, R32, h->Btmp);
      LAUNCH_OK();
    }
    ++its;
    {                                   // the update wrote kBgBlocks partials per column
      PROF("k_bsum", 8.0 * (kBgBlocks + 1) * NB, s);
      KLAUNCH(NB, dev::kBlock, 0, s, dev::k_bsum<NB>, kBgBlocks, (const double*)h->Btmp,
              h->Btmp_s);
      LAUNCH_OK();
    }
    bparts_to_host(h, h->Btmp_s, NB, 0, s);
    HIP_OK(hipStreamSynchronize(s));
    double rr[NB];
    bhost_sums(h, NB, 0, rr);
    bool pass = true;
    for (int j = 0; j < nr; ++j) {
      rn[j] = std::sqrt(rr[j]);
      if (!std::isfinite(rn[j])) throw DevError{LSAMG_ENOTSPD, "block CG breakdown (non-finite residual)"};
      pass = pass && (nb[j] == 0.0 || rn[j] <= tol * nb[j]);
    }
    if (pass) {
      // true residuals b - A x (A x into BZ)
      bcg_apply<NB>(h, h->BX, h->BZ, h->Btmp, h->Btmp_s, s);
      KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bres_parts<NB>, n, (const double*)h->BBi,
               (const double*)h->BZ, h->Btmp);
      LAUNCH_OK();
      double t2[NB];
      col_sums(t2);
      bool tpass = true;
      for (int j = 0; j < nr; ++j) {
        tr[j] = std::sqrt(t2[j]);
        tpass = tpass && (nb[j] == 0.0 || tr[j] <= tol * nb[j]);
      }
      if (tpass) {
        conv = true;
        break;
      }
      if (its >= maxit) break;
      // restart from the true residual: R = B - A X, P = Z = B R
      KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_sub, nn, (const double*)h->BBi, (const double*)h->BZ,
               h->BR);
      LAUNCH_OK();
      if (mixed) {
        KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_convert<double, float>, nn, (const double*)h->BR, R32);
        LAUNCH_OK();
      }
      ++restarts;
      precondition_into_p();
      continue;
    }
    if (its >= maxit) break;
    bcg_z<NB>(h, s, 0, nullptr);                                      // Z = B R
    gram(h->BQ, h->BZ, h->Bg_F);                                      // E = Q^T Z
    fetch(h->Bg_F, Fh);
    HIP_OK(hipStreamSynchronize(s));
    step_matrix(Fh, -1.0);                                            // D = -G^+ E
    {
      PROF("k_bdir64", 8.0 * nn * 3 + 8.0 * 4096, s);
      KLAUNCH(kBgBlocks, dev::kBlock, 0, s, dev::k_bdir64, n, (const double*)h->BZ,
              (const double*)h->Bg_C, h->BP);
      LAUNCH_OK();
    }
  }
  if (!conv) {                           // true residuals of the final iterate
    bcg_apply<NB>(h, h->BX, h->BZ, h->Btmp, h->Btmp_s, s);
    KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bres_parts<NB>, n, (const double*)h->BBi,
             (const double*)h->BZ, h->Btmp);
    LAUNCH_OK();
    double t2[NB];
    col_sums(t2);
    for (int j = 0; j < nr; ++j) tr[j] = std::sqrt(t2[j]);
  }
  KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_bperm_out<NB>, n, nr, ld, (const int64_t*)h->perm,
           (const double*)h->BX, x);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bool all = true;
  for (int j = 0; j < nr; ++j) {
    const bool cj = nb[j] == 0.0 || tr[j] <= tol * nb[j];
    all = all && cj;
    if (!st) continue;
    st[j].iters = its;
    st[j].converged = cj ? 1 : 0;
    st[j].rel_res = nb[j] > 0 ? rn[j] / nb[j] : 0.0;
    st[j].true_rel_res = nb[j] > 0 ? tr[j] / nb[j] : 0.0;
    st[j].rho = (its > 0 && nb[j] > 0) ? std::pow(rn[j] / nb[j], 1.0 / its) : 0.0;
    st[j].restarts = restarts;
    st[j].seconds = secs;
  }
  return all ? LSAMG_OK : LSAMG_ENOCONV;
}

// Y = B X for nr <= NB columns through the multi-right-hand-side V-cycle
// (the preconditioner step of pcg_batched), user numbering in and out.
template <int NB>
void bapply_vcycle(lsamg_handle* h, const double* X, double* Y, int nr, int64_t ld,
                   hipStream_t s) {
  ensure_batched(h, NB);
  if (h->precision == LSAMG_MIXED && h->use_mfma) mm_tune_all<NB>(h, s);
  if (h->precision == LSAMG_FP64 && h->use_mfma && NB == 64) fp64_tune(h, s);
  DLevel& L0 = h->L[0];
  auto& B0 = h->BL[0];
  const int64_t n = L0.n;
  const unsigned ge = nblocks(n * NB);
  KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_bperm_in<NB>, n, nr, ld, (const int64_t*)h->perm, X,
           h->BR);
  LAUNCH_OK();
  const bool stage = !L0.coarsest;
  if (h->precision == LSAMG_MIXED) {
    KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_convert<double, float>, n * NB, (const double*)h->BR,
             B0.fb);
    LAUNCH_OK();
    bvcycle<float, NB>(h, 0, B0.fb, B0.fx, s, false);
    KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bcg_z<float, NB>, n, (const float*)B0.fx,
             stage ? L0.cptr : nullptr, L0.cpos, (const float*)B0.ftb, (const double*)h->BR, h->BZ,
             h->Btmp, (const double*)nullptr, (double*)nullptr);
  } else {
    bvcycle<double, NB>(h, 0, h->BR, B0.x, s, false);
    KLAUNCH0(kBNP, dev::kBlock, 0, s, dev::k_bcg_z<double, NB>, n, (const double*)B0.x,
             stage ? L0.cptr : nullptr, L0.cpos, (const double*)B0.tb, (const double*)h->BR,
             h->BZ, h->Btmp, (const double*)nullptr, (double*)nullptr);
  }
  LAUNCH_OK();
  KLAUNCH0(ge, dev::kBlock, 0, s, dev::k_bperm_out<NB>, n, nr, ld, (const int64_t*)h->perm,
           (const double*)h->BZ, Y);
  LAUNCH_OK();
  HIP_OK(hipStreamSynchronize(s));
}

int solve_batched(lsamg_handle* h, const double* b, double* x, int nr, int64_t ld, double tol,
                  int maxit, hipStream_t s, lsamg_stats* st) {
  if (nr <= 8) return pcg_batched<8>(h, b, x, nr, ld, tol, maxit, s, st);
  if (nr <= 16) return pcg_batched<16>(h, b, x, nr, ld, tol, maxit, s, st);
  if (nr <= 32) return pcg_batched<32>(h, b, x, nr, ld, tol, maxit, s, st);
  return pcg_batched<64>(h, b, x, nr, ld, tol, maxit, s, st);
}

int fail_with(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace

namespace {

// lsamg_setup; with upload_now false the handle stays host-only (device -1)
// even when p->device names the device that a device setup runs on
int setup_impl(const lsamg_csr* G, const lsamg_params* p, bool upload_now, lsamg_handle** out) {
  if (!G || !p || !out) return fail_with(LSAMG_EINVAL, "null argument");
  *out = nullptr;
  if (p->precision != LSAMG_FP64 && p->precision != LSAMG_MIXED)
    return fail_with(LSAMG_EINVAL, "bad precision");
  lsamg_handle* h = new (std::nothrow) lsamg_handle();
  if (!h) return fail_with(LSAMG_ENOMEM, "handle allocation failed");
  std::string msg;
  int rc = build_hierarchy(*G, *p, h->H, msg);
  if (rc != LSAMG_OK) {
    delete h;
    return fail_with(rc, msg);
  }
  h->precision = p->precision;
  h->device = upload_now ? p->device : -1;
  if (upload_now) {
    try {
      int ndev = 0;
      if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= p->device)
        throw DevError{LSAMG_ENODEV, "no such HIP device"};
      DeviceGuard g(p->device);
      upload(h);
      HIP_OK(hipDeviceSynchronize());
    } catch (const DevError& e) {
      h->free_all();
      delete h;
      return fail_with(e.code, e.msg);
    } catch (const std::bad_alloc&) {
      h->free_all();
      delete h;
      return fail_with(LSAMG_ENOMEM, "host allocation failed during upload");
    }
  }
  *out = h;
  return LSAMG_OK;
}

}  // namespace

extern "C" {

void lsamg_params_default(lsamg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->max_levels = 10;
  p->max_coarse = 2000;
  p->block = 4;
  p->omega_max = 800;
  p->n_eig_fixed = 0;
  p->kappa = 50.0;
  p->cmin[0] = 2;
  p->ncmin = 1;
  p->tie_rtol = 1e-8;
  p->tie_atol = 1e-12;
  p->pinv_rtol = 1e-6;
  p->thresh_margin = 1e-10;
  p->stall_ratio = 0.9;
  p->precision = LSAMG_FP64;
  p->device = 0;
  p->nthreads = 0;
  p->verbose = 0;
  p->dense_tail = 16384;
  p->aggregation = LSAMG_AGG_LATTICE;
  p->agg_passes[0] = 1;
  p->nagg_passes = 1;
  p->setup_device = LSAMG_SETUP_AUTO;
}

const char* lsamg_last_error(void) { return g_last_error.c_str(); }

int lsamg_setup(const lsamg_csr* G, const lsamg_params* p, lsamg_handle** out) {
  return setup_impl(G, p, p && p->device >= 0, out);
}

int lsamg_solve(lsamg_handle* h, const double* b, double* x, int32_t nrhs, int64_t ld, double tol,
                int32_t maxit, void* stream, lsamg_stats* stats) {
  if (!h || nrhs < 0 || maxit < 0 || !(tol >= 0.0)) return fail_with(LSAMG_EINVAL, "bad argument");
  if (nrhs == 0) return LSAMG_OK;
  if (!b || !x) return fail_with(LSAMG_EINVAL, "null vector");
  if (h->device < 0 || h->L.empty()) return fail_with(LSAMG_ENODEV, "handle has no device copy");
  const int64_t n = h->L[0].n;
  if (ld < n) return fail_with(LSAMG_EINVAL, "ld < n");
  try {
    DeviceGuard g(h->device);
    ProfGuard pg(&h->prof);
    hipStream_t s = (hipStream_t)stream;
    int rc = LSAMG_OK;
    if (nrhs == 1 || h->batch_mode == 0 || h->H.params.cycle == LSAMG_CYCLE_ADDITIVE) {
      for (int32_t c = 0; c < nrhs; ++c) {
        int r1 = pcg_one(h, b + (size_t)c * ld, x + (size_t)c * ld, tol, maxit, s,
                         stats ? stats + c : nullptr);
        if (r1 != LSAMG_OK) rc = r1;
      }
    } else {
      for (int32_t c0 = 0; c0 < nrhs; c0 += kBMax) {
        const int nr = std::min<int32_t>(kBMax, nrhs - c0);
        int r1 = h->krylov == LSAMG_KRYLOV_BLOCK
                     ? pcg_block(h, b + (size_t)c0 * ld, x + (size_t)c0 * ld, nr, ld, tol, maxit, s,
                                 stats ? stats + c0 : nullptr)
                     : solve_batched(h, b + (size_t)c0 * ld, x + (size_t)c0 * ld, nr, ld, tol,
                                     maxit, s, stats ? stats + c0 : nullptr);
        if (r1 != LSAMG_OK) rc = r1;
      }
    }
    if (rc == LSAMG_ENOCONV) g_last_error = "maximum iterations reached";
    return rc;
  } catch (const DevError& e) {
    return fail_with(e.code, e.msg);
  }
}

int lsamg_apply_op(lsamg_handle* h, int32_t op, const double* x, double* y, void* stream) {
  if (!h || !x || !y) return fail_with(LSAMG_EINVAL, "null argument");
  if (h->device < 0 || h->L.empty()) return fail_with(LSAMG_ENODEV, "handle has no device copy");
  if (op < LSAMG_OP_A || op > LSAMG_OP_VCYCLE) return fail_with(LSAMG_EINVAL, "bad op");
  DLevel& L0 = h->L[0];
  if ((op == LSAMG_OP_RAS || op == LSAMG_OP_RAST) && L0.coarsest)
    return fail_with(LSAMG_EINVAL, "single-level hierarchy has no smoother");
  try {
    DeviceGuard g(h->device);
    ProfGuard pg(&h->prof);
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = L0.n;
    const unsigned gb = nblocks(n);
    KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_perm_in, n, h->perm, x, h->bi);
    LAUNCH_OK();
    const bool mixed = h->precision == LSAMG_MIXED;
    if (op == LSAMG_OP_A) {
      apply_A(h, h->bi, h->z, s);
    } else if (op == LSAMG_OP_VCYCLE) {
      precondition(h, h->bi, h->z, s);
    } else if (mixed) {
      KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_convert<double, float>, n, h->bi, L0.f.b);
      LAUNCH_OK();
      if (op == LSAMG_OP_RAS) {
        ras<float>(L0, L0.f.b, L0.f.x, s);
      } else {
        HIP_OK(hipMemsetAsync(L0.f.x, 0, n * sizeof(float), s));
        ras_t_stage<float>(L0, L0.f.b, s);
        gather_add<float>(L0, L0.f.x, s);
      }
      KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_convert<float, double>, n, L0.f.x, h->z);
      LAUNCH_OK();
    } else {
      if (op == LSAMG_OP_RAS) {
        ras<double>(L0, h->bi, h->z, s);
      } else {
        KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_fill, n, 0.0, h->z);
        LAUNCH_OK();
        ras_t_stage<double>(L0, h->bi, s);
        gather_add<double>(L0, h->z, s);
      }
    }
    KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_perm_out, n, h->perm, h->z, y);
    LAUNCH_OK();
    HIP_OK(hipStreamSynchronize(s));
    return LSAMG_OK;
  } catch (const DevError& e) {
    return fail_with(e.code, e.msg);
  }
}

int lsamg_apply_op_noalloc(lsamg_handle* h, int32_t op, const double* x, double* y,
                           void* stream) {
  if (!h || !x || !y) return fail_with(LSAMG_EINVAL, "null argument");
  if (op < LSAMG_OP_A || op > LSAMG_OP_VCYCLE) return fail_with(LSAMG_EINVAL, "bad op");
  if (h->H.levels.empty()) return fail_with(LSAMG_EINVAL, "empty hierarchy");
  // staging in the per-GPU array: the permuted input and the output before
  // the permutation (n each), plus the rows of G x for op A
  const Level& H0 = h->H.levels[0];
  const int64_t n = H0.n;
  const int64_t rows = H0.G.total_rows();
  const int64_t need = 2 * n + (op == LSAMG_OP_A ? rows : 0);
  if (need > kScratchDoubles)
    return fail_with(LSAMG_EINVAL,
                     "lsamg_apply_op_noalloc: this operator needs " + std::to_string(need * 8) +
                         " bytes of staging, more than the " +
                         std::to_string((long long)LSAMG_NOALLOC_SCRATCH_BYTES) +
                         " bytes the allocation-free entry point holds per GPU");
  if (h->device < 0 || h->L.empty()) return fail_with(LSAMG_ENODEV, "handle has no device copy");
  DLevel& L0 = h->L[0];
  if ((op == LSAMG_OP_RAS || op == LSAMG_OP_RAST) && L0.coarsest)
    return fail_with(LSAMG_EINVAL, "single-level hierarchy has no smoother");
  if (L0.n != n || (op == LSAMG_OP_A && L0.nrows > rows))
    return fail_with(LSAMG_EINVAL, "device hierarchy does not match the host one");
  try {
    DeviceGuard g(h->device);
    hipStream_t s = (hipStream_t)stream;
    double* base = scratch_on(h->device);
    double* xi = base;                  // input in the internal numbering
    double* zo = base + n;              // output before the permutation
    double* gy = base + 2 * n;          // G x (op A)
    const unsigned gb = nblocks(n);
    KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_perm_in, n, h->perm, x, xi);
    LAUNCH_OK();
    const bool mixed = h->precision == LSAMG_MIXED;
    if (op == LSAMG_OP_A) {
      spmv_csr<double>(L0.nrows, L0.lanes_g, L0.g_ptr, L0.g_col, L0.d.g_val, xi, gy, s, L0.nnz,
                       L0.n);
      spmv_csr<double>(L0.n, L0.lanes_gt, L0.gt_ptr, L0.gt_col, L0.d.gt_val, gy, zo, s, L0.nnz,
                       L0.nrows);
    } else if (op == LSAMG_OP_VCYCLE) {
      precondition(h, xi, zo, s);       // kernels launched one by one, no graph
    } else if (mixed) {
      KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_convert<double, float>, n, xi, L0.f.b);
      LAUNCH_OK();
      if (op == LSAMG_OP_RAS) {
        ras<float>(L0, L0.f.b, L0.f.x, s);
      } else {
        KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_fill_f32, n, 0.0f, L0.f.x);
        LAUNCH_OK();
        ras_t_stage<float>(L0, L0.f.b, s);
        gather_add<float>(L0, L0.f.x, s);
      }
      KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_convert<float, double>, n, L0.f.x, zo);
      LAUNCH_OK();
    } else {
      if (op == LSAMG_OP_RAS) {
        ras<double>(L0, xi, zo, s);
      } else {
        KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_fill, n, 0.0, zo);
        LAUNCH_OK();
        ras_t_stage<double>(L0, xi, s);
        gather_add<double>(L0, zo, s);
      }
    }
    KLAUNCH0(gb, dev::kBlock, 0, s, dev::k_perm_out, n, h->perm, zo, y);
    LAUNCH_OK();
    return LSAMG_OK;
  } catch (const DevError& e) {
    return fail_with(e.code, e.msg);
  }
}

int lsamg_apply_vcycle_batch(lsamg_handle* h, const double* X, double* Y, int32_t nrhs,
                             int64_t ld, void* stream) {
  if (!h || !X || !Y || nrhs < 1 || nrhs > kBMax) return fail_with(LSAMG_EINVAL, "bad argument");
  if (h->device < 0 || h->L.empty()) return fail_with(LSAMG_ENODEV, "handle has no device copy");
  if (ld < h->L[0].n) return fail_with(LSAMG_EINVAL, "ld < n");
  if (h->H.params.cycle != LSAMG_CYCLE_V)
    return fail_with(LSAMG_EINVAL, "the multi-column cycle is the V-cycle");
  try {
    DeviceGuard g(h->device);
    ProfGuard pg(&h->prof);
    hipStream_t s = (hipStream_t)stream;
    if (nrhs <= 8)
      bapply_vcycle<8>(h, X, Y, nrhs, ld, s);
    else if (nrhs <= 16)
      bapply_vcycle<16>(h, X, Y, nrhs, ld, s);
    else if (nrhs <= 32)
      bapply_vcycle<32>(h, X, Y, nrhs, ld, s);
    else
      bapply_vcycle<64>(h, X, Y, nrhs, ld, s);
    return LSAMG_OK;
  } catch (const DevError& e) {
    return fail_with(e.code, e.msg);
  }
}

int lsamg_set_option(lsamg_handle* h, int32_t opt, int64_t value) {
  if (!h || value < 0 || (opt == LSAMG_OPT_DENSE_SPLIT && value > 17) ||
      (opt == LSAMG_OPT_BGROUP && value > 2) || (opt == LSAMG_OPT_ATA_TILES && value > 3) ||
      (opt == LSAMG_OPT_KRYLOV && value > 2) ||
      (opt != LSAMG_OPT_MFMA_TILE && opt != LSAMG_OPT_DENSE_SPLIT && opt != LSAMG_OPT_BGROUP &&
       opt != LSAMG_OPT_ATA_TILES && opt != LSAMG_OPT_KRYLOV && value > 1))
    return fail_with(LSAMG_EINVAL, "bad argument");
  if (opt == LSAMG_OPT_BATCHED) {
    h->batch_mode = (int)value;
  } else if (opt == LSAMG_OPT_MFMA) {
    h->use_mfma = value != 0;
    if (!h->use_mfma) {                 // back to k_bgemm; task lists stay until the buffers go
      for (auto& D : h->L) {
        for (GemvPlan* P : {&D.ras, &D.rast, &D.rst, &D.pro, &D.dense}) P->mm.rt = P->mmd.rt = 0;
        D.dmm_split = D.dmmd_split = 0;
        D.bg_on = false;
      }
      h->mm_tuned = false;
      h->mm_tuned64 = h->dmmd_tuned = false;
    }
    h->drop_graphs(true);               // captured batched V-cycles name the old kernels
  } else if (opt == LSAMG_OPT_GRAPH) {
    h->use_graphs = value != 0;
  } else if (opt == LSAMG_OPT_KRYLOV) {
    h->krylov = (int)value;
  } else if (opt == LSAMG_OPT_ONEPASS_ATA) {
    for (auto& D : h->L) D.fuse_ata = value != 0 && D.fuse_ok;
    h->drop_graphs(true);
  } else if (opt == LSAMG_OPT_BGROUP) {
    h->bgroup = (int)value;
    for (auto& D : h->L) D.bg_on = false;
    h->mm_tuned = false;                // decided again with the tiles on the next batched solve
    h->mm_tuned64 = h->dmmd_tuned = false;
    for (auto& D : h->L) {
      for (GemvPlan* P : {&D.ras, &D.rast, &D.rst, &D.pro, &D.dense}) P->mm.rt = P->mmd.rt = 0;
      D.dmm_split = D.dmmd_split = 0;
    }
    h->drop_graphs(true);
  } else if (opt == LSAMG_OPT_ATA_TILES) {
    for (auto& D : h->L) {
      D.at_on = value != 0 && D.at_ok;
      D.at_form = value >= 2 ? (int)value : 0;
      D.at1_on = value != 0 && D.at1_ok;
    }
    h->drop_graphs(true);
  } else if (opt == LSAMG_OPT_MFMA_TILE) {
    const int64_t rt = value / 100, u = (value / 10) % 10, sp = value % 10;
    if (value != 0 && (value >= 1000 || (rt != 1 && rt != 2 && rt != 4) ||
                       (u != 2 && u != 8 && !(u == 0 && rt == 4)) ||
                       (sp != 1 && sp != 2 && sp != 4 && sp != 8)))
      return fail_with(LSAMG_EINVAL, "bad tile shape");
    h->mm_fixed = (int)value;
    for (auto& D : h->L) {
      for (GemvPlan* P : {&D.ras, &D.rast, &D.rst, &D.pro, &D.dense}) P->mm.rt = P->mmd.rt = 0;
      D.dmm_split = D.dmmd_split = 0;
    }
    h->mm_tuned = false;                // retuned (or fixed) on the next batched solve
    h->mm_tuned64 = h->dmmd_tuned = false;
    h->drop_graphs(true);
  } else if (opt == LSAMG_OPT_DENSE_SPLIT) {
    h->dense_split = (int)value;
    for (auto& D : h->L) {
      for (GemvPlan* P : {&D.ras, &D.rast, &D.rst, &D.pro, &D.dense}) P->mm.rt = P->mmd.rt = 0;
      D.dmm_split = D.dmmd_split = 0;
    }
    h->mm_tuned = false;
    h->mm_tuned64 = h->dmmd_tuned = false;
    h->drop_graphs(true);
  } else {
    return fail_with(LSAMG_EINVAL, "unknown option");
  }
  return LSAMG_OK;
}

int lsamg_profile(lsamg_handle* h, int32_t mode, const char* only) {
  if (!h || mode < 0 || mode > 2) return fail_with(LSAMG_EINVAL, "bad argument");
  if (h->device < 0) return fail_with(LSAMG_ENODEV, "handle has no device copy");
  try {
    DeviceGuard g(h->device);
    Profiler& P = h->prof;
    if (mode != 0 && P.pool.empty()) {
      P.pool.resize(2 * 32768);
      for (auto& e : P.pool) HIP_OK(hipEventCreate(&e));
    }
    P.on = mode != 0;
    P.by_level = mode == 2;
    P.only = only ? only : "";
    return LSAMG_OK;
  } catch (const DevError& e) {
    return fail_with(e.code, e.msg);
  }
}

int lsamg_profile_read(lsamg_handle* h, lsamg_kprof* out, int32_t cap, int32_t* count) {
  if (!h || !count || cap < 0 || (cap > 0 && !out)) return fail_with(LSAMG_EINVAL, "bad argument");
  if (h->device < 0) return fail_with(LSAMG_ENODEV, "handle has no device copy");
  try {
    DeviceGuard g(h->device);
    Profiler& P = h->prof;
    HIP_OK(hipDeviceSynchronize());
    std::vector<std::string> names;
    std::vector<lsamg_kprof> acc;
    for (auto& r : P.recs) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
      size_t i = std::find(names.begin(), names.end(), r.name) - names.begin();
      if (i == names.size()) {
        names.push_back(r.name);
        lsamg_kprof k;
        std::memset(&k, 0, sizeof(k));
        std::strncpy(k.name, r.name.c_str(), sizeof(k.name) - 1);
        acc.push_back(k);
      }
      acc[i].launches += 1;
      acc[i].ms += ms;
      acc[i].bytes += r.bytes;
      acc[i].flops += r.flops;
    }
    P.recs.clear();
    P.used = 0;
    const int32_t nw = (int32_t)std::min<size_t>(acc.size(), (size_t)cap);
    for (int32_t i = 0; i < nw; ++i) out[i] = acc[i];
    *count = nw;
    return LSAMG_OK;
  } catch (const DevError& e) {
    return fail_with(e.code, e.msg);
  }
}

int lsamg_set_precision(lsamg_handle* h, int32_t precision) {
  if (!h || (precision != LSAMG_FP64 && precision != LSAMG_MIXED))
    return fail_with(LSAMG_EINVAL, "bad argument");
  h->precision = precision;
  return LSAMG_OK;
}

int lsamg_info_get(const lsamg_handle* h, lsamg_info* out) {
  if (!h || !out) return fail_with(LSAMG_EINVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  const Hierarchy& H = h->H;
  out->nlevels = (int32_t)std::min<size_t>(H.levels.size(), 16);
  out->n0 = H.levels.empty() ? 0 : H.levels[0].n;
  out->m0 = H.m0;
  out->setup_seconds = H.setup_seconds;
  out->device_bytes = h->bytes;
  double a0 = H.levels.empty() ? 1.0 : (double)std::max<int64_t>(1, H.levels[0].a_nnz);
  double oc = 0, sc = 0;
  for (int l = 0; l < out->nlevels; ++l) {
    const Level& L = H.levels[l];
    lsamg_level_info& I = out->level[l];
    I.n = L.n;
    I.nagg = L.nagg;
    for (int64_t g = 0; g < L.G.ng(); ++g) {
      const int64_t c = L.G.sptr[g + 1] - L.G.sptr[g];
      const int r = L.G.nrows[g];
      I.g_rows += r;
      I.g_nnz += (r > 1) ? (int64_t)r * c - (int64_t)r * (r - 1) / 2 : c;
    }
    I.a_nnz = L.a_nnz;
    oc += (double)L.a_nnz / a0;
    if (!L.coarsest) {
      for (int64_t a = 0; a < L.nagg; ++a)
        I.smoother_entries += (L.astart[a + 1] - L.astart[a]) * (L.optr[a + 1] - L.optr[a]);
      I.p_entries = (int64_t)L.Zhat.size();
      I.block = L.block;
      I.n_color = L.n_color;
      I.n_mult = L.n_mult;
      I.kmin = L.k.empty() ? 0 : *std::min_element(L.k.begin(), L.k.end());
      I.kmax = L.k.empty() ? 0 : *std::max_element(L.k.begin(), L.k.end());
      I.thresh = L.thresh;
      I.hazards = L.hazards;
      sc += (double)I.smoother_entries / a0;
    }
  }
  out->op_complexity = oc;
  out->smoother_complexity = sc;
  out->tail_level = -1;
  for (size_t l = 0; l < h->L.size(); ++l)
    if (h->L[l].tail) out->tail_level = (int32_t)l;
  return LSAMG_OK;
}

int lsamg_export_setup(lsamg_handle* h, int32_t level, lsamg_setup_view* out) {
  if (!h || !out) return fail_with(LSAMG_EINVAL, "null argument");
  if (level < 0 || level >= (int32_t)h->H.levels.size())
    return fail_with(LSAMG_EINVAL, "bad level");
  const Level& L = h->H.levels[level];
  std::memset(out, 0, sizeof(*out));
  out->n = L.n;
  if (L.coarsest) return LSAMG_OK;
  out->nagg = L.nagg;
  h->ex_agg.assign(L.n, -1);
  for (int64_t a = 0; a < L.nagg; ++a)
    for (int64_t d = L.astart[a]; d < L.astart[a + 1]; ++d) h->ex_agg[L.canon[d]] = (int32_t)a;
  h->ex_optr = L.optr;
  h->ex_oidx.resize(L.oidx.size());
  for (int64_t a = 0; a < L.nagg; ++a) {
    const int64_t o0 = L.optr[a], nw = L.astart[a + 1] - L.astart[a];
    for (int64_t o = o0; o < L.optr[a + 1]; ++o) h->ex_oidx[o] = L.canon[L.oidx[o]];
    std::sort(h->ex_oidx.begin() + o0, h->ex_oidx.begin() + o0 + nw);
    std::sort(h->ex_oidx.begin() + o0 + nw, h->ex_oidx.begin() + L.optr[a + 1]);
  }
  h->ex_k = L.k;
  h->ex_mu = L.mu;
  h->ex_muptr = L.muptr;
  out->agg = h->ex_agg.data();
  out->optr = h->ex_optr.data();
  out->oidx = h->ex_oidx.data();
  out->k = h->ex_k.data();
  out->mu = h->ex_mu.data();
  out->muptr = h->ex_muptr.data();
  if (level == 0) {
    h->ex_M = L.M;
    out->M = h->ex_M.data();
  }
  out->block = L.block;
  out->n_color = L.n_color;
  out->n_mult = L.n_mult;
  out->thresh = L.thresh;
  return LSAMG_OK;
}

size_t lsamg_device_bytes(const lsamg_handle* h) { return h ? h->bytes : 0; }

void lsamg_destroy(lsamg_handle* h) {
  if (!h) return;
  if (h->device >= 0) {
    int old = -1;
    (void)hipGetDevice(&old);
    (void)hipSetDevice(h->device);
    h->free_all();
    if (old >= 0) (void)hipSetDevice(old);
  }
  delete h;
}

}  // extern "C"

// ===========================================================================
// Continuous-batching server (lsamg_server_*)
// ===========================================================================
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct SReq {
  lsamg_request r;
  std::vector<double> b;
  int64_t n = 0;
  double t_submit = 0;
  // while solving
  double t_taken = 0, t_setup = 0;
  int hit = 0, joined_at = 0, batch_max = 0, cols_left = 0;
  bool posted = false;
  int col[64];                 // engine column of each right-hand side
};

struct SEntry {
  lsamg_handle* h = nullptr;
  size_t bytes = 0;
  bool ready = false, busy = false, failed = false;
  int err = 0;
  std::string msg;
  uint64_t last_use = 0;
};

// Device bytes a multi-right-hand-side solve of width NB may add to h: the
// batched buffers (when not yet sized for NB, exactly as ensure_batched
// makes them) and, while a width or precision is not tuned yet, an upper
// bound of what the autotuners keep (split-loop partial sums, the dense
// level's padded copies, task lists) plus their 512 MiB cache-flush buffer.
size_t batched_reserve(const lsamg_handle* h, int NB) {
  size_t b = 0;
  auto add = [&](int64_t count, size_t sz) { b += (size_t)std::max<int64_t>(count, 1) * sz; };
  const bool fresh = !(h->batched_ready && h->bwidth >= NB);
  const int64_t W = fresh ? NB : h->bwidth;
  if (fresh) {
    for (const DLevel& L : h->L) {
      const int64_t n = L.n * W, ny = std::max<int64_t>(L.nrows, 1) * W,
                    nt = std::max<int64_t>(L.ntb, 1) * W;
      for (int k = 0; k < 3; ++k) add(n, 8);
      add(ny, 8);
      add(nt, 8);
      for (int k = 0; k < 3; ++k) add(n, 4);
      add(ny, 4);
      add(nt, 4);
      if (L.bg_ok) add(L.bg_nstg * W, 4);
    }
    const int64_t n0 = h->L[0].n * W;
    for (int k = 0; k < 6; ++k) add(n0, 8);
    for (int k = 0; k < 6; ++k) add(kBNP * W, 8);
    for (int k = 0; k < 6; ++k) add(W, 8);
    add(192, 4);
  }
  // the autotuners run on the first FP32 solve of >= 16 columns (and again
  // on the first of 64) and on the first FP64 solve of 64 columns; buffers
  // made afresh drop what was tuned before
  const bool mixed = h->precision == LSAMG_MIXED;
  const bool tune = h->use_mfma &&
                    (mixed ? NB >= 16 && (fresh || !h->mm_tuned || (NB == 64 && !h->mm_tuned64))
                           : NB == 64 && (fresh || !h->dmmd_tuned));
  if (tune) {
    int64_t cap = 0;
    for (size_t l = 0; l < h->L.size(); ++l) {
      const DLevel& L = h->L[l];
      if (L.coarsest || L.tail) {
        cap = std::max<int64_t>(cap, 16 * L.n * W);
        const int64_t ld = (L.n + 3) / 4 * 4;
        add(L.n * ld, 4);                  // padded FP32 copy (k_dense_mm64)
        add(L.n * ld, 8);                  // padded FP64 copy (k_dense_mm64d)
        add(16 * L.n * 64, 8);             // its partial sums
        add(5 * 16 * 2 * (L.n / 16 + 2), 4);
        break;
      }
      if (l > 0) cap = std::max<int64_t>(cap, 4 * std::max(L.n, L.ntb) * W);
      for (const GemvPlan* P : {&L.ras, &L.rast, &L.rst, &L.pro})
        add(5 * 16 * 2 * (P->out / 16 + P->nagg + 1), 4);   // k_bmm and k_bmmd task lists
    }
    add(cap, 4);
    b += (size_t)512 << 20;                // the tuners' flush buffer (freed after)
  }
  return b + b / 50 + ((size_t)1 << 20);
}

}  // namespace

// HBM a device setup may hold while it runs (its batches' blocks, at most
// 2^31 doubles, plus the factorisations' workspace), admitted by the server
// for the duration of a setup on the device
constexpr size_t kSetupTransient = (size_t)24 << 30;

struct lsamg_server {
  int device = 0;
  size_t budget = 0;
  int slots = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SReq> queue;
  std::unordered_map<uint64_t, SEntry> cache;
  std::deque<lsamg_done> done;
  std::vector<std::thread> workers;
  bool stop = false;
  size_t resident = 0, peak = 0;
  uint64_t tick = 0;
  int64_t submitted = 0, completed = 0, hits = 0, misses = 0, evictions = 0, joins = 0,
          reserve_misses = 0;
  std::atomic<int64_t> iterations{0};    // PCG iterations run by all solves
  int active = 0, waiting = 0;

  void account(size_t add, size_t sub) {
    resident = resident + add - sub;
    peak = std::max(peak, resident);
  }

  // post a completion (lock held)
  void post(const SReq& q, int status, int its, double trr, double t_solve,
            const std::string& msg = std::string()) {
    lsamg_done d;
    std::memset(&d, 0, sizeof(d));
    std::snprintf(d.msg, sizeof(d.msg), "%s", msg.c_str());
    d.id = q.r.id;
    d.status = status;
    d.cache_hit = q.hit;
    d.batch_rhs = q.batch_max;
    d.iters_max = its;
    d.true_rel_res_max = trr;
    d.t_queue = q.t_taken - q.t_submit;
    d.t_setup = q.t_setup;
    d.t_solve = t_solve;
    d.t_total = now_s() - q.t_submit;
    d.joined_at = q.joined_at;
    done.push_back(d);
    ++completed;
    cv_done.notify_all();
  }

  // evict the least-recently-used idle hierarchy (lock held); false if none
  bool evict_one() {
    auto best = cache.end();
    for (auto it = cache.begin(); it != cache.end(); ++it)
      if (it->second.ready && !it->second.busy &&
          (best == cache.end() || it->second.last_use < best->second.last_use))
        best = it;
    if (best == cache.end()) return false;
    lsamg_handle* h = best->second.h;
    account(0, best->second.bytes);
    cache.erase(best);
    ++evictions;
    lsamg_destroy(h);
    return true;
  }

  // make room for `need` more bytes (lock held): evict idle hierarchies,
  // else wait for running solves to release memory.  False when it cannot
  // fit: more than the budget, or every other slot is waiting as well.
  bool make_room(std::unique_lock<std::mutex>& lk, size_t need) {
    while (resident + need > budget) {
      if (evict_one()) continue;
      if (need > budget || waiting + 1 >= active) return false;
      ++waiting;
      cv_done.wait_for(lk, std::chrono::milliseconds(50));
      --waiting;
    }
    return true;
  }

  void worker();
  template <int NB>
  void session(std::unique_lock<std::mutex>& lk, uint64_t key, SReq first, hipStream_t st,
               double*& stage, size_t& stage_cap);
};

// One multi-right-hand-side PCG of width NB on operator `key`, with the
// lock held on entry and exit.  Requests for the operator that arrive while
// it runs are loaded into free columns at the next iteration boundary and
// start their own CG there; each request is reported as soon as its last
// column finishes, and its columns take new requests.  The solve ends when
// no column is active and no queued request for the operator fits (or it
// drains for a wider solve, see admit).
template <int NB>
void lsamg_server::session(std::unique_lock<std::mutex>& lk, uint64_t key, SReq first,
                           hipStream_t st, double*& stage, size_t& stage_cap) {
  SEntry* e = &cache[key];
  lsamg_handle* h = e->h;
  const int64_t n = first.n;
  std::vector<std::unique_ptr<SReq>> live;
  SReq* owner[NB] = {};
  int iter = 0;
  auto free_cols = [&]() {
    int k = 0;
    for (int j = 0; j < NB; ++j) k += owner[j] == nullptr;
    return k;
  };
  auto take = [&](SReq&& q) {          // lock held
    live.push_back(std::make_unique<SReq>(std::move(q)));
    SReq* p = live.back().get();
    int c = 0;
    for (int j = 0; j < NB && c < p->r.nrhs; ++j)
      if (!owner[j]) {
        owner[j] = p;
        p->col[c++] = j;
      }
    p->cols_left = p->r.nrhs;
    p->joined_at = iter;
    p->t_taken = now_s();
    return p;
  };
  // queued requests for this operator, first come first served, while they
  // fit the free columns (a request that does not fit stops the scan, so
  // narrower later ones cannot starve it).  When the columns still waiting
  // amount to a full batch of this width, the solve stops taking requests
  // and drains: the next solve on the operator starts at the width the
  // queue then asks for (lock held)
  bool draining = false;
  auto admit = [&](std::vector<SReq*>& fresh) {
    if (draining) return;
    int waiting = 0;
    for (size_t i = 0; i < queue.size();) {
      if (queue[i].r.op_key != key || queue[i].n != n) {
        ++i;
      } else if (waiting == 0 && queue[i].r.nrhs <= free_cols()) {
        SReq* p = take(std::move(queue[i]));
        p->hit = 1;
        if (iter > 0) ++joins;
        fresh.push_back(p);
        queue.erase(queue.begin() + i);
      } else {
        waiting += queue[i].r.nrhs;
        ++i;
      }
    }
    if (NB < 64 && waiting >= NB) draining = true;
  };
  std::vector<SReq*> fresh;
  fresh.push_back(take(std::move(first)));
  admit(fresh);
  lk.unlock();
  int rc = LSAMG_OK;
  std::string msg;
  try {
    DeviceGuard g(device);
    BatchCG<NB> E(h, st);
    for (;;) {
      // load the newly taken requests' columns through the staging buffer
      for (SReq* p : fresh) {
        const size_t need = (size_t)n * p->r.nrhs;
        if (need > stage_cap) throw DevError{LSAMG_EINVAL, "staging smaller than a request"};
        HIP_OK(hipMemcpyAsync(stage, p->b.data(), need * sizeof(double), hipMemcpyHostToDevice,
                              st));
        for (int c = 0; c < p->r.nrhs; ++c)
          E.load(p->col[c], 1, stage + (size_t)c * n, n, p->r.tol, p->r.maxit);
        // the next copy into the staging waits for these loads (same stream)
      }
      fresh.clear();
      E.norms();
      const int nact = E.nactive();
      // collect finished columns; report requests whose columns are all done
      std::vector<SReq*> finished;
      for (auto& up : live) {
        SReq* p = up.get();
        if (p->cols_left == 0) continue;
        int left = 0;
        bool bad = false;
        for (int c = 0; c < p->r.nrhs; ++c) {
          const BCol& q = E.c[p->col[c]];
          left += !q.done;
          bad = bad || q.bad;
        }
        p->batch_max = std::max(p->batch_max, nact);
        if (bad) {                       // a non-finite right-hand side: drop the request
          for (int c = 0; c < p->r.nrhs; ++c) {
            E.c[p->col[c]].active = 0;
            E.c[p->col[c]].done = 1;
          }
          left = 0;
        }
        p->cols_left = left;
        if (left == 0) finished.push_back(p);
      }
      for (SReq* p : finished) {
        int its = 0, status = LSAMG_OK;
        double trr = 0;
        bool bad = false;
        for (int c = 0; c < p->r.nrhs; ++c) {
          const BCol& q = E.c[p->col[c]];
          E.store(p->col[c], 1, stage + (size_t)c * n, n);
          its = std::max(its, q.its);
          trr = std::max(trr, q.nb > 0 ? q.tr / q.nb : 0.0);
          if (!q.conv) status = LSAMG_ENOCONV;
          bad = bad || q.bad;
        }
        if (bad) status = LSAMG_EBADINPUT;
        HIP_OK(hipMemcpyAsync(p->r.x, stage, (size_t)n * p->r.nrhs * sizeof(double),
                              hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        const double ts = now_s() - p->t_taken;
        lk.lock();
        for (int c = 0; c < p->r.nrhs; ++c) owner[p->col[c]] = nullptr;
        post(*p, status, its, trr, ts);
        p->posted = true;
        lk.unlock();
      }
      lk.lock();
      admit(fresh);
      const bool more = std::any_of(queue.begin(), queue.end(),
                                    [&](const SReq& q) { return q.r.op_key == key; });
      lk.unlock();
      if (!fresh.empty()) continue;      // load them before the next iteration
      if (E.nactive() == 0) break;
      E.prepare();
      E.step(more);
      ++iter;
      ++iterations;
    }
  } catch (const DevError& de) {
    rc = de.code;
    msg = de.msg;
  }
  lk.lock();
  if (rc != LSAMG_OK) {                  // every request still in the solve fails with it
    for (auto& up : live)
      if (!up->posted) post(*up, rc, 0, 0, now_s() - up->t_taken, msg);
  }
}

void lsamg_server::worker() {
  (void)hipSetDevice(device);
  hipStream_t st = nullptr;
  (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  double* stage = nullptr;               // n x 64 doubles of request columns in and out
  size_t stage_cap = 0;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    // first queued request whose operator is resident and idle, or unknown
    size_t pick = queue.size();
    bool miss = false;
    for (size_t i = 0; i < queue.size(); ++i) {
      auto it = cache.find(queue[i].r.op_key);
      if (it == cache.end()) {
        pick = i;
        miss = true;
        break;
      }
      if (it->second.failed || (it->second.ready && !it->second.busy)) {
        pick = i;
        break;
      }
    }
    if (pick == queue.size()) {
      if (stop && queue.empty() && active == 0) break;
      cv_work.wait_for(lk, std::chrono::milliseconds(50));
      continue;
    }
    SReq first = std::move(queue[pick]);
    queue.erase(queue.begin() + pick);
    const uint64_t key = first.r.op_key;
    ++active;
    first.t_taken = now_s();
    if (!miss && cache[key].failed) {
      post(first, cache[key].err, 0, 0, 0, cache[key].msg);
      --active;
      cv_work.notify_all();
      continue;
    }
    SEntry* e = nullptr;
    if (miss) {
      ++misses;
      e = &cache[key];
      e->busy = true;
      // a setup on the device holds transient buffers (batches of at most
      // 8 GiB of blocks, plus the factorisations' workspace): admitted
      // against the budget for its duration
      lsamg_params p = *first.r.params;
      p.device = device;
      bool on_dev = setup_on_device(p, first.r.G->n);
      bool room = !on_dev || make_room(lk, kSetupTransient);
      if (on_dev && !room && p.setup_device == LSAMG_SETUP_AUTO) {
        on_dev = false;                    // no room: the host does the setup
        room = true;
      }
      if (on_dev) account(kSetupTransient, 0);
      lk.unlock();
      p.setup_device = on_dev ? LSAMG_SETUP_DEVICE : LSAMG_SETUP_HOST;
      p.device = on_dev ? device : -1;     // upload only after admission
      lsamg_handle* h = nullptr;
      int rc = room ? setup_impl(first.r.G, &p, false, &h) : LSAMG_ENOMEM;
      std::string msg = rc == LSAMG_OK ? "" : room ? lsamg_last_error()
                                                  : "no room in the device budget for the setup";
      if (on_dev) {
        std::lock_guard<std::mutex> g(mu);
        account(0, kSetupTransient);
      }
      size_t need = 0;
      if (rc == LSAMG_OK) {
        h->device = device;
        h->precision = first.r.params->precision;
        try {
          need = planned_device_bytes(h);
        } catch (const DevError& de) {
          rc = de.code;
          msg = de.msg;
        }
      }
      lk.lock();
      e = &cache[key];
      // admission against the budget: evict idle hierarchies, else wait for
      // running solves to finish; a hierarchy larger than the budget fails
      if (rc == LSAMG_OK && !make_room(lk, need)) {
        rc = LSAMG_ENOMEM;
        msg = "hierarchy does not fit the device budget";
      }
      e = &cache[key];
      if (rc == LSAMG_OK) {
        account(need, 0);                  // reserve before uploading
        lk.unlock();
        try {
          DeviceGuard g(device);
          upload(h);                       // synchronous copies: nothing pending
        } catch (const DevError& de) {
          rc = de.code;
          msg = de.msg;
        }
        lk.lock();
        e = &cache[key];
        account(h->bytes, need);
      }
      if (rc != LSAMG_OK) {
        if (h) lsamg_destroy(h);
        e->failed = true;
        e->busy = false;
        e->err = rc;
        e->msg = msg;
        first.t_setup = now_s() - first.t_taken;
        post(first, rc, 0, 0, 0, msg);
        --active;
        cv_work.notify_all();
        continue;
      }
      e->h = h;
      e->bytes = h->bytes;
      e->ready = true;
      first.t_setup = now_s() - first.t_taken;
    } else {
      ++hits;
      first.hit = 1;
      e = &cache[key];
      e->busy = true;
    }
    // width of the solve: room for the columns queued for this operator now
    // and as many again arriving while it runs
    int cols = first.r.nrhs;
    for (const SReq& q : queue)
      if (q.r.op_key == key) cols += q.r.nrhs;
    int NB = 8;
    while (NB < 64 && NB < std::min(64, 2 * cols)) NB *= 2;
    NB = std::max(NB, first.r.nrhs <= 8 ? 8 : first.r.nrhs <= 16 ? 16 : first.r.nrhs <= 32 ? 32 : 64);
    // admission of the solve's own device memory (batched buffers, tuning,
    // request staging), narrower widths first if the widest does not fit
    lsamg_handle* h = e->h;
    const size_t stage_need = (size_t)first.n * 64 * sizeof(double);
    const size_t stage_grow = stage_need > stage_cap * sizeof(double) ? stage_need - stage_cap * sizeof(double) : 0;
    size_t reserve = 0;
    bool fits = false;
    for (; NB >= 8; NB /= 2) {
      if (NB < first.r.nrhs) break;
      reserve = batched_reserve(h, NB) + stage_grow;
      if (make_room(lk, reserve)) {
        fits = true;
        break;
      }
    }
    e = &cache[key];
    if (!fits) {
      e->busy = false;
      e->last_use = ++tick;
      post(first, LSAMG_ENOMEM, 0, 0, 0, "the solve's device memory does not fit the budget");
      --active;
      cv_work.notify_all();
      continue;
    }
    account(reserve, 0);
    const size_t before = h->bytes;
    if (stage_grow > 0) {
      lk.unlock();
      bool ok = true;
      {
        DeviceGuard g(device);
        if (stage) (void)hipFree(stage);
        stage = nullptr;
        stage_cap = 0;
        if (hipMalloc(&stage, stage_need) != hipSuccess) {
          (void)hipGetLastError();
          stage = nullptr;
          ok = false;
        }
      }
      lk.lock();
      if (!ok) {
        account(0, reserve);
        e = &cache[key];
        e->busy = false;
        post(first, LSAMG_ENOMEM, 0, 0, 0, "staging allocation failed");
        --active;
        cv_work.notify_all();
        continue;
      }
      stage_cap = (size_t)first.n * 64;
    }
    switch (NB) {
      case 8: session<8>(lk, key, std::move(first), st, stage, stage_cap); break;
      case 16: session<16>(lk, key, std::move(first), st, stage, stage_cap); break;
      case 32: session<32>(lk, key, std::move(first), st, stage, stage_cap); break;
      default: session<64>(lk, key, std::move(first), st, stage, stage_cap); break;
    }
    // replace the reservation by what the solve really added
    e = &cache[key];
    const size_t grown = h->bytes > before ? h->bytes - before : 0;
    if (grown + stage_grow > reserve) ++reserve_misses;
    account(h->bytes + stage_grow, before + reserve);
    e->bytes = h->bytes;
    e->busy = false;
    e->last_use = ++tick;
    --active;
    cv_work.notify_all();
  }
  lk.unlock();
  if (stage) (void)hipFree(stage);
  if (st) (void)hipStreamDestroy(st);
}

extern "C" {

int lsamg_server_create(int32_t device, size_t hbm_budget, int32_t max_slots,
                        lsamg_server** out) {
  if (!out || max_slots < 1 || max_slots > 64 || hbm_budget == 0)
    return fail_with(LSAMG_EINVAL, "bad argument");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail_with(LSAMG_ENODEV, "no such HIP device");
  // the device setup's libraries are opened now, before any worker launches
  // kernels: opening them later, in one worker, while another launches, has
  // made those launches fail ("invalid device function").  Without them a
  // setup on the device fails with its own message, and host setups work.
  {
    std::string pmsg;
    (void)device_setup_preload(device, pmsg);
  }
  lsamg_server* s = new (std::nothrow) lsamg_server();
  if (!s) return fail_with(LSAMG_ENOMEM, "server allocation failed");
  s->device = device;
  s->budget = hbm_budget;
  s->slots = max_slots;
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([s]() { s->worker(); });
  *out = s;
  return LSAMG_OK;
}

int lsamg_server_submit(lsamg_server* s, const lsamg_request* req) {
  if (!s || !req || !req->G || !req->params || !req->b || !req->x || req->nrhs < 1 ||
      req->nrhs > 64 || req->maxit < 0 || !(req->tol >= 0.0) || req->G->n <= 0)
    return fail_with(LSAMG_EINVAL, "bad request");
  if (req->params->cycle != LSAMG_CYCLE_V)
    return fail_with(LSAMG_EINVAL, "the server solves with the V-cycle");
  SReq q;
  q.r = *req;
  q.n = req->G->n;
  q.b.assign(req->b, req->b + (size_t)q.n * req->nrhs);
  q.t_submit = now_s();
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return fail_with(LSAMG_EINVAL, "server is stopping");
  s->queue.push_back(std::move(q));
  ++s->submitted;
  s->cv_work.notify_one();
  return LSAMG_OK;
}

int lsamg_server_poll(lsamg_server* s, lsamg_done* out, int32_t cap, int32_t* count,
                      int32_t wait_ms) {
  if (!s || !count || cap < 0 || (cap > 0 && !out)) return fail_with(LSAMG_EINVAL, "bad argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [s] { return !s->done.empty(); });
  int32_t k = 0;
  while (k < cap && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *count = k;
  return LSAMG_OK;
}

int lsamg_server_stats_get(lsamg_server* s, lsamg_server_stats* out) {
  if (!s || !out) return fail_with(LSAMG_EINVAL, "bad argument");
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->hits = s->hits;
  out->misses = s->misses;
  out->evictions = s->evictions;
  out->joins = s->joins;
  out->iterations = s->iterations.load();
  out->reserve_misses = s->reserve_misses;
  out->resident_bytes = s->resident;
  out->peak_bytes = s->peak;
  out->budget = s->budget;
  out->queued = (int32_t)s->queue.size();
  out->active = s->active;
  return LSAMG_OK;
}

void lsamg_server_destroy(lsamg_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->cache)
    if (kv.second.h) lsamg_destroy(kv.second.h);
  delete s;
}

}  // extern "C"
