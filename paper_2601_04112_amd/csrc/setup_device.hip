// Setup on the HIP device: the dense local problems of Algorithm 1 (sec. 3.2)
// for a batch of aggregates at once, in FP64.
//
// Per aggregate i (sec. 3.1.1, eq:gevp, eq:gevp-S):
//   1. the pseudo-inverse Schur complement S~ = B_w^T (I - Q Q^T) B_w, with
//      B = W^{1/2} G_{nz_i} split into its Gamma_i columns B_Gamma and its
//      omega_i columns B_w, and Q the left singular vectors of B_Gamma whose
//      singular values exceed rtol times the largest.  Blocks with at least
//      as many rows as columns are first reduced by a batched Householder QR
//      of [B_Gamma B_w] to its R factor [R11 R12; 0 R22] (the SVD is then
//      that of R11, and the R22 part is added as R22^T R22), as the host
//      setup does; otherwise the SVD is that of B_Gamma.  The dropped
//      vectors are zeroed, then C = Q^T B_w, E = B_w - Q C and S~ = E^T E
//      are batched GEMMs;
//   2. the reduced eigenproblem S~ u = mu A_ww u through the Cholesky factor
//      A_ww = L L^T: C = L^{-1} S~ L^{-T} (batched triangular solves),
//      symmetrised, then the batched eigensolver (Jacobi for blocks of up
//      to 64 unknowns, divide and conquer above; ascending mu) and
//      u = L^{-T} y;
//   3. the smoother rows: A_i = A(Omega_i, Omega_i) = L_i L_i^T and the
//      columns A_i^{-1} e_j for j in omega_i (or all of A_i^{-1} for the
//      additive cycle) from the batched Cholesky solve.
// Blocks of one batch share padded sizes: zero rows and columns in B (they
// add zero singular values, below any cut), identity on the padded diagonal
// of A_ww and A_i (block-diagonal factors, exact zeros off the true block),
// and on the padded diagonal of C a value above every true eigenvalue (the
// Gershgorin bound of the true block), so the true eigenpairs come first in
// ascending order with exact zeros in their padded entries.
//
// The dense factorisations are rocSOLVER's and the products rocBLAS's; both
// libraries are opened with dlopen on the first call, so the library loads
// on hosts without them and only the device setup needs them.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace lsamg {
namespace {

struct SetupDevError {
  int code;
  std::string msg;
};

#define SD_HIP(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw SetupDevError{e_ == hipErrorOutOfMemory ? LSAMG_ENOMEM : LSAMG_EHIP,      \
                          std::string(#expr) + ": " + hipGetErrorString(e_)};         \
  } while (0)

#define SD_ROC(expr)                                                                  \
  do {                                                                                \
    rocblas_status st_ = (expr);                                                      \
    if (st_ != rocblas_status_success)                                                \
      throw SetupDevError{st_ == rocblas_status_memory_error ? LSAMG_ENOMEM : LSAMG_EHIP, \
                          std::string(#expr) + ": rocBLAS/rocSOLVER status " +        \
                              std::to_string((int)st_)};                              \
  } while (0)

// rocBLAS / rocSOLVER entry points, resolved on first use
struct RocApi {
  decltype(&rocblas_create_handle) create_handle = nullptr;
  decltype(&rocblas_destroy_handle) destroy_handle = nullptr;
  decltype(&rocblas_set_stream) set_stream = nullptr;
  decltype(&rocblas_dgemm_strided_batched) gemm = nullptr;
  decltype(&rocblas_dtrsm_strided_batched) trsm = nullptr;
  decltype(&rocsolver_dgesvd_strided_batched) gesvd = nullptr;
  decltype(&rocsolver_dgeqrf_strided_batched) geqrf = nullptr;
  decltype(&rocsolver_dpotrf_strided_batched) potrf = nullptr;
  decltype(&rocsolver_dpotrs_strided_batched) potrs = nullptr;
  decltype(&rocsolver_dsyevj_strided_batched) syevj = nullptr;
  decltype(&rocsolver_dsyevd_strided_batched) syevd = nullptr;
  bool ok = false;
  std::string err;
};

void* open_first(const char* const* names, std::string& tried) {
  for (const char* const* n = names; *n; ++n) {
    void* h = dlopen(*n, RTLD_NOW | RTLD_LOCAL);
    if (h) return h;
    tried += std::string(" ") + *n;
  }
  return nullptr;
}

const RocApi& roc_api() {
  static RocApi api;
  static std::once_flag once;
  std::call_once(once, [] {
    std::string root = "/opt/rocm";
    if (const char* e = std::getenv("ROCM_PATH")) root = e;
    const std::string b0 = root + "/lib/librocblas.so.5", s0 = root + "/lib/librocsolver.so.0";
    const char* bn[] = {b0.c_str(), "librocblas.so.5", "librocblas.so", nullptr};
    const char* sn[] = {s0.c_str(), "librocsolver.so.0", "librocsolver.so", nullptr};
    std::string tried;
    void* hb = open_first(bn, tried);
    void* hs = hb ? open_first(sn, tried) : nullptr;
    if (!hb || !hs) {
      api.err = "setup on the device: cannot open rocBLAS/rocSOLVER (tried" + tried + ")";
      return;
    }
    bool all = true;
    auto get = [&](void* h, const char* nm, auto& fp) {
      fp = reinterpret_cast<std::remove_reference_t<decltype(fp)>>(dlsym(h, nm));
      if (!fp) {
        all = false;
        api.err = std::string("setup on the device: missing symbol ") + nm;
      }
    };
    get(hb, "rocblas_create_handle", api.create_handle);
    get(hb, "rocblas_destroy_handle", api.destroy_handle);
    get(hb, "rocblas_set_stream", api.set_stream);
    get(hb, "rocblas_dgemm_strided_batched", api.gemm);
    get(hb, "rocblas_dtrsm_strided_batched", api.trsm);
    get(hs, "rocsolver_dgesvd_strided_batched", api.gesvd);
    get(hs, "rocsolver_dgeqrf_strided_batched", api.geqrf);
    get(hs, "rocsolver_dpotrf_strided_batched", api.potrf);
    get(hs, "rocsolver_dpotrs_strided_batched", api.potrs);
    get(hs, "rocsolver_dsyevj_strided_batched", api.syevj);
    get(hs, "rocsolver_dsyevd_strided_batched", api.syevd);
    api.ok = all;
  });
  return api;
}

// Zero the columns of U (R x mn per aggregate) whose singular value is not
// above rtol times the largest (or is zero); rank[b] = columns kept.  One
// workgroup per aggregate.
__global__ void __launch_bounds__(256) k_keep_mask(int R, int mn, double rtol,
                                                   const double* __restrict__ S,
                                                   double* __restrict__ U,
                                                   int32_t* __restrict__ rank) {
  __shared__ double red[256];
  __shared__ int cnt;
  const int b = blockIdx.x, t = threadIdx.x;
  const double* s = S + (size_t)b * mn;
  double* u = U + (size_t)b * R * mn;
  double m = 0.0;
  for (int j = t; j < mn; j += 256) m = fmax(m, fabs(s[j]));
  red[t] = m;
  if (t == 0) cnt = 0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double cut = rtol * red[0];
  for (int j = 0; j < mn; ++j) {
    const double sj = fabs(s[j]);
    if (sj > cut && sj != 0.0) {
      if (t == 0) ++cnt;
      continue;
    }
    for (int i = t; i < R; i += 256) u[(size_t)j * R + i] = 0.0;
  }
  __syncthreads();
  if (t == 0) rank[b] = cnt;
}

// From the Householder QR of B (R x (Gm + W) per aggregate, R factor in the
// upper triangle): R11 (Gm x Gm) and R22 (W x W, rows and columns Gm ..
// Gm + W - 1), upper triangular with zeros below the diagonal.  One
// workgroup per aggregate.
__global__ void __launch_bounds__(256) k_upper_blocks(int R, int Gm, int W,
                                                      const double* __restrict__ B,
                                                      double* __restrict__ R11,
                                                      double* __restrict__ R22) {
  const int b = blockIdx.x, t = threadIdx.x;
  const double* a = B + (size_t)b * R * (Gm + W);
  double* r11 = R11 + (size_t)b * Gm * Gm;
  double* r22 = R22 + (size_t)b * W * W;
  for (int64_t e = t; e < (int64_t)Gm * Gm; e += 256) {
    const int i = (int)(e % Gm), j = (int)(e / Gm);
    r11[e] = i <= j ? a[(size_t)j * R + i] : 0.0;
  }
  for (int64_t e = t; e < (int64_t)W * W; e += 256) {
    const int i = (int)(e % W), j = (int)(e / W);
    r22[e] = i <= j ? a[(size_t)(Gm + j) * R + Gm + i] : 0.0;
  }
}

// Symmetrise the true nw[b] x nw[b] block of C (W x W per aggregate) as
// (C + C^T) / 2, and set the padded rows and columns to zero with 2 g + 1 on
// the diagonal, g the largest absolute row sum of the true block (a bound on
// its eigenvalues).  One workgroup per aggregate.
__global__ void __launch_bounds__(256) k_sym_pad(int W, const int32_t* __restrict__ nw,
                                                 double* __restrict__ C) {
  __shared__ double red[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const int n = nw[b];
  double* c = C + (size_t)b * W * W;
  for (int64_t e = t; e < (int64_t)n * n; e += 256) {
    const int i = (int)(e % n), j = (int)(e / n);
    if (i <= j) continue;
    const double s = 0.5 * (c[(size_t)j * W + i] + c[(size_t)i * W + j]);
    c[(size_t)j * W + i] = s;
    c[(size_t)i * W + j] = s;
  }
  __syncthreads();
  double g = 0.0;
  for (int i = t; i < n; i += 256) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j) rs += fabs(c[(size_t)j * W + i]);
    g = fmax(g, rs);
  }
  red[t] = g;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double pad = 2.0 * red[0] + 1.0;
  for (int64_t e = t; e < (int64_t)W * W; e += 256) {
    const int i = (int)(e % W), j = (int)(e / W);
    if (i < n && j < n) continue;
    c[e] = i == j ? pad : 0.0;
  }
}

// X (rows x cols per aggregate, column-major) = the first cols columns of
// the rows x rows identity
__global__ void __launch_bounds__(256) k_eye(int64_t total, int rows, int cols,
                                             double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t w = e % ((int64_t)rows * cols);
  X[e] = (w % rows) == (w / rows) ? 1.0 : 0.0;
}

// Local eigenproblems up to this size go to the batched Jacobi eigensolver,
// larger ones to tridiagonalisation and divide and conquer (faster there)
constexpr int kJacobiMax = 64;

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

// Device buffers, stream and rocBLAS handle of one call, released on every
// exit path
struct Ctx {
  const RocApi& api;
  int prev = -1;
  hipStream_t s = nullptr;
  rocblas_handle hb = nullptr;
  std::vector<void*> bufs;
  explicit Ctx(int device, const RocApi& a) : api(a) {
    SD_HIP(hipGetDevice(&prev));
    SD_HIP(hipSetDevice(device));
    SD_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    SD_ROC(api.create_handle(&hb));
    SD_ROC(api.set_stream(hb, s));
  }
  ~Ctx() {
    if (s) (void)hipStreamSynchronize(s);
    for (void* p : bufs) (void)hipFree(p);
    if (hb) (void)api.destroy_handle(hb);
    if (s) (void)hipStreamDestroy(s);
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  template <typename T>
  T* alloc(size_t n) {
    void* p = nullptr;
    SD_HIP(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)));
    bufs.push_back(p);
    return (T*)p;
  }
  template <typename T>
  T* upload(const T* h, size_t n) {
    T* d = alloc<T>(n);
    if (n) SD_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
  }
  template <typename T>
  void download(T* h, const T* d, size_t n) {
    if (n) SD_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    SD_HIP(hipStreamSynchronize(s));
  }
  // every info entry zero, else throw (code, msg)
  void check_info(const rocblas_int* d, int nb, int code, const char* msg) {
    std::vector<rocblas_int> h(nb);
    download(h.data(), d, (size_t)nb);
    for (int b = 0; b < nb; ++b)
      if (h[b] != 0) throw SetupDevError{code, msg};
  }
};

}  // namespace

int device_local_problems(int device, int nb, int R, int W, int Gm, int O, double rtol,
                          const int32_t* nw, const double* B, const double* Aww, const double* Ai,
                          double* mu, double* U, double* Z, double* Ainv, int32_t* rank,
                          double* phase, std::string& msg) {
  if (nb <= 0) return LSAMG_OK;
  if (R < 0 || W <= 0 || Gm < 0 || O < W || !nw || !B || !Aww || !Ai || !mu || !U || !Z ||
      !rank) {
    msg = "device setup: bad batch sizes or pointers";
    return LSAMG_EINVAL;
  }
  const RocApi& api = roc_api();
  if (!api.ok) {
    msg = api.err;
    return LSAMG_EINVAL;
  }
  try {
    Ctx c(device, api);
    const size_t nbz = (size_t)nb;
    const double one = 1.0, zero = 0.0, mone = -1.0;
    // phase seconds (when asked): 0 uploads, 1 SVD (and the QR before it),
    // 2 Schur products, 3 Cholesky and triangular solves, 4 eigensolver,
    // 5 local inverses, 6 downloads
    auto t_last = std::chrono::steady_clock::now();
    auto mark = [&](int i) {
      if (!phase) return;
      SD_HIP(hipStreamSynchronize(c.s));
      const auto t = std::chrono::steady_clock::now();
      phase[i] += std::chrono::duration<double>(t - t_last).count();
      t_last = t;
    };
    const int nc = Gm + W;                      // columns of B: Gamma first, then omega
    const rocblas_stride sB = (rocblas_stride)R * nc;
    int32_t* dnw = c.upload(nw, nbz);
    double* dB = c.upload(B, nbz * R * nc);
    double* dBw = dB + (size_t)R * Gm;          // omega columns (leading dimension R)
    rocblas_int* info = c.alloc<rocblas_int>(nbz);
    int32_t* drank = c.alloc<int32_t>(nbz);
    SD_HIP(hipMemsetAsync(drank, 0, nbz * sizeof(int32_t), c.s));
    double* dAww = c.upload(Aww, nbz * W * W);
    double* dAi = c.upload(Ai, nbz * O * O);
    mark(0);
    // 1. S~ = B_w^T (I - Q Q^T) B_w
    double* dSm = c.alloc<double>(nbz * W * W);
    if (Gm > 0 && R >= nc) {
      // tall blocks: B = [B_Gamma B_w] = Q [R11 R12; 0 R22] (Householder QR),
      // R11 = W Sigma Y^T; with W_k the kept left vectors,
      // S~ = (R12 - W_k W_k^T R12)^T (R12 - W_k W_k^T R12) + R22^T R22
      double* dtau = c.alloc<double>(nbz * nc);
      SD_ROC(api.geqrf(c.hb, R, nc, dB, R, sB, dtau, nc, nb));
      double* dR11 = c.alloc<double>(nbz * Gm * Gm);
      double* dR22 = c.alloc<double>(nbz * W * W);
      hipLaunchKernelGGL(k_upper_blocks, dim3(nb), dim3(256), 0, c.s, R, Gm, W, (const double*)dB,
                         dR11, dR22);
      SD_HIP(hipGetLastError());
      double* dS = c.alloc<double>(nbz * Gm);
      double* dU = c.alloc<double>(nbz * Gm * Gm);
      double* dE = c.alloc<double>(nbz * std::max(Gm - 1, 1));
      SD_ROC(api.gesvd(c.hb, rocblas_svect_singular, rocblas_svect_none, Gm, Gm, dR11, Gm,
                       (rocblas_stride)Gm * Gm, dS, Gm, dU, Gm, (rocblas_stride)Gm * Gm, nullptr, 1,
                       1, dE, std::max(Gm - 1, 1), rocblas_outofplace, info, nb));
      c.check_info(info, nb, LSAMG_ENOTSPD, "singular value iteration did not converge");
      mark(1);
      hipLaunchKernelGGL(k_keep_mask, dim3(nb), dim3(256), 0, c.s, Gm, Gm, rtol, dS, dU, drank);
      SD_HIP(hipGetLastError());
      double* dC = c.alloc<double>(nbz * Gm * W);
      SD_ROC(api.gemm(c.hb, rocblas_operation_transpose, rocblas_operation_none, Gm, W, Gm, &one, dU,
                      Gm, (rocblas_stride)Gm * Gm, dBw, R, sB, &zero, dC, Gm,
                      (rocblas_stride)Gm * W, nb));
      SD_ROC(api.gemm(c.hb, rocblas_operation_none, rocblas_operation_none, Gm, W, Gm, &mone, dU, Gm,
                      (rocblas_stride)Gm * Gm, dC, Gm, (rocblas_stride)Gm * W, &one, dBw, R, sB,
                      nb));
      SD_ROC(api.gemm(c.hb, rocblas_operation_transpose, rocblas_operation_none, W, W, Gm, &one, dBw,
                      R, sB, dBw, R, sB, &zero, dSm, W, (rocblas_stride)W * W, nb));
      SD_ROC(api.gemm(c.hb, rocblas_operation_transpose, rocblas_operation_none, W, W, W, &one, dR22,
                      W, (rocblas_stride)W * W, dR22, W, (rocblas_stride)W * W, &one, dSm, W,
                      (rocblas_stride)W * W, nb));
    } else {
      // S~ from the left singular vectors of B_Gamma itself
      const int mn = std::min(R, Gm);
      if (mn > 0) {
        double* dS = c.alloc<double>(nbz * mn);
        double* dU = c.alloc<double>(nbz * R * mn);
        double* dE = c.alloc<double>(nbz * std::max(mn - 1, 1));
        SD_ROC(api.gesvd(c.hb, rocblas_svect_singular, rocblas_svect_none, R, Gm, dB, R, sB, dS, mn,
                         dU, R, (rocblas_stride)R * mn, nullptr, 1, 1, dE, std::max(mn - 1, 1),
                         rocblas_outofplace, info, nb));
        c.check_info(info, nb, LSAMG_ENOTSPD, "singular value iteration did not converge");
        mark(1);
        hipLaunchKernelGGL(k_keep_mask, dim3(nb), dim3(256), 0, c.s, R, mn, rtol, dS, dU, drank);
        SD_HIP(hipGetLastError());
        double* dC = c.alloc<double>(nbz * mn * W);
        SD_ROC(api.gemm(c.hb, rocblas_operation_transpose, rocblas_operation_none, mn, W, R, &one,
                        dU, R, (rocblas_stride)R * mn, dBw, R, sB, &zero, dC, mn,
                        (rocblas_stride)mn * W, nb));
        SD_ROC(api.gemm(c.hb, rocblas_operation_none, rocblas_operation_none, R, W, mn, &mone, dU, R,
                        (rocblas_stride)R * mn, dC, mn, (rocblas_stride)mn * W, &one, dBw, R, sB,
                        nb));
      }
      SD_ROC(api.gemm(c.hb, rocblas_operation_transpose, rocblas_operation_none, W, W, R, &one, dBw,
                      R, sB, dBw, R, sB, &zero, dSm, W, (rocblas_stride)W * W, nb));
    }
    mark(2);
    // 2. S~ u = mu A_ww u
    SD_ROC(api.potrf(c.hb, rocblas_fill_lower, W, dAww, W, (rocblas_stride)W * W, info, nb));
    c.check_info(info, nb, LSAMG_ENOTSPD, "A(omega,omega) is not SPD");
    SD_ROC(api.trsm(c.hb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_none,
                    rocblas_diagonal_non_unit, W, W, &one, dAww, W, (rocblas_stride)W * W, dSm, W,
                    (rocblas_stride)W * W, nb));
    SD_ROC(api.trsm(c.hb, rocblas_side_right, rocblas_fill_lower, rocblas_operation_transpose,
                    rocblas_diagonal_non_unit, W, W, &one, dAww, W, (rocblas_stride)W * W, dSm, W,
                    (rocblas_stride)W * W, nb));
    hipLaunchKernelGGL(k_sym_pad, dim3(nb), dim3(256), 0, c.s, W, dnw, dSm);
    SD_HIP(hipGetLastError());
    mark(3);
    double* dmu = c.alloc<double>(nbz * W);
    double* dres = c.alloc<double>(nbz);
    rocblas_int* dsw = c.alloc<rocblas_int>(nbz);
    if (W <= kJacobiMax) {
      SD_ROC(api.syevj(c.hb, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_lower,
                       W, dSm, W, (rocblas_stride)W * W, 0.0, dres, 100, dsw, dmu, W, info, nb));
    } else {
      double* dOff = c.alloc<double>(nbz * W);
      SD_ROC(api.syevd(c.hb, rocblas_evect_original, rocblas_fill_lower, W, dSm, W,
                       (rocblas_stride)W * W, dmu, W, dOff, W, info, nb));
    }
    c.check_info(info, nb, LSAMG_ENOTSPD, "eigensolver did not converge");
    mark(4);
    SD_ROC(api.trsm(c.hb, rocblas_side_left, rocblas_fill_lower, rocblas_operation_transpose,
                    rocblas_diagonal_non_unit, W, W, &one, dAww, W, (rocblas_stride)W * W, dSm, W,
                    (rocblas_stride)W * W, nb));
    c.download(mu, dmu, nbz * W);
    c.download(U, dSm, nbz * W * W);
    c.download(rank, drank, nbz);
    mark(6);
    // 3. A_i^{-1} e_j, j < W (and all of A_i^{-1})
    SD_ROC(api.potrf(c.hb, rocblas_fill_lower, O, dAi, O, (rocblas_stride)O * O, info, nb));
    c.check_info(info, nb, LSAMG_ENOTSPD, "local block A(Omega,Omega) is not SPD");
    const int ncol = Ainv ? O : W;
    double* dZ = c.alloc<double>(nbz * O * ncol);
    hipLaunchKernelGGL(k_eye, dim3(grid_of((int64_t)nbz * O * ncol)), dim3(256), 0, c.s,
                       (int64_t)nbz * O * ncol, O, ncol, dZ);
    SD_HIP(hipGetLastError());
    SD_ROC(api.potrs(c.hb, rocblas_fill_lower, O, ncol, dAi, O, (rocblas_stride)O * O, dZ, O,
                     (rocblas_stride)O * ncol, nb));
    mark(5);
    if (Ainv) {
      c.download(Ainv, dZ, nbz * O * O);
      for (size_t b = 0; b < nbz; ++b)          // Z: the first W columns of each inverse
        std::copy(Ainv + b * O * O, Ainv + b * O * O + (size_t)O * W, Z + b * O * W);
    } else {
      c.download(Z, dZ, nbz * O * W);
    }
    mark(6);
  } catch (const SetupDevError& e) {
    msg = e.msg;
    return e.code;
  }
  return LSAMG_OK;
}

int device_setup_preload(int device, std::string& msg) {
  const RocApi& api = roc_api();
  if (!api.ok) {
    msg = api.err;
    return LSAMG_EINVAL;
  }
  try {
    Ctx c(device, api);                 // a rocBLAS handle made and released
  } catch (const SetupDevError& e) {
    msg = e.msg;
    return e.code;
  }
  return LSAMG_OK;
}

int device_spd_inverse(int device, int n, const double* A, double* Ainv, std::string& msg) {
  if (n <= 0) return LSAMG_OK;
  if (!A || !Ainv) {
    msg = "device setup: null matrix";
    return LSAMG_EINVAL;
  }
  const RocApi& api = roc_api();
  if (!api.ok) {
    msg = api.err;
    return LSAMG_EINVAL;
  }
  try {
    Ctx c(device, api);
    const size_t nn = (size_t)n * n;
    double* dA = c.upload(A, nn);
    rocblas_int* info = c.alloc<rocblas_int>(1);
    SD_ROC(api.potrf(c.hb, rocblas_fill_lower, n, dA, n, (rocblas_stride)nn, info, 1));
    c.check_info(info, 1, LSAMG_ENOTSPD, "coarsest matrix is not SPD");
    double* dX = c.alloc<double>(nn);
    hipLaunchKernelGGL(k_eye, dim3(grid_of((int64_t)nn)), dim3(256), 0, c.s, (int64_t)nn, n, n, dX);
    SD_HIP(hipGetLastError());
    SD_ROC(api.potrs(c.hb, rocblas_fill_lower, n, n, dA, n, (rocblas_stride)nn, dX, n,
                     (rocblas_stride)nn, 1));
    c.download(Ainv, dX, nn);
  } catch (const SetupDevError& e) {
    msg = e.msg;
    return e.code;
  }
  return LSAMG_OK;
}

}  // namespace lsamg
