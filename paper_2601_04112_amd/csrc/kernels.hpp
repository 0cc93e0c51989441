// HIP kernels of the LS-AMG-DD solve phase for CDNA4 (gfx950, wave64).
//
// Every V-cycle kernel is templated on the V-cycle scalar type T (double for
// the FP64 path, float for the mixed-precision path).  Unknowns are in the
// library's internal numbering, where each aggregate omega_i is the
// contiguous range [astart[i], astart[i+1]) and its coarse unknowns are the
// contiguous range [cstart[i], cstart[i+1]) of the next level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsamg {
namespace dev {

constexpr int kBlock = 256;

template <typename T>
__device__ __forceinline__ T wave_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// ---------------------------------------------------------------------------
// A = G^T G applied in two passes (eq:Ax=b): y = G x, then r = b - G^T y.
// One group of `lanes` threads per row; lanes stride over the row.
// ---------------------------------------------------------------------------
template <typename T, int LANES>
__global__ void __launch_bounds__(kBlock) k_spmv(int64_t nrows, const int64_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col,
                                                 const T* __restrict__ val,
                                                 const T* __restrict__ x, T* __restrict__ y) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t row = gid / LANES;
  const int lane = (int)(gid % LANES);
  if (row >= nrows) return;  // LANES divides the block, so whole groups exit
  T s = 0;
  for (int64_t e = ptr[row] + lane; e < ptr[row + 1]; e += LANES) s += val[e] * x[col[e]];
  if (LANES > 1) s = wave_sum(s, LANES);
  if (lane == 0) y[row] = s;
}

// r = b - G^T y  (rows of G^T = unknowns); G^T stored as CSR by unknown.
template <typename T, int LANES>
__global__ void __launch_bounds__(kBlock) k_resid_t(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const T* __restrict__ y,
                                                    const T* __restrict__ b, T* __restrict__ r) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t row = gid / LANES;
  const int lane = (int)(gid % LANES);
  if (row >= n) return;
  T s = 0;
  for (int64_t e = ptr[row] + lane; e < ptr[row + 1]; e += LANES) s += val[e] * y[col[e]];
  if (LANES > 1) s = wave_sum(s, LANES);
  if (lane == 0) r[row] = (b ? b[row] : T(0)) - s;
}

// ---------------------------------------------------------------------------
// RAS (eq:ras) from a zero initial guess: x(omega_i) = Z_i b(Omega_i), with
// Z_i = A_i^{-1}(omega_i, Omega_i) stored column-major (Omega-major) so that
// consecutive threads read consecutive rows of one column.  One workgroup per
// aggregate; b(Omega_i) is gathered into LDS first.  The Boolean partition
// of unity makes every unknown written by exactly one workgroup.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_ras(const int64_t* __restrict__ astart,
                                                const int64_t* __restrict__ optr,
                                                const int32_t* __restrict__ oidx,
                                                const int64_t* __restrict__ zoff,
                                                const T* __restrict__ Zc, const T* __restrict__ b,
                                                T* __restrict__ x) {
  extern __shared__ unsigned char smem_raw[];
  T* sb = reinterpret_cast<T*>(smem_raw);
  const int64_t a = blockIdx.x;
  const int64_t w0 = astart[a];
  const int nw = (int)(astart[a + 1] - w0);
  const int64_t o0 = optr[a];
  const int nO = (int)(optr[a + 1] - o0);
  T* part = sb + nO;  // kBlock partial sums
  for (int c = threadIdx.x; c < nO; c += kBlock) sb[c] = b[oidx[o0 + c]];
  __syncthreads();
  const T* Z = Zc + zoff[a];
  int nwp = 1;
  while (nwp < nw) nwp <<= 1;
  if (nwp <= kBlock) {
    const int groups = kBlock / nwp;
    const int p = threadIdx.x % nwp, g = threadIdx.x / nwp;
    T s = 0;
    if (p < nw)
      for (int c = g; c < nO; c += groups) s += Z[(int64_t)c * nw + p] * sb[c];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < nw) {
      T t = 0;
      for (int gg = 0; gg < groups; ++gg) t += part[gg * nwp + threadIdx.x];
      x[w0 + threadIdx.x] = t;
    }
  } else {
    for (int p = threadIdx.x; p < nw; p += kBlock) {
      T s = 0;
      for (int c = 0; c < nO; ++c) s += Z[(int64_t)c * nw + p] * sb[c];
      x[w0 + p] = s;
    }
  }
}

// RAS-T (eq:ras-t), first half: t_i = Z_i^T r(omega_i) = A_i^{-1}(Omega_i,
// omega_i) r(omega_i), with Z_i stored row-major (omega-major).  The |Omega_i|
// values are written to the staging buffer tb at optr[i]; k_gather_add then
// adds them into x in a fixed order (deterministic, no atomics).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_rast(const int64_t* __restrict__ astart,
                                                 const int64_t* __restrict__ optr,
                                                 const int64_t* __restrict__ zoff,
                                                 const T* __restrict__ Zr,
                                                 const T* __restrict__ r, T* __restrict__ tb) {
  extern __shared__ unsigned char smem_raw[];
  T* sr = reinterpret_cast<T*>(smem_raw);
  const int64_t a = blockIdx.x;
  const int64_t w0 = astart[a];
  const int nw = (int)(astart[a + 1] - w0);
  const int64_t o0 = optr[a];
  const int nO = (int)(optr[a + 1] - o0);
  T* part = sr + nw;
  for (int p = threadIdx.x; p < nw; p += kBlock) sr[p] = r[w0 + p];
  __syncthreads();
  const T* Z = Zr + zoff[a];
  int nOp = 1;
  while (nOp < nO) nOp <<= 1;
  if (nOp <= kBlock) {
    const int groups = kBlock / nOp;
    const int c = threadIdx.x % nOp, g = threadIdx.x / nOp;
    T s = 0;
    if (c < nO)
      for (int p = g; p < nw; p += groups) s += Z[(int64_t)p * nO + c] * sr[p];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < nO) {
      T t = 0;
      for (int gg = 0; gg < groups; ++gg) t += part[gg * nOp + threadIdx.x];
      tb[o0 + threadIdx.x] = t;
    }
  } else {
    for (int c = threadIdx.x; c < nO; c += kBlock) {
      T s = 0;
      for (int p = 0; p < nw; ++p) s += Z[(int64_t)p * nO + c] * sr[p];
      tb[o0 + c] = s;
    }
  }
}

// x[j] += sum of the staged RAS-T contributions to unknown j (ascending
// staging position, i.e. ascending aggregate id).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gather_add(int64_t n, const int64_t* __restrict__ cptr,
                                                       const int64_t* __restrict__ cpos,
                                                       const T* __restrict__ tb,
                                                       T* __restrict__ x) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  T s = x[j];
  for (int64_t e = cptr[j]; e < cptr[j + 1]; ++e) s += tb[cpos[e]];
  x[j] = s;
}

// ---------------------------------------------------------------------------
// Restriction r_c = P^T r and prolongation x += P e (eq:mg-p, eq:cgc): P is
// block diagonal, block i = Zhat_i (|omega_i| x k_i, row-major); the coarse
// unknowns of aggregate i are [cstart[i], cstart[i] + k_i) (not ordered by i).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict(const int64_t* __restrict__ astart,
                                                     const int64_t* __restrict__ cstart,
                                                     const int32_t* __restrict__ kk,
                                                     const int64_t* __restrict__ poff,
                                                     const T* __restrict__ Zh,
                                                     const T* __restrict__ r, T* __restrict__ rc) {
  extern __shared__ unsigned char smem_raw[];
  T* sr = reinterpret_cast<T*>(smem_raw);
  const int64_t a = blockIdx.x;
  const int64_t w0 = astart[a];
  const int nw = (int)(astart[a + 1] - w0);
  const int64_t c0 = cstart[a];
  const int k = kk[a];
  for (int p = threadIdx.x; p < nw; p += kBlock) sr[p] = r[w0 + p];
  __syncthreads();
  const T* Z = Zh + poff[a];
  for (int s = threadIdx.x; s < k; s += kBlock) {
    T acc = 0;
    for (int p = 0; p < nw; ++p) acc += Z[(int64_t)p * k + s] * sr[p];
    rc[c0 + s] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong(const int64_t* __restrict__ astart,
                                                    const int64_t* __restrict__ cstart,
                                                    const int32_t* __restrict__ kk,
                                                    const int64_t* __restrict__ poff,
                                                    const T* __restrict__ Zh,
                                                    const T* __restrict__ e, T* __restrict__ x) {
  extern __shared__ unsigned char smem_raw[];
  T* se = reinterpret_cast<T*>(smem_raw);
  const int64_t a = blockIdx.x;
  const int64_t w0 = astart[a];
  const int nw = (int)(astart[a + 1] - w0);
  const int64_t c0 = cstart[a];
  const int k = kk[a];
  for (int s = threadIdx.x; s < k; s += kBlock) se[s] = e[c0 + s];
  __syncthreads();
  const T* Z = Zh + poff[a];
  for (int p = threadIdx.x; p < nw; p += kBlock) {
    T acc = 0;
    for (int s = 0; s < k; ++s) acc += Z[(int64_t)p * k + s] * se[s];
    x[w0 + p] += acc;
  }
}

// Coarsest level: e = A_L^{-1} r with the dense inverse (row-major); one
// wavefront per row.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(int64_t n, const T* __restrict__ M,
                                                       const T* __restrict__ r,
                                                       T* __restrict__ e) {
  const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n) return;
  const T* mr = M + row * n;
  T s = 0;
  for (int64_t j = lane; j < n; j += 64) s += mr[j] * r[j];
  s = wave_sum(s, 64);
  if (lane == 0) e[row] = s;
}

// ---------------------------------------------------------------------------
// Vector kernels of the outer FP64 CG.
// ---------------------------------------------------------------------------
// Block partial sums of a.b (deterministic two-stage reduction).
__global__ void __launch_bounds__(kBlock) k_dot_partial(int64_t n, const double* __restrict__ a,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ part) {
  __shared__ double sm[kBlock / 64];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    s += a[i] * b[i];
  s = wave_sum(s, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < kBlock / 64; ++w) t += sm[w];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_sum_final(int nparts, const double* __restrict__ part,
                                                      double* __restrict__ out) {
  __shared__ double sm[kBlock];
  double s = 0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sm[0];
}

// x += alpha p ; r -= alpha q   with alpha = s[0] / s[1] read on the device
__global__ void __launch_bounds__(kBlock) k_cg_update(int64_t n, const double* __restrict__ sc,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double alpha = sc[0] / sc[1];
  x[i] += alpha * p[i];
  r[i] -= alpha * q[i];
}

// p = z + beta p   with beta = s[2] / s[0]
__global__ void __launch_bounds__(kBlock) k_cg_dir(int64_t n, const double* __restrict__ sc,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double beta = sc[2] / sc[0];
  p[i] = z[i] + beta * p[i];
}

template <typename Ti, typename To>
__global__ void __launch_bounds__(kBlock) k_convert(int64_t n, const Ti* __restrict__ a,
                                                    To* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = (To)a[i];
}

// out[i] = in[perm[i]]  (user numbering -> internal)
__global__ void __launch_bounds__(kBlock) k_perm_in(int64_t n, const int64_t* __restrict__ perm,
                                                    const double* __restrict__ in,
                                                    double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

// out[perm[i]] = in[i]  (internal -> user numbering)
__global__ void __launch_bounds__(kBlock) k_perm_out(int64_t n, const int64_t* __restrict__ perm,
                                                     const double* __restrict__ in,
                                                     double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[perm[i]] = in[i];
}

__global__ void __launch_bounds__(kBlock) k_copy(int64_t n, const double* __restrict__ a,
                                                 double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// out = a - b
__global__ void __launch_bounds__(kBlock) k_sub(int64_t n, const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void __launch_bounds__(kBlock) k_fill(int64_t n, double v, double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = v;
}

// count of non-finite entries (for input validation)
__global__ void __launch_bounds__(kBlock) k_nonfinite(int64_t n, const double* __restrict__ a,
                                                      int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && !isfinite(a[i])) atomicOr(flag, 1);
}

}  // namespace dev
}  // namespace lsamg
