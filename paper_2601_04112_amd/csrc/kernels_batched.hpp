// Multi-right-hand-side (batched) kernels of the LS-AMG-DD solve phase.
//
// A batch of NB <= 64 right-hand sides is stored interleaved: entry (i, j) of
// an n x NB block is at i*NB + j, so the NB values of one unknown are
// contiguous and every gather of a vector entry becomes one coalesced row of
// NB values.  Each matrix entry (Z_i, Zhat_i, G, the coarsest inverse) is then
// read once per batch instead of once per right-hand side, and the local
// solves of the smoothers become small GEMMs per aggregate.
#pragma once

#include "kernels.hpp"

namespace lsamg {
namespace dev {

// Y = G X: one group of NB lanes per row, lanes along the right-hand sides.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bspmv(int64_t nrows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ val,
                                                  const T* __restrict__ X, T* __restrict__ Y) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t row = gid / NB;
  const int j = (int)(gid % NB);
  if (row >= nrows) return;
  const int64_t e0 = ptr[row], e1 = ptr[row + 1];
  T s0 = 0, s1 = 0;
  int64_t e = e0;
  for (; e + 1 < e1; e += 2) {
    const int32_t c0 = col[e], c1 = col[e + 1];
    const T v0 = val[e], v1 = val[e + 1];
    s0 += v0 * X[(int64_t)c0 * NB + j];
    s1 += v1 * X[(int64_t)c1 * NB + j];
  }
  if (e < e1) s0 += val[e] * X[(int64_t)col[e] * NB + j];
  Y[row * NB + j] = s0 + s1;
}

// R = B - G^T Y (B == nullptr: R = G^T Y)
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bresid_t(int64_t n, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col,
                                                     const T* __restrict__ val,
                                                     const T* __restrict__ Y,
                                                     const T* __restrict__ B,
                                                     T* __restrict__ R) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t d = gid / NB;
  const int j = (int)(gid % NB);
  if (d >= n) return;
  const int64_t e0 = ptr[d], e1 = ptr[d + 1];
  T s0 = 0, s1 = 0;
  int64_t e = e0;
  for (; e + 1 < e1; e += 2) {
    const int32_t c0 = col[e], c1 = col[e + 1];
    const T v0 = val[e], v1 = val[e + 1];
    s0 += v0 * Y[(int64_t)c0 * NB + j];
    s1 += v1 * Y[(int64_t)c1 * NB + j];
  }
  if (e < e1) s0 += val[e] * Y[(int64_t)col[e] * NB + j];
  const T s = s0 + s1;
  R[d * NB + j] = B ? B[d * NB + j] - s : s;
}

// Batched form of the aggregate GEMV family (see k_gemv_*):
//   OUT[obase_a + jj][:] (=|+=) sum_l M_a[l][jj] * IN_a[l][:]
// Task = (aggregate a, 64-wide slice j0 of its outputs) x all NB columns.
// Thread t: output row jj = j0 + (t % 64) (lanes along the contiguous matrix
// index), right-hand sides [(t/64)*NB/4, (t/64+1)*NB/4).  The input rows are
// staged through LDS in chunks of LC loop indices; every lane of a wave reads
// the same staged value (broadcast).  LDS: LC * NB * sizeof(T).
template <typename T, int MODE, bool ADD, int NB>
__global__ void __launch_bounds__(kBlock) k_bgemm(const int32_t* __restrict__ task_a,
                                                  const int32_t* __restrict__ task_j0,
                                                  GemvOp op, const int32_t* __restrict__ gidx,
                                                  const int64_t* __restrict__ cptr,
                                                  const int64_t* __restrict__ cpos,
                                                  const T* __restrict__ tb,
                                                  const T* __restrict__ M,
                                                  const T* __restrict__ in,
                                                  T* __restrict__ out) {
  constexpr int LC = 32;            // loop indices staged per chunk
  constexpr int RW = NB / 4;        // right-hand sides per thread
  __shared__ T sv[LC * NB];
  const int64_t a = task_a[blockIdx.x];
  const int j0 = task_j0[blockIdx.x];
  const int nj = op.lj[a], nl = op.ll[a];
  const int64_t ib = op.ibase[a];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jj = j0 + lane;
  const bool jv = jj < nj;
  const T* m = M + op.moff[a] + (jv ? jj : 0);
  T acc[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) acc[r] = 0;
  for (int l0 = 0; l0 < nl; l0 += LC) {
    const int lc = min(LC, nl - l0);
    __syncthreads();
    for (int e = threadIdx.x; e < lc * NB; e += kBlock) {
      const int l = e / NB, c = e % NB;
      const int64_t i = ib + l0 + l;
      T v;
      if (MODE == IN_GATHER) {
        v = in[(int64_t)gidx[i] * NB + c];
      } else if (MODE == IN_TB) {
        v = in[i * NB + c];
        for (int64_t q = cptr[i]; q < cptr[i + 1]; ++q) v += tb[cpos[q] * NB + c];
      } else {
        v = in[i * NB + c];
      }
      sv[e] = v;
    }
    __syncthreads();
    if (jv) {
      for (int l = 0; l < lc; ++l) {
        const T mv = m[(int64_t)(l0 + l) * nj];
        const T* s = sv + l * NB + wave * RW;
#pragma unroll
        for (int r = 0; r < RW; ++r) acc[r] += mv * s[r];
      }
    }
  }
  if (jv) {
    T* dst = out + (op.obase[a] + jj) * NB + wave * RW;
#pragma unroll
    for (int r = 0; r < RW; ++r) dst[r] = ADD ? dst[r] + acc[r] : acc[r];
  }
}

// X[j][:] += staged RAS-T contributions (batched k_gather_add)
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bgather_add(int64_t n, const int64_t* __restrict__ cptr,
                                                        const int64_t* __restrict__ cpos,
                                                        const T* __restrict__ tb,
                                                        T* __restrict__ X) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t d = gid / NB;
  const int c = (int)(gid % NB);
  if (d >= n) return;
  T s = X[d * NB + c];
  for (int64_t e = cptr[d]; e < cptr[d + 1]; ++e) s += tb[cpos[e] * NB + c];
  X[d * NB + c] = s;
}

// ---------------------------------------------------------------------------
// Batched FP64 CG.  Column j has its own scalars; partial sums are stored per
// workgroup and column (part[blockIdx.x * NB + j]) and re-summed in fixed
// order by the consuming kernel.  active[j] = 0 freezes a converged column.
// ---------------------------------------------------------------------------
template <int NB>
__device__ __forceinline__ void bwrite_parts(double v, double* __restrict__ part) {
  // threads of one column j = tid % NB share kBlock/NB slots
  __shared__ double sm[kBlock];
  sm[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < NB) {
    double s = 0;
    for (int t = threadIdx.x; t < kBlock; t += NB) s += sm[t];
    part[(int64_t)blockIdx.x * NB + threadIdx.x] = s;
  }
  __syncthreads();
}

// value of column j summed over np workgroups (same order everywhere)
__device__ __forceinline__ double bsum(const double* __restrict__ part, int np, int NB, int j) {
  double s = 0;
  for (int b = 0; b < np; ++b) s += part[(int64_t)b * NB + j];
  return s;
}

template <int NB>
__global__ void __launch_bounds__(kBlock) k_bdot(int64_t n, const double* __restrict__ A,
                                                 const double* __restrict__ B,
                                                 double* __restrict__ part) {
  const int j = threadIdx.x % NB;
  double v = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock)
    v += A[e] * B[e];
  (void)j;
  bwrite_parts<NB>(v, part);
}

// Q = G^T Y (finest level) and partials of P . Q per column
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_apq(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val,
                                                    const double* __restrict__ Y,
                                                    const double* __restrict__ P,
                                                    double* __restrict__ Q,
                                                    double* __restrict__ part) {
  const int j = threadIdx.x % NB;
  double v = 0;
  for (int64_t d = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / NB; d < n;
       d += (int64_t)gridDim.x * (kBlock / NB)) {
    double s = 0;
    for (int64_t e = ptr[d]; e < ptr[d + 1]; ++e) s += val[e] * Y[(int64_t)col[e] * NB + j];
    Q[d * NB + j] = s;
    v += s * P[d * NB + j];
  }
  bwrite_parts<NB>(v, part);
}

// alpha_j = rho_j / pq_j (0 for inactive columns); X += alpha P; R -= alpha Q;
// R32 = (float) R (if given); partials of R . R
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_update(int64_t n, const double* __restrict__ rz_part,
                                                       const double* __restrict__ pq_part,
                                                       const int* __restrict__ active,
                                                       const double* __restrict__ P,
                                                       const double* __restrict__ Q,
                                                       double* __restrict__ X,
                                                       double* __restrict__ R,
                                                       float* __restrict__ R32,
                                                       double* __restrict__ rr_part) {
  const int np = gridDim.x;
  const int j = threadIdx.x % NB;
  bool act = active[j] != 0;
  const double pq = act ? bsum(pq_part, np, NB, j) : 0.0;
  act = act && pq != 0.0;
  const double alpha = act ? bsum(rz_part, np, NB, j) / pq : 0.0;
  double v = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock) {
    if (!act) continue;               // a converged column is left untouched
    X[e] += alpha * P[e];
    const double ri = R[e] - alpha * Q[e];
    R[e] = ri;
    if (R32) R32[e] = (float)ri;
    v += ri * ri;
  }
  bwrite_parts<NB>(v, rr_part);
}

// Z = XV + staged RAS-T contributions (V-cycle precision T); partials of R . Z
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_z(int64_t n, const T* __restrict__ XV,
                                                  const int64_t* __restrict__ cptr,
                                                  const int64_t* __restrict__ cpos,
                                                  const T* __restrict__ tb,
                                                  const double* __restrict__ R,
                                                  double* __restrict__ Z,
                                                  double* __restrict__ rz_part) {
  const int c = threadIdx.x % NB;
  double v = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock) {
    const int64_t d = e / NB;
    T s = XV[e];
    if (cptr)
      for (int64_t q = cptr[d]; q < cptr[d + 1]; ++q) s += tb[cpos[q] * NB + c];
    const double zi = (double)s;
    Z[e] = zi;
    v += R[e] * zi;
  }
  bwrite_parts<NB>(v, rz_part);
}

// P = Z + beta P, beta_j = rz_new_j / rz_old_j (rz_old == nullptr: P = Z)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_dir(int64_t n, const double* __restrict__ rz_new,
                                                    const double* __restrict__ rz_old,
                                                    const double* __restrict__ Z,
                                                    double* __restrict__ P) {
  const int np = gridDim.x;
  const int j = threadIdx.x % NB;
  double beta = 0.0;
  if (rz_old) {
    const double o = bsum(rz_old, np, NB, j);
    beta = o != 0.0 ? bsum(rz_new, np, NB, j) / o : 0.0;   // an all-zero column stays zero
  }
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock)
    P[e] = rz_old ? Z[e] + beta * P[e] : Z[e];   // first direction: P = Z (P may hold stale data)
}

// Bi[i][j] = b[j*ld + perm[i]]  (user column-major -> internal interleaved)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bperm_in(int64_t n, int nrhs, int64_t ld,
                                                     const int64_t* __restrict__ perm,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ Bi) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * NB) return;
  const int64_t i = e / NB;
  const int j = (int)(e % NB);
  Bi[e] = j < nrhs ? b[(int64_t)j * ld + perm[i]] : 0.0;
}

// x[j*ld + perm[i]] = X[i][j]
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bperm_out(int64_t n, int nrhs, int64_t ld,
                                                      const int64_t* __restrict__ perm,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * NB) return;
  const int64_t i = e / NB;
  const int j = (int)(e % NB);
  if (j < nrhs) x[(int64_t)j * ld + perm[i]] = X[e];
}

}  // namespace dev
}  // namespace lsamg
