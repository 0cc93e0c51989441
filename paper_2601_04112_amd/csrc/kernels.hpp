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

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// XCD-aware block order.  The command processor deals consecutive workgroups
// of a launch to the 8 XCDs in turn, and each XCD has its own L2; this
// bijection of [0, nb) gives XCD x = b % 8 the contiguous range of logical
// blocks [x*q + min(x, r), ...) (q = nb / 8, r = nb % 8), so workgroups that
// touch neighbouring rows (and gather the same vector entries) share an L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb) {
  constexpr int64_t X = 8;
  const int64_t q = nb / X, r = nb % X;
  const int64_t x = b % X, k = b / X;
  return x * q + (x < r ? x : r) + k;
}

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
  // each group of LANES threads owns two rows, processed together so that
  // their loads overlap
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t r0 = (gid / LANES) * 2;
  const int lane = (int)(gid % LANES);
  if (r0 >= nrows) return;  // LANES divides the block, so whole groups exit
  const bool two = r0 + 1 < nrows;
  const int64_t b0 = ptr[r0], e0 = ptr[r0 + 1];
  const int64_t e1 = two ? ptr[r0 + 2] : e0;
  T s0 = 0, s1 = 0;
  int64_t p = b0 + lane, q = e0 + lane;
  for (; p < e0 && q < e1; p += LANES, q += LANES) {
    const T v0 = val[p], v1 = val[q];
    const int32_t c0 = col[p], c1 = col[q];
    s0 += v0 * x[c0];
    s1 += v1 * x[c1];
  }
  for (; p < e0; p += LANES) s0 += val[p] * x[col[p]];
  for (; q < e1; q += LANES) s1 += val[q] * x[col[q]];
  if (LANES > 1) {
    s0 = wave_sum(s0, LANES);
    s1 = wave_sum(s1, LANES);
  }
  if (lane == 0) {
    y[r0] = s0;
    if (two) y[r0 + 1] = s1;
  }
}

// r = b - G^T y  (rows of G^T = unknowns); G^T stored as CSR by unknown.
// b == nullptr gives r = G^T y (no subtraction, no sign change).
template <typename T, int LANES>
__global__ void __launch_bounds__(kBlock) k_resid_t(int64_t n, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const T* __restrict__ y,
                                                    const T* __restrict__ b, T* __restrict__ r) {
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t r0 = (gid / LANES) * 2;
  const int lane = (int)(gid % LANES);
  if (r0 >= n) return;
  const bool two = r0 + 1 < n;
  const int64_t b0 = ptr[r0], e0 = ptr[r0 + 1];
  const int64_t e1 = two ? ptr[r0 + 2] : e0;
  T s0 = 0, s1 = 0;
  int64_t p = b0 + lane, q = e0 + lane;
  for (; p < e0 && q < e1; p += LANES, q += LANES) {
    const T v0 = val[p], v1 = val[q];
    const int32_t c0 = col[p], c1 = col[q];
    s0 += v0 * y[c0];
    s1 += v1 * y[c1];
  }
  for (; p < e0; p += LANES) s0 += val[p] * y[col[p]];
  for (; q < e1; q += LANES) s1 += val[q] * y[col[q]];
  if (LANES > 1) {
    s0 = wave_sum(s0, LANES);
    s1 = wave_sum(s1, LANES);
  }
  if (lane == 0) {
    r[r0] = b ? b[r0] - s0 : s0;
    if (two) r[r0 + 1] = b ? b[r0 + 1] - s1 : s1;
  }
}

// ---------------------------------------------------------------------------
// Batched small dense GEMV over aggregates: the smoothers and the transfer
// operators of the V-cycle are all of the form
//
//     out[obase_a + j]  (=|+=)  sum_l  M_a[l][j] * in_a[l],   j < lj_a, l < ll_a
//
// with M_a stored so that j is contiguous (M_a[l][j] at moff_a + l*lj_a + j):
//   RAS    (eq:ras):   M = A_i^{-1}(omega_i, Omega_i) column-major, j = row of
//                      omega_i, l = Omega_i entry, in = b gathered via Omega_i
//   RAS-T  (eq:ras-t): M = the same block row-major, j = Omega_i entry,
//                      l = row of omega_i, in = r(omega_i), out = staging tb
//   P^T    (eq:mg-p):  M = Zhat_i row-major, j = coarse unknown, l = row
//   P      (eq:mg-p):  M = Zhat_i column-major, j = row, l = coarse unknown,
//                      out += ; the input may add the coarse level's staged
//                      RAS-T contributions on the fly (IN_TB)
// Lanes run along j (coalesced loads), the loop runs along l, and every
// output is reduced in a fixed order (deterministic, no atomics).
// ---------------------------------------------------------------------------
enum { IN_DIRECT = 0, IN_GATHER = 1, IN_TB = 2, IN_RESG = 3 };

struct GemvOp {
  const int64_t* moff;   // [nagg] offset of M_a
  const int32_t* lj;     // [nagg] output length (contiguous dimension)
  const int32_t* ll;     // [nagg] input length (loop dimension)
  const int64_t* ibase;  // [nagg] input base (index-list base for IN_GATHER)
  const int64_t* obase;  // [nagg] output base
  int pad;               // rows of M_a: 0 unpadded, 1 padded to a multiple of 4
                         // entries, else to a multiple of pad (a multiple of 4)
};

// Row stride of M_a: lj, or lj rounded up to a multiple of 4 or of pad
// (padded layout: every row starts 16-byte aligned, or on a 128-byte line
// for pad 32 in FP32, and the padding is zero).
__device__ __forceinline__ int64_t mrow(int nj, int pad) {
  if (pad == 0) return nj;
  if (pad == 1) return (int64_t)((nj + 3) & ~3);
  return (int64_t)((nj + pad - 1) / pad) * pad;
}

// Where the input vector entries come from (MODE):
//   IN_DIRECT  in[i]
//   IN_GATHER  in[idx[i]]
//   IN_TB      in[i] + sum_{e in [ptr[i], ptr[i+1])} v1[pos[e]]       (staged RAS-T)
//   IN_RESG    in[i] - sum_{e in [ptr[i], ptr[i+1])} v1[e] * v2[idx[e]] (row i of G^T
//              applied to v2 = G x): the residual b - A x formed on the fly, so
//              the residual vector of the level is never written to memory
template <typename T>
struct InSpec {
  const int32_t* idx;
  const int64_t* ptr;
  const int64_t* pos;
  const T* v1;
  const T* v2;
};

template <typename T, int MODE>
__device__ __forceinline__ T load_in(const T* __restrict__ in, int64_t i, const InSpec<T>& sp) {
  if (MODE == IN_GATHER) return in[sp.idx[i]];
  if (MODE == IN_DIRECT) return in[i];
  const int64_t e0 = sp.ptr[i], e1 = sp.ptr[i + 1];
  T v = in[i];
  if (MODE == IN_TB) {
    for (int64_t e = e0; e < e1; ++e) v += sp.v1[sp.pos[e]];
    return v;
  }
  T t = 0;
  for (int64_t e = e0; e < e1; ++e) t += sp.v1[e] * sp.v2[sp.idx[e]];
  return v - t;
}

// IN_RESG staging in two steps.  The G^T rows of the consecutive inputs
// ib .. ib+nl-1 form one contiguous range of entries, so the threads first
// form every product v1[e] * v2[idx[e]] of that range with coalesced loads
// into pr (LDS); after a barrier each input adds its own products in entry
// order (the same order as load_in).
template <typename T, int MODE>
__device__ __forceinline__ void stage_products(T* pr, int64_t ib, int nl, const InSpec<T>& sp,
                                               int tid, int nt) {
  if (MODE != IN_RESG) return;
  const int64_t eb = sp.ptr[ib], ee = sp.ptr[ib + nl];
  for (int64_t e = eb + tid; e < ee; e += nt) pr[e - eb] = sp.v1[e] * sp.v2[sp.idx[e]];
}

template <typename T, int MODE>
__device__ __forceinline__ void stage_inputs(T* sv, const T* pr, const T* __restrict__ in,
                                             int64_t ib, int nl, const InSpec<T>& sp, int tid,
                                             int nt) {
  for (int l = tid; l < nl; l += nt) {
    if (MODE == IN_RESG) {
      const int64_t eb = sp.ptr[ib];
      T t = 0;
      for (int64_t e = sp.ptr[ib + l]; e < sp.ptr[ib + l + 1]; ++e) t += pr[e - eb];
      sv[l] = in[ib + l] - t;
    } else {
      sv[l] = load_in<T, MODE>(in, ib + l, sp);
    }
  }
}

// Narrow form (every lj_a <= G <= 64): one wavefront per aggregate, the
// wavefront split into 64/G lane groups that share the loop over l; four
// aggregates per 256-thread workgroup.  LDS: 4 * (lmax + emax) * sizeof(T)
// (emax: the most G^T entries of one aggregate's inputs, IN_RESG only).
template <typename T, int MODE, bool ADD, int G>
__global__ void __launch_bounds__(kBlock) k_gemv_narrow(int64_t nagg, GemvOp op, int lmax,
                                                        int emax, InSpec<T> spec,
                                                        const T* __restrict__ M,
                                                        const T* __restrict__ in,
                                                        T* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int S = 64 / G;
  constexpr int U = 8;                       // independent loads in flight per lane
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t a = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + wave;
  const bool valid = a < nagg;
  T* sv = reinterpret_cast<T*>(smem_raw) + (size_t)wave * (lmax + emax);
  T* pr = sv + lmax;
  const int s = lane / G, j = lane % G;
  int nj = 0, nl = 0;
  int64_t ib = 0, ld = 0;
  const T* m = M;
  T mv[U];
  if (valid) {
    nj = op.lj[a];
    nl = op.ll[a];
    m = M + op.moff[a] + (j < nj ? j : 0);
    ld = mrow(nj, op.pad);
    // the first U matrix entries of the lane do not depend on the staged
    // input: their loads are issued before the staging gather and barrier
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = s + u * S;
      mv[u] = (j < nj && l < nl) ? __builtin_nontemporal_load(&m[(int64_t)l * ld]) : T(0);
    }
    ib = op.ibase[a];
    if (MODE == IN_RESG)
      stage_products<T, MODE>(pr, ib, nl, spec, lane, 64);
    else
      stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, lane, 64);
  }
  if (MODE == IN_RESG) {
    __syncthreads();
    if (valid) stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, lane, 64);
  }
  __syncthreads();
  if (!valid) return;
  T acc = 0;
  if (j < nj) {
    T av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = s + u * S;
      av[u] = l < nl ? mv[u] * sv[l] : T(0);
    }
    int l = s + U * S;
    for (; l + (U - 1) * S < nl; l += U * S) {
#pragma unroll
      for (int u = 0; u < U; ++u) mv[u] = __builtin_nontemporal_load(&m[(int64_t)(l + u * S) * ld]);
#pragma unroll
      for (int u = 0; u < U; ++u) av[u] += mv[u] * sv[l + u * S];
    }
    for (; l < nl; l += S) av[0] += __builtin_nontemporal_load(&m[(int64_t)l * ld]) * sv[l];
    acc = ((av[0] + av[1]) + (av[2] + av[3])) + ((av[4] + av[5]) + (av[6] + av[7]));
  }
  for (int o = G; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (s == 0 && j < nj) {
    T* dst = out + op.obase[a] + j;
    *dst = ADD ? *dst + acc : acc;
  }
}

// Narrow form with one aggregate per lane group (every lj_a <= G < 64): a
// wavefront takes 64/G aggregates, lane group s owning the s-th; each lane
// runs the whole loop over l for its output (U loads in flight), so a
// wavefront carries 64/G aggregates' loads through each memory round trip.
// LDS: 4 * (64/G) * (lmax + emax) * sizeof(T).
template <typename T, int MODE, bool ADD, int G>
__global__ void __launch_bounds__(kBlock) k_gemv_narrow_m(int64_t nagg, GemvOp op, int lmax,
                                                          int emax, InSpec<T> spec,
                                                          const T* __restrict__ M,
                                                          const T* __restrict__ in,
                                                          T* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int S = 64 / G;
  constexpr int U = 8;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = lane / G, j = lane % G;
  const int64_t a = (xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + wave) * S + s;
  const bool valid = a < nagg;
  T* sv = reinterpret_cast<T*>(smem_raw) + (size_t)(wave * S + s) * (lmax + emax);
  T* pr = sv + lmax;
  int nj = 0, nl = 0;
  int64_t ib = 0, ld = 0;
  const T* m = M;
  T mv[U];
  if (valid) {
    nj = op.lj[a];
    nl = op.ll[a];
    m = M + op.moff[a] + (j < nj ? j : 0);
    ld = mrow(nj, op.pad);
#pragma unroll
    for (int u = 0; u < U; ++u) mv[u] = (j < nj && u < nl) ? m[(int64_t)u * ld] : T(0);
    ib = op.ibase[a];
    if (MODE == IN_RESG)
      stage_products<T, MODE>(pr, ib, nl, spec, j, G);
    else
      stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, j, G);
  }
  if (MODE == IN_RESG) {
    __syncthreads();
    if (valid) stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, j, G);
  }
  __syncthreads();
  if (!valid || j >= nj) return;
  T av[U];
#pragma unroll
  for (int u = 0; u < U; ++u) av[u] = u < nl ? mv[u] * sv[u] : T(0);
  int l = U;
  for (; l + U - 1 < nl; l += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) mv[u] = m[(int64_t)(l + u) * ld];
#pragma unroll
    for (int u = 0; u < U; ++u) av[u] += mv[u] * sv[l + u];
  }
  for (; l < nl; ++l) av[0] += m[(int64_t)l * ld] * sv[l];
  const T acc = ((av[0] + av[1]) + (av[2] + av[3])) + ((av[4] + av[5]) + (av[6] + av[7]));
  T* dst = out + op.obase[a] + j;
  *dst = ADD ? *dst + acc : acc;
}

// Narrow form with 16-byte loads (every lj_a <= 64): one wavefront per
// aggregate, four aggregates per workgroup.  With V = 16 / sizeof(T)
// outputs per vector, the lanes of a wavefront are Q = ceil(lj/V) output
// vectors by LG = 64/Q row groups; lane (g, q) loads rows l = g, g+LG, ...
// of output vector q (rows are padded to multiples of 4 entries and blocks
// start 16-byte aligned), U rows in flight, so one load instruction moves a
// contiguous stretch of the aggregate's block.  The LG partial vectors of
// each q are then added in row-group order through LDS.
// LDS per wavefront: (round4(lmax + emax) + 64 V) * sizeof(T).
template <typename T, int MODE, bool ADD>
__global__ void __launch_bounds__(kBlock) k_gemv_narrow4(int64_t nagg, GemvOp op, int lmax,
                                                         int emax, InSpec<T> spec,
                                                         const T* __restrict__ M,
                                                         const T* __restrict__ in,
                                                         T* __restrict__ out) {
  constexpr int V = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(V)));
  constexpr int U = 4;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t a = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + wave;
  const bool valid = a < nagg;
  const int stride = ((lmax + emax + 3) & ~3) + 64 * V;
  T* sv = reinterpret_cast<T*>(smem_raw) + (size_t)wave * stride;
  T* pr = sv + lmax;
  vec* red = reinterpret_cast<vec*>(sv + ((lmax + emax + 3) & ~3));
  int nj = 0, nl = 0, Q = 1, LG = 64, g = 0, q = 0;
  int64_t ib = 0, ld = 0;
  const T* m = M;
  vec mv[U];
  const vec zero = {};
  if (valid) {
    nj = op.lj[a];
    nl = op.ll[a];
    Q = (nj + V - 1) / V;
    LG = 64 / Q;
    g = lane / Q;
    q = lane % Q;
    ld = mrow(nj, op.pad);
    m = M + op.moff[a] + V * q;
    // the first U rows of the lane do not depend on the staged input
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = g + u * LG;
      mv[u] = (g < LG && l < nl) ? __builtin_nontemporal_load((const vec*)(m + (int64_t)l * ld))
                                 : zero;
    }
    ib = op.ibase[a];
    if (MODE == IN_RESG)
      stage_products<T, MODE>(pr, ib, nl, spec, lane, 64);
    else
      stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, lane, 64);
  }
  if (MODE == IN_RESG) {
    __syncthreads();
    if (valid) stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, lane, 64);
  }
  __syncthreads();
  vec acc = zero;
  if (valid && g < LG) {
    vec av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = g + u * LG;
      av[u] = l < nl ? mv[u] * sv[l] : zero;
    }
    int l = g + U * LG;
    for (; l + (U - 1) * LG < nl; l += U * LG) {
#pragma unroll
      for (int u = 0; u < U; ++u)
        mv[u] = __builtin_nontemporal_load((const vec*)(m + (int64_t)(l + u * LG) * ld));
#pragma unroll
      for (int u = 0; u < U; ++u) av[u] += mv[u] * sv[l + u * LG];
    }
    for (; l < nl; l += LG) av[0] += __builtin_nontemporal_load((const vec*)(m + (int64_t)l * ld)) * sv[l];
    acc = (av[0] + av[1]) + (av[2] + av[3]);
  }
  red[lane] = acc;
  __syncthreads();
  if (valid && g == 0 && q < Q) {
    vec t = red[q];
    for (int gg = 1; gg < LG; ++gg) t += red[gg * Q + q];
    T* dst = out + op.obase[a] + V * q;
#pragma unroll
    for (int k = 0; k < V; ++k)
      if (V * q + k < nj) dst[k] = ADD ? dst[k] + t[k] : t[k];
  }
}

// Wide form: one workgroup of NW wavefronts per task (aggregate a, 64-wide
// slice j0 of its outputs); the waves split the loop over l and their
// partial sums are added in wave order through LDS.
// LDS: (lmax + emax + NW*64) * sizeof(T).
template <typename T, int MODE, bool ADD, int NW>
__global__ void __launch_bounds__(NW * 64) k_gemv_wide(const int32_t* __restrict__ task_a,
                                                       const int32_t* __restrict__ task_j0,
                                                       GemvOp op, int lmax, int emax,
                                                       InSpec<T> spec,
                                                       const T* __restrict__ M,
                                                       const T* __restrict__ in,
                                                       T* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  T* sv = reinterpret_cast<T*>(smem_raw);
  T* pr = sv + lmax;
  T* part = pr + emax;
  const int64_t task = xcd_block(blockIdx.x, gridDim.x);
  const int64_t a = task_a[task];
  const int j0 = task_j0[task];
  const int nj = op.lj[a], nl = op.ll[a];
  const int64_t ib = op.ibase[a];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = j0 + lane;
  constexpr int U = 8;                      // independent loads in flight per lane
  const T* m = M + op.moff[a] + (j < nj ? j : 0);
  const int64_t ld = mrow(nj, op.pad);
  // the first U matrix entries of the lane do not depend on the staged input:
  // their loads are issued before the staging gather and barrier
  T mv0[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int l = wave + u * NW;
    mv0[u] = (j < nj && l < nl) ? __builtin_nontemporal_load(&m[(int64_t)l * ld]) : T(0);
  }
  if (MODE == IN_RESG) {
    stage_products<T, MODE>(pr, ib, nl, spec, threadIdx.x, NW * 64);
    __syncthreads();
  }
  stage_inputs<T, MODE>(sv, pr, in, ib, nl, spec, threadIdx.x, NW * 64);
  __syncthreads();
  T acc = 0;
  if (j < nj) {
    T av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = wave + u * NW;
      av[u] = l < nl ? mv0[u] * sv[l] : T(0);
    }
    int l = wave + U * NW;
    for (; l + (U - 1) * NW < nl; l += U * NW) {
      T mv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) mv[u] = __builtin_nontemporal_load(&m[(int64_t)(l + u * NW) * ld]);
#pragma unroll
      for (int u = 0; u < U; ++u) av[u] += mv[u] * sv[l + u * NW];
    }
    for (; l < nl; l += NW) av[0] += __builtin_nontemporal_load(&m[(int64_t)l * ld]) * sv[l];
#pragma unroll
    for (int w = U / 2; w > 0; w >>= 1)     // fixed pairwise tree over the U partial sums
#pragma unroll
      for (int u = 0; u < w; ++u) av[u] += av[u + w];
    acc = av[0];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  if (wave == 0 && j < nj) {
    T t = part[lane];
    for (int w = 1; w < NW; ++w) t += part[w * 64 + lane];
    T* dst = out + op.obase[a] + j;
    *dst = ADD ? *dst + t : t;
  }
}

// Wide form with four outputs per lane (FP32, padded rows): a task covers up
// to 256 consecutive outputs, lane L taking outputs j0 + 4L .. j0 + 4L + 3
// with one 16-byte load per matrix row (rows are padded to a multiple of 4
// entries and start 16-byte aligned, so the load never leaves the block); the
// NW waves split the loop over l and their partial sums are added in wave
// order through LDS.  LDS: (round_up(lmax + emax, 4) + NW*256) * 4 bytes.
template <int MODE, bool ADD, int NW>
__global__ void __launch_bounds__(NW * 64) k_gemv_wide4(const int32_t* __restrict__ task_a,
                                                        const int32_t* __restrict__ task_j0,
                                                        GemvOp op, int lmax, int emax,
                                                        InSpec<float> spec,
                                                        const float* __restrict__ M,
                                                        const float* __restrict__ in,
                                                        float* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  float* sv = reinterpret_cast<float*>(smem_raw);
  float* pr = sv + lmax;
  float* part = sv + ((lmax + emax + 3) & ~3);      // 16-byte aligned
  const int64_t task = xcd_block(blockIdx.x, gridDim.x);
  const int64_t a = task_a[task];
  const int j0 = task_j0[task];
  const int nj = op.lj[a], nl = op.ll[a];
  const int64_t ib = op.ibase[a];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = j0 + 4 * lane;
  const bool jv = j < nj;
  const int64_t ld = mrow(nj, op.pad);
  const float* m = M + op.moff[a] + (jv ? j : 0);
  constexpr int U = 8;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 mv0[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int l = wave + u * NW;
    mv0[u] = (jv && l < nl) ? __builtin_nontemporal_load((const f32x4*)(m + (int64_t)l * ld)) : zero;
  }
  if (MODE == IN_RESG) {
    stage_products<float, MODE>(pr, ib, nl, spec, threadIdx.x, NW * 64);
    __syncthreads();
  }
  stage_inputs<float, MODE>(sv, pr, in, ib, nl, spec, threadIdx.x, NW * 64);
  __syncthreads();
  f32x4 acc = zero;
  if (jv) {
    f32x4 av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = wave + u * NW;
      av[u] = l < nl ? mv0[u] * sv[l] : zero;
    }
    int l = wave + U * NW;
    for (; l + (U - 1) * NW < nl; l += U * NW) {
      f32x4 mv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) mv[u] = __builtin_nontemporal_load((const f32x4*)(m + (int64_t)(l + u * NW) * ld));
#pragma unroll
      for (int u = 0; u < U; ++u) av[u] += mv[u] * sv[l + u * NW];
    }
    for (; l < nl; l += NW) av[0] += __builtin_nontemporal_load((const f32x4*)(m + (int64_t)l * ld)) * sv[l];
#pragma unroll
    for (int w = U / 2; w > 0; w >>= 1)     // fixed pairwise tree over the U partial sums
#pragma unroll
      for (int u = 0; u < w; ++u) av[u] += av[u + w];
    acc = av[0];
  }
  *(f32x4*)(part + (wave * 64 + lane) * 4) = acc;
  __syncthreads();
  if (wave == 0 && jv) {
    f32x4 t = *(const f32x4*)(part + lane * 4);
    for (int w = 1; w < NW; ++w) t += *(const f32x4*)(part + (w * 64 + lane) * 4);
    float* dst = out + op.obase[a] + j;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (j + k < nj) dst[k] = ADD ? dst[k] + t[k] : t[k];
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
// A = G^T G on a coarse level in one pass over the stored rows.  A coarse
// G_l is stored as row groups; group g covers the support columns supp_g
// (c of them) with an upper-trapezoidal block R_g (row t holds columns
// t..c-1), so A_l = sum_g R_g^T R_g.  A task is a range of rows [t0, t0+nr)
// of one group; it forms y_t = R_g[t, :] x(supp_g) for its rows and stages
// its contribution sum_t R_g[t, j] y_t to unknown supp_g[j] (t0 <= j < c) at
// stg[soff + j - t0].  Each matrix entry is read once and used for both
// products from registers; the consumer sums the staged values of an unknown
// in a fixed order.  Row t0+i of a task starts at
// vstart + i*(c - t0) - i*(i-1)/2, so the loop has no pointer loads.
// ---------------------------------------------------------------------------
struct GrpTasks {
  const int64_t* vstart;   // value offset of the task's first row
  const int32_t* nrow;     // rows in the task
  const int32_t* t0;       // index of the first row within its group
  const int32_t* c;        // support size of the group
  const int64_t* s0;       // offset of the group's support list
  const int64_t* soff;     // staging offset of the task
};

// Small groups: LW lanes per task of at most RW rows, lane chunk k covers
// j = t0 + lane + k*LW.  Every row of the task is loaded before any product
// is formed, so a task costs one memory round trip for its matrix entries.
template <typename T, int LW, int KC, int RW>
__global__ void __launch_bounds__(kBlock) k_grp_ata(int64_t ntask, GrpTasks tk,
                                                    const T* __restrict__ val,
                                                    const int32_t* __restrict__ supp,
                                                    const T* __restrict__ x,
                                                    T* __restrict__ stg) {
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t task = gid / LW;
  const int lane = (int)(gid % LW);
  if (task >= ntask) return;    // LW divides the wavefront: whole lane groups exit
  const int nr = tk.nrow[task], t0 = tk.t0[task], c = tk.c[task];
  const int w = c - t0;
  const int64_t v0 = tk.vstart[task];
  // support indices first: the x gather waits only for them, not for the
  // matrix entries issued after them
  const int32_t* sp = supp + tk.s0[task] + t0;
  int32_t col[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int q = lane + k * LW;
    col[k] = sp[q < w ? q : 0];
  }
  // local row i holds local columns q = i..w-1 at v0 + i*w - i*(i-1)/2 + (q - i);
  // out-of-range lanes load the task's first entry and discard it (no branches)
  T rv[RW][KC];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int64_t o = v0 + (int64_t)i * w - (int64_t)i * (i - 1) / 2 - i;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int q = lane + k * LW;
      const bool ok = i < nr && q >= i && q < w;
      const T v = val[ok ? o + q : v0];
      rv[i][k] = ok ? v : T(0);
    }
  }
  T xv[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int q = lane + k * LW;
    const T v = x[col[k]];
    xv[k] = q < w ? v : T(0);
  }
  T y[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    T p = 0;
#pragma unroll
    for (int k = 0; k < KC; ++k) p += rv[i][k] * xv[k];
    y[i] = p;
  }
#pragma unroll
  for (int i = 0; i < RW; ++i) y[i] = wave_sum(y[i], LW);
  T* dst = stg + tk.soff[task];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    T acc = 0;
#pragma unroll
    for (int i = 0; i < RW; ++i) acc += y[i] * rv[i][k];
    const int q = lane + k * LW;
    if (q < w) dst[q] = acc;
  }
}

// Large groups (c - t0 <= 64*KC): one workgroup of NW wavefronts per task of
// at most NW*RW rows; wave v takes local rows v, v+NW, ..., loads them all,
// then forms its products; the waves' partial sums are added in wave
// order through LDS.  LDS: NW*KC*64*sizeof(T).
template <typename T, int KC, int NW, int RW>
__global__ void __launch_bounds__(NW * 64) k_grp_ata_wg(GrpTasks tk, const T* __restrict__ val,
                                                        const int32_t* __restrict__ supp,
                                                        const T* __restrict__ x,
                                                        T* __restrict__ stg) {
  extern __shared__ unsigned char smem_raw[];
  T* red = reinterpret_cast<T*>(smem_raw);     // NW*KC*64
  const int64_t task = xcd_block(blockIdx.x, gridDim.x);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nr = tk.nrow[task], t0 = tk.t0[task], c = tk.c[task];
  const int w = c - t0;
  const int64_t v0 = tk.vstart[task];
  const int32_t* sp = supp + tk.s0[task] + t0;
  int32_t col[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int q = lane + 64 * k;
    col[k] = sp[q < w ? q : 0];
  }
  T rv[RW][KC];
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    const int i = wave + NW * u;      // rows dealt round-robin over the waves
    const int64_t o = v0 + (int64_t)i * w - (int64_t)i * (i - 1) / 2 - i;
#pragma unroll
    for (int k = 0; k < KC; ++k) {
      const int q = lane + 64 * k;
      const bool ok = i < nr && q >= i && q < w;
      const T v = val[ok ? o + q : v0];
      rv[u][k] = ok ? v : T(0);
    }
  }
  T xv[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int q = lane + 64 * k;
    const T v = x[col[k]];
    xv[k] = q < w ? v : T(0);
  }
  T y[RW];
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    T p = 0;
#pragma unroll
    for (int k = 0; k < KC; ++k) p += rv[u][k] * xv[k];
    y[u] = p;
  }
#pragma unroll
  for (int u = 0; u < RW; ++u) y[u] = wave_sum(y[u], 64);
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    T acc = 0;
#pragma unroll
    for (int u = 0; u < RW; ++u) acc += y[u] * rv[u][k];
    red[(wave * KC + k) * 64 + lane] = acc;
  }
  __syncthreads();
  T* dst = stg + tk.soff[task];
  for (int q = threadIdx.x; q < w; q += NW * 64) {
    const int k = q >> 6, ln = q & 63;
    T t = 0;
    for (int v = 0; v < NW; ++v) t += red[(v * KC + k) * 64 + ln];
    dst[q] = t;
  }
}

// r = b - (sum of the staged values of each unknown).  8 lanes per unknown
// split its list (lane l takes entries l, l+8, ...) and are added in a fixed
// tree order.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_resid_stg(int64_t n, const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ pos,
                                                      const T* __restrict__ stg,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ r) {
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t i = gid >> 3;
  const int lane = (int)(gid & 7);
  if (i >= n) return;          // whole groups of 8 lanes exit together
  T t = 0;
  for (int64_t e = ptr[i] + lane; e < ptr[i + 1]; e += 8) t += stg[pos[e]];
  t = wave_sum(t, 8);
  if (lane == 0) r[i] = b[i] - t;
}

// ---------------------------------------------------------------------------
// Symmetric dense level operator S (the coarsest inverse or the dense tail)
// in packed 64x64 tiles: only the tiles (I, J) with J <= I are stored (S
// zero-padded to nT = ceil(n/64) tiles per side), each row-major and
// contiguous, tile (I, J) at (I(I+1)/2 + J) * 4096.  y = S x reads every
// stored tile once: the workgroup of tile (I, J) adds S_IJ x_J to row block I
// and, off the diagonal, S_IJ^T x_I to row block J, each into its own slot of
// part (slot J of block I, slot I of block J), so that every slot of every
// row block is written exactly once; k_sym_reduce then adds the nT slots of
// each row in slot order (deterministic, no atomics).  Half the bytes of the
// full matrix, and 16-byte aligned loads.
// ---------------------------------------------------------------------------
constexpr int kTile = 64;

__device__ __forceinline__ void tile_ij(int64_t t, int& I, int& J) {
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  I = i;
  J = (int)(t - (int64_t)i * (i + 1) / 2);
}

// one workgroup per stored tile: S_packed(I, J) = A(I, J) (A row-major n x n)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sym_pack(int64_t n, const double* __restrict__ A,
                                                     T* __restrict__ S) {
  int I, J;
  tile_ij(blockIdx.x, I, J);
  T* dst = S + (int64_t)blockIdx.x * kTile * kTile;
  for (int e = threadIdx.x; e < kTile * kTile; e += kBlock) {
    const int64_t r = (int64_t)I * kTile + e / kTile, c = (int64_t)J * kTile + e % kTile;
    dst[e] = (r < n && c < n) ? (T)A[r * n + c] : T(0);
  }
}

template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ p, T (&m)[4]);
template <>
__device__ __forceinline__ void load4<float>(const float* __restrict__ p, float (&m)[4]) {
  typedef float v4 __attribute__((ext_vector_type(4)));
  const v4 t = *(const v4*)p;
  m[0] = t[0];
  m[1] = t[1];
  m[2] = t[2];
  m[3] = t[3];
}
template <>
__device__ __forceinline__ void load4<double>(const double* __restrict__ p, double (&m)[4]) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 t0 = *(const v2*)p, t1 = *(const v2*)(p + 2);
  m[0] = t0[0];
  m[1] = t0[1];
  m[2] = t1[0];
  m[3] = t1[1];
}

// part: nT slots of nT*64 values.  Lane l of wave w holds the 4x4 block of
// the tile at rows 4*rb .. 4*rb+3, columns 4*cb .. 4*cb+3 with cb = l % 16 and
// rb = 4*w + l / 16: the sixteen lanes of a row group read 256 contiguous
// bytes per row.  Row sums (S_IJ x_J) reduce over cb inside the wave;
// column sums (S_IJ^T x_I) reduce over rb across lanes, then over the four
// wavefronts through LDS; every sum is taken in a fixed order.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sym_gemv(int64_t n, int nT, const T* __restrict__ S,
                                                     const T* __restrict__ x,
                                                     T* __restrict__ part) {
  __shared__ T sm[4][kTile];
  int I, J;
  tile_ij(blockIdx.x, I, J);
  const int64_t npad = (int64_t)nT * kTile;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cb = lane & 15, rb = 4 * w + (lane >> 4);
  const T* src = S + (int64_t)blockIdx.x * kTile * kTile + (4 * rb) * kTile + 4 * cb;
  T m[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i) load4<T>(src + i * kTile, m[i]);
  const int64_t r0 = (int64_t)I * kTile + 4 * rb, c0 = (int64_t)J * kTile + 4 * cb;
  T xc[4], xr[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    xc[k] = c0 + k < n ? x[c0 + k] : T(0);
    xr[k] = r0 + k < n ? x[r0 + k] : T(0);
  }
  // S_IJ x_J: rows 4rb + i, summed over the 16 lanes of the row group
  T d[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    d[i] = (m[i][0] * xc[0] + m[i][1] * xc[1]) + (m[i][2] * xc[2] + m[i][3] * xc[3]);
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) d[i] += __shfl_xor(d[i], o);
  }
  if (cb < 4) part[(int64_t)J * npad + r0 + cb] = cb == 0 ? d[0] : cb == 1 ? d[1] : cb == 2 ? d[2] : d[3];
  if (I != J) {                    // uniform over the workgroup
    // S_IJ^T x_I: columns 4cb + k, summed over the rows of the lane, the four
    // row groups of the wave, then the four waves
    T t[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      t[k] = (m[0][k] * xr[0] + m[1][k] * xr[1]) + (m[2][k] * xr[2] + m[3][k] * xr[3]);
      t[k] += __shfl_xor(t[k], 16);
      t[k] += __shfl_xor(t[k], 32);
    }
    if (lane < 16) {
#pragma unroll
      for (int k = 0; k < 4; ++k) sm[w][4 * cb + k] = t[k];
    }
    __syncthreads();
    if (threadIdx.x < kTile)
      part[(int64_t)I * npad + (int64_t)J * kTile + threadIdx.x] =
          (sm[0][threadIdx.x] + sm[1][threadIdx.x]) + (sm[2][threadIdx.x] + sm[3][threadIdx.x]);
  }
}

// y[i] = sum over the nT slots s of part[s*npad + i] in a fixed order: a
// workgroup takes 16 rows; thread (g, i) adds slots g, g + 16, ...; the 16
// partial sums of a row are then added in g order.  Grid: ceil(npad / 16).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_sym_reduce(int64_t n, int nT, const T* __restrict__ part,
                                                       T* __restrict__ y) {
  __shared__ T sm[16][16];
  const int il = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int64_t i = (int64_t)blockIdx.x * 16 + il;
  const int64_t npad = (int64_t)nT * kTile;
  T t = 0;
  for (int s = g; s < nT; s += 16) t += part[(int64_t)s * npad + i];
  sm[g][il] = t;
  __syncthreads();
  if (g == 0 && i < n) {
    T u = 0;
    for (int q = 0; q < 16; ++q) u += sm[q][il];
    y[i] = u;
  }
}

// Dense tail construction: E = columns j0..j0+NB-1 of the identity in the
// interleaved n x NB layout of the multi-right-hand-side path.
template <int NB>
__global__ void __launch_bounds__(kBlock) k_unit_block(int64_t n, int64_t j0,
                                                       double* __restrict__ E) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= n * NB) return;
  const int64_t i = gid / NB;
  const int c = (int)(gid % NB);
  E[gid] = (i == j0 + c) ? 1.0 : 0.0;
}

// M[:, j0 + c] = X[:, c] for the columns that exist (M column-major n x n)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_scatter_cols(int64_t n, int64_t j0,
                                                         const double* __restrict__ X,
                                                         double* __restrict__ M) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= n * NB) return;
  const int64_t i = gid / NB;
  const int c = (int)(gid % NB);
  if (j0 + c < n) M[(j0 + c) * n + i] = X[gid];
}

// M = (M + M^T) / 2 in place (the tail operator is symmetric in exact
// arithmetic; this removes the rounding asymmetry, so row- and column-major
// reads agree)
__global__ void __launch_bounds__(kBlock) k_symmetrize(int64_t n, double* __restrict__ M) {
  const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (gid >= n * n) return;
  const int64_t i = gid / n, j = gid % n;
  if (i >= j) return;
  const double v = 0.5 * (M[i * n + j] + M[j * n + i]);
  M[i * n + j] = v;
  M[j * n + i] = v;
}

// ---------------------------------------------------------------------------
// Fused FP64 CG kernels.  A dot product is produced as one partial sum per
// workgroup (part[blockIdx.x]); the kernel that needs the scalar re-adds the
// partials itself, every workgroup in the same fixed order, so the value is
// identical everywhere and deterministic, with no atomics and no fences.
// All CG kernels run on the same grid of np = gridDim.x <= 1024 workgroups.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sm[kBlock / 64];
  __shared__ double tot;
  v = wave_sum(v, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < kBlock / 64; ++w) s += sm[w];
    tot = s;
  }
  __syncthreads();
  return tot;
}

// sum of np partials, same value in every workgroup and thread
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int np) {
  double s = 0;
  for (int i = threadIdx.x; i < np; i += kBlock) s += part[i];
  return block_sum(s);
}

__device__ __forceinline__ void write_part(double v, double* __restrict__ part) {
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// partials of a . b
__global__ void __launch_bounds__(kBlock) k_dot(int64_t n, const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ part) {
  double v = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    v += a[i] * b[i];
  write_part(v, part);
}

// q = G^T y (finest level, CSR of G^T, LANES threads per row) and partials
// of p . q
template <int LANES>
__global__ void __launch_bounds__(kBlock) k_cg_apq(int64_t n, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ p,
                                                   double* __restrict__ q,
                                                   double* __restrict__ part) {
  const int lane = threadIdx.x % LANES;
  const int64_t groups = (int64_t)gridDim.x * (kBlock / LANES);
  double v = 0;
  for (int64_t row = (int64_t)blockIdx.x * (kBlock / LANES) + threadIdx.x / LANES; row < n;
       row += groups) {
    double s = 0;
    for (int64_t e = ptr[row] + lane; e < ptr[row + 1]; e += LANES) s += val[e] * y[col[e]];
    if (LANES > 1) s = wave_sum(s, LANES);
    if (lane == 0) {
      q[row] = s;
      v += s * p[row];
    }
  }
  write_part(v, part);
}

// alpha = rho / pq from the partials; x += alpha p; r -= alpha q;
// r32 = (float) r (if given); partials of r . r; pq_keep (if given) receives
// a copy of the p . q partials (the flexible-CG denominator, which the next
// A-apply would overwrite)
__global__ void __launch_bounds__(kBlock) k_cg_update(int64_t n, const double* __restrict__ rz_part,
                                                      const double* __restrict__ pq_part,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      float* __restrict__ r32,
                                                      double* __restrict__ rr_part,
                                                      double* __restrict__ pq_keep) {
  const int np = gridDim.x;
  // the first element's operands do not depend on alpha: loaded before the
  // partial sums are reduced, so the two latencies overlap
  const int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double p0 = 0, q0 = 0, x0 = 0, r0 = 0;
  if (i0 < n) {
    p0 = p[i0];
    q0 = q[i0];
    x0 = x[i0];
    r0 = r[i0];
  }
  const double alpha = sum_parts(rz_part, np) / sum_parts(pq_part, np);
  if (pq_keep && blockIdx.x == 0)
    for (int i = threadIdx.x; i < np; i += kBlock) pq_keep[i] = pq_part[i];
  double v = 0;
  for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * kBlock) {
    const bool pre = i == i0;
    x[i] = (pre ? x0 : x[i]) + alpha * (pre ? p0 : p[i]);
    const double ri = (pre ? r0 : r[i]) - alpha * (pre ? q0 : q[i]);
    r[i] = ri;
    if (r32) r32[i] = (float)ri;
    v += ri * ri;
  }
  write_part(v, rr_part);
}

// z = xv + staged RAS-T contributions (the finest level's V-cycle output in
// the V-cycle precision T, widened to FP64); partials of r . z, and with q
// given the partials of -(z . q) (the flexible-CG numerator, q = A p_old)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_cg_z(int64_t n, const T* __restrict__ xv,
                                                 const int64_t* __restrict__ cptr,
                                                 const int64_t* __restrict__ cpos,
                                                 const T* __restrict__ tb,
                                                 const double* __restrict__ r,
                                                 double* __restrict__ z,
                                                 double* __restrict__ rz_part,
                                                 const double* __restrict__ q,
                                                 double* __restrict__ zq_part) {
  double v = 0, w = 0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    T s = xv[i];
    if (cptr)
      for (int64_t e = cptr[i]; e < cptr[i + 1]; ++e) s += tb[cpos[e]];
    const double zi = (double)s;
    z[i] = zi;
    v += r[i] * zi;
    if (q) w += zi * q[i];
  }
  write_part(v, rz_part);
  if (q) write_part(-w, zq_part);
}

// p = z + beta p with beta = rho_new / rho_old (rho_old_part == nullptr: p = z)
__global__ void __launch_bounds__(kBlock) k_cg_dir(int64_t n,
                                                   const double* __restrict__ rz_new,
                                                   const double* __restrict__ rz_old,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ p) {
  const int np = gridDim.x;
  const double beta = rz_old ? sum_parts(rz_new, np) / sum_parts(rz_old, np) : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = rz_old ? z[i] + beta * p[i] : z[i];   // first direction: p = z
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

__global__ void __launch_bounds__(kBlock) k_fill_f32(int64_t n, float v, float* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) b[i] = v;
}

}  // namespace dev
}  // namespace lsamg
