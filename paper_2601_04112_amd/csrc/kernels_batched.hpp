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

// With NB = 64 a wavefront works on one row (or unknown) at a time; the
// index is then made explicitly wave-uniform, so that the row's CSR
// pointers, column indices and values are fetched by scalar loads once per
// wavefront and only the gathers of the NB vector values use vector loads.
// Callers keep row counts below 2^31.
template <int NB>
__device__ __forceinline__ int64_t wave_row(int64_t r) {
  if constexpr (NB == 64)
    return (int64_t)__builtin_amdgcn_readfirstlane((int)r);
  else
    return r;
}

// Value of v held by lane L (L wave-uniform): a scalar register.
__device__ __forceinline__ int32_t lane_val(int32_t v, int L) {
  return __builtin_amdgcn_readlane(v, L);
}
__device__ __forceinline__ float lane_val(float v, int L) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}
__device__ __forceinline__ double lane_val(double v, int L) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), L);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), L);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Sum of the staged values tb[pos[e]][lane] for e in [e0, e1) (NB = 64, e0
// and e1 wave-uniform), in e order: lane k loads pos[e0 + k], and the
// wavefront walks the positions, each broadcast from its lane.
template <typename T>
__device__ __forceinline__ T staged_sum64(int64_t e0, int64_t e1, const int64_t* __restrict__ pos,
                                          const T* __restrict__ tb, int lane) {
  T s = 0;
  for (int64_t b = e0; b < e1; b += 64) {
    const int cnt = (int)(e1 - b < 64 ? e1 - b : 64);
    const int64_t p = pos[b + (lane < cnt ? lane : cnt - 1)];
    const int plo = (int)(p & 0xffffffff), phi = (int)(p >> 32);
    for (int L = 0; L < cnt; ++L) {
      const int64_t q = ((int64_t)__builtin_amdgcn_readlane(phi, L) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane(plo, L);
      s += tb[q * 64 + lane];
    }
  }
  return s;
}

// NB = 64, one row per wavefront (e0, e1 wave-uniform): the lanes load 64
// entries of the row (indices and values) with one vector load each, and the
// wavefront then walks them, each entry's index and value broadcast from its
// lane, gathering one 64-wide row of X per entry.
template <typename T>
__device__ __forceinline__ T row_dot64(int64_t e0, int64_t e1, const int32_t* __restrict__ col,
                                       const T* __restrict__ val, const T* __restrict__ X,
                                       int lane) {
  // 16 gathers in flight per round; entries past the row end repeat its last
  // index (an L1 hit) with a zero weight
  constexpr int U = 16;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int64_t b = e0; b < e1; b += 64) {
    const int cnt = (int)(e1 - b < 64 ? e1 - b : 64);
    const int64_t f = b + (lane < cnt ? lane : cnt - 1);
    const int32_t c = col[f];
    const T v = lane < cnt ? val[f] : T(0);
    for (int L = 0; L < cnt; L += U) {
      T x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = L + u < cnt ? L + u : cnt - 1;
        x[u] = X[(int64_t)lane_val(c, k) * 64 + lane];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc[u & 3] += lane_val(v, (L + u) & 63) * x[u];
    }
  }
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// sum over e in [e0, e1) of val[e] * X[col[e]][j]: eight entries at a time,
// all their indices and values loaded before the gathers are issued, so a
// wavefront keeps eight gathers in flight
template <typename T, int NB>
__device__ __forceinline__ T row_dot(int64_t e0, int64_t e1, const int32_t* __restrict__ col,
                                     const T* __restrict__ val, const T* __restrict__ X, int j) {
  constexpr int U = 8;
  T acc[U];
#pragma unroll
  for (int u = 0; u < U; ++u) acc[u] = 0;
  int64_t e = e0;
  for (; e + U <= e1; e += U) {
    int32_t c[U];
    T v[U], x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = col[e + u];
      v[u] = val[e + u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = X[(int64_t)c[u] * NB + j];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] += v[u] * x[u];
  }
  if (e < e1) {                             // remainder: 1 .. U-1 entries, loads clamped
#pragma unroll
    for (int u = 0; u < U - 1; ++u) {
      const int64_t f = e + u < e1 ? e + u : e1 - 1;
      const int32_t c = col[f];
      const T v = val[f];
      acc[u] += (e + u < e1 ? v : T(0)) * X[(int64_t)c * NB + j];
    }
  }
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// Y = G X: one group of NB lanes per row, lanes along the right-hand sides.
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bspmv(int64_t nrows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col,
                                                  const T* __restrict__ val,
                                                  const T* __restrict__ X, T* __restrict__ Y) {
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t row = wave_row<NB>(gid / NB);
  const int j = (int)(gid % NB);
  if (row >= nrows) return;
  if constexpr (NB == 64)
    Y[row * NB + j] = row_dot64<T>(ptr[row], ptr[row + 1], col, val, X, j);
  else
    Y[row * NB + j] = row_dot<T, NB>(ptr[row], ptr[row + 1], col, val, X, j);
}

// R = B - G^T Y (B == nullptr: R = G^T Y)
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bresid_t(int64_t n, const int64_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ col,
                                                     const T* __restrict__ val,
                                                     const T* __restrict__ Y,
                                                     const T* __restrict__ B,
                                                     T* __restrict__ R) {
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t d = wave_row<NB>(gid / NB);
  const int j = (int)(gid % NB);
  if (d >= n) return;
  T s;
  if constexpr (NB == 64)
    s = row_dot64<T>(ptr[d], ptr[d + 1], col, val, Y, j);
  else
    s = row_dot<T, NB>(ptr[d], ptr[d + 1], col, val, Y, j);
  R[d * NB + j] = B ? B[d * NB + j] - s : s;
}

// Y[r] = B[r] - sum_e val[e] X[col[e]] (B == nullptr: Y[r] = the sum) for
// NB = 64 and rows of a few entries: a wavefront takes rpw consecutive rows,
// whose entries are one contiguous CSR range; the lanes load 64 entries of it
// at a time (indices and values, one vector load each) and the row pointers
// of the wave's rows, the wavefront issues 16 gathers, then walks the
// entries in order, writing each row as soon as its last entry is added
// (row boundaries are wave-uniform, so the walk has no divergence).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bspmm64(int64_t nrows, int rpw,
                                                    const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const T* __restrict__ X,
                                                    const T* __restrict__ B,
                                                    T* __restrict__ Y) {
  constexpr int U = 16;
  const int lane = threadIdx.x & 63;
  const int64_t w = xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6);
  const int64_t r0 = (int64_t)__builtin_amdgcn_readfirstlane((int)(w * rpw));
  if (r0 >= nrows) return;
  const int nr = (int)(nrows - r0 < rpw ? nrows - r0 : rpw);       // 1 .. rpw <= 63
  // lane k (k <= nr) holds ptr[r0 + k]
  const int64_t pk = ptr[r0 + (lane <= nr ? lane : nr)];
  const int plo = (int)(pk & 0xffffffff), phi = (int)(pk >> 32);
  auto rowptr = [&](int k) -> int64_t {
    return ((int64_t)__builtin_amdgcn_readlane(phi, k) << 32) |
           (uint32_t)__builtin_amdgcn_readlane(plo, k);
  };
  const int64_t eb = rowptr(0), ee = rowptr(nr);
  int k = 0;                          // current row r0 + k
  int64_t rend = rowptr(1);
  T acc = 0;
  for (int64_t b = eb; b < ee; b += 64) {
    const int cnt = (int)(ee - b < 64 ? ee - b : 64);
    const int64_t f = b + (lane < cnt ? lane : cnt - 1);
    const int32_t c = col[f];
    const T v = lane < cnt ? val[f] : T(0);
    for (int L = 0; L < cnt; L += U) {
      T x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = L + u < cnt ? L + u : cnt - 1;
        x[u] = X[(int64_t)lane_val(c, q) * 64 + lane];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (L + u >= cnt) break;
        const int64_t e = b + L + u;
        while (e >= rend) {           // finished rows (empty rows included)
          const int64_t r = r0 + k;
          Y[r * 64 + lane] = B ? B[r * 64 + lane] - acc : acc;
          acc = 0;
          ++k;
          rend = rowptr(k + 1);
        }
        acc += lane_val(v, L + u) * x[u];
      }
    }
  }
  for (; k < nr; ++k) {               // the last row, and trailing empty rows
    const int64_t r = r0 + k;
    Y[r * 64 + lane] = B ? B[r * 64 + lane] - acc : acc;
    acc = 0;
  }
}

// One row of A = G^T G applied to NB interleaved columns (column j) at
// unknown d, for a G whose rows are short (the finest level): the (at most
// ME) rows of G that touch d (its row of G^T) are recomputed, y_r = g_r . X
// (at most MF entries each) from cached entries, so G X is never written to
// memory.  All indices of one level of the chain (G^T entries, row
// pointers, row entries) are loaded before the next level, so the gathers of
// every row are in flight together.
template <typename T, int NB, int ME, int MF>
__device__ __forceinline__ T ata_row(int64_t d, const int64_t* __restrict__ gt_ptr,
                                     const int32_t* __restrict__ gt_col,
                                     const T* __restrict__ gt_val,
                                     const int64_t* __restrict__ g_ptr,
                                     const int32_t* __restrict__ g_col,
                                     const T* __restrict__ g_val, const T* __restrict__ X, int j) {
  // every load is unconditional, from an index clamped into the row (rows
  // and columns of G are never empty), and masked afterwards: no branch
  // separates the loads of one level, so they are issued together
  const int64_t e0 = gt_ptr[d];
  const int ne = (int)(gt_ptr[d + 1] - e0);
  int64_t r[ME], f0[ME];
  int nf[ME];
  T w[ME];
#pragma unroll
  for (int k = 0; k < ME; ++k) {
    const int64_t e = e0 + (k < ne ? k : ne - 1);
    r[k] = gt_col[e];
    const T wv = gt_val[e];
    w[k] = k < ne ? wv : T(0);
  }
#pragma unroll
  for (int k = 0; k < ME; ++k) {
    f0[k] = g_ptr[r[k]];
    nf[k] = (int)(g_ptr[r[k] + 1] - f0[k]);
  }
  int32_t c[ME][MF];
  T v[ME][MF];
#pragma unroll
  for (int k = 0; k < ME; ++k)
#pragma unroll
    for (int q = 0; q < MF; ++q) {
      const int64_t f = f0[k] + (q < nf[k] ? q : nf[k] - 1);
      c[k][q] = g_col[f];
      const T vv = g_val[f];
      v[k][q] = q < nf[k] ? vv : T(0);
    }
  T acc = 0;
#pragma unroll
  for (int k = 0; k < ME; ++k) {
    T y = 0;
#pragma unroll
    for (int q = 0; q < MF; ++q) y += v[k][q] * X[(int64_t)c[k][q] * NB + j];
    acc += w[k] * y;
  }
  return acc;
}

// NB = 64 form of ata_row (d wave-uniform): lane k loads G^T entry k and
// the row pointers of its row r_k; lane k*MF + q loads entry q of row r_k;
// the wavefront then walks the ME*MF entries, each index and value broadcast
// from its lane, gathering X rows: three vector loads of indices in sequence
// instead of a chain of scalar loads per row.
template <typename T, int ME, int MF>
__device__ __forceinline__ T ata_row64(int64_t d, const int64_t* __restrict__ gt_ptr,
                                       const int32_t* __restrict__ gt_col,
                                       const T* __restrict__ gt_val,
                                       const int64_t* __restrict__ g_ptr,
                                       const int32_t* __restrict__ g_col,
                                       const T* __restrict__ g_val, const T* __restrict__ X,
                                       int lane) {
  static_assert(ME * MF <= 64, "one entry per lane");
  const int64_t e0 = gt_ptr[d];
  const int ne = (int)(gt_ptr[d + 1] - e0);
  const int k1 = lane < ne ? lane : ne - 1;                 // columns of G are never empty
  const int32_t r = gt_col[e0 + k1];
  const T wv = gt_val[e0 + k1];
  const T w = lane < ne ? wv : T(0);
  const int64_t f0 = g_ptr[r];
  const int nf = (int)(g_ptr[(int64_t)r + 1] - f0);          // rows of G are never empty
  const int k3 = lane / MF, q3 = lane % MF;
  const int64_t f0k = __shfl(f0, k3);
  const int nfk = __shfl(nf, k3);
  const int32_t c = g_col[f0k + (q3 < nfk ? q3 : nfk - 1)];
  const T vv = g_val[f0k + (q3 < nfk ? q3 : nfk - 1)];
  const T v = (q3 < nfk && k3 < ne) ? vv : T(0);
  T acc = 0;
#pragma unroll
  for (int k = 0; k < ME; ++k) {
    T x[MF];
#pragma unroll
    for (int q = 0; q < MF; ++q) x[q] = X[(int64_t)lane_val(c, k * MF + q) * 64 + lane];
    T y = 0;
#pragma unroll
    for (int q = 0; q < MF; ++q) y += lane_val(v, k * MF + q) * x[q];
    acc += lane_val(w, k) * y;
  }
  return acc;
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
  const int64_t task = xcd_block(blockIdx.x, gridDim.x);
  const int64_t a = task_a[task];
  const int j0 = task_j0[task];
  const int nj = op.lj[a], nl = op.ll[a];
  const int64_t ib = op.ibase[a];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jj = j0 + lane;
  const bool jv = jj < nj;
  const T* m = M + op.moff[a] + (jv ? jj : 0);
  const int64_t ld = mrow(nj, op.pad);
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
        const T mv = m[(int64_t)(l0 + l) * ld];
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

// ---------------------------------------------------------------------------
// Matrix-core form of k_bgemm for the FP32 V-cycle and NB >= 16 right-hand
// sides: every per-aggregate product OUT_a = M_a^T IN_a is tiled into
// v_mfma_f32_16x16x4f32 operations (FP32 operands, FP32 accumulation).
//
// One wavefront runs one task at a time: aggregate a, output rows
// [j0, j0 + 16*RT) (RT row tiles), loop indices [k0, k1), all NB columns
// (CT = NB/16 column tiles); the loads of U loop steps are issued before
// their matrix operations.  The launch is persistent: its waves stride over
// the task list, which the host orders longest-first (size buckets), so one
// launch covers every aggregate of a level.
//
// v_mfma_f32_16x16x4f32 computes D(16x16) += A(16x4) B(4x16); lane L = i +
// 16 g supplies A[i][g] and B[g][i] and receives D[4g + v][i] in acc[v].
// Here A[i][g] = M_a[l][j0 + 16 r + i] and B[g][i] = IN_a[l][CT i + q] with
// l = k + g (row tile r, column tile q): the sixteen lanes of a group read
// 64 contiguous bytes of M_a and 64*CT contiguous bytes of one input row, so
// the input is fetched with one CT-wide vector load per lane, and each
// output row is written back the same way.
//
// Tasks with slot >= 0 (a loop split across waves) store their partial sums
// to part[slot][row][:] (row = obase_a + output index) for k_bmm_reduce; the
// others write (or add to) out.  With a split, every aggregate has one task
// per slot (an empty loop range writes zeros), so every slot of every output
// row is written.
// ---------------------------------------------------------------------------
struct MmTasks {
  const int32_t* a;     // aggregate
  const int32_t* j0;    // first output row
  const int32_t* k0;    // loop range [k0, k1)
  const int32_t* k1;
  const int32_t* slot;  // partial-sum slot, or -1
};


template <int CT>
__device__ __forceinline__ void vload(const float* __restrict__ p, float (&v)[CT]) {
  if constexpr (CT == 4) {
    const f32x4 t = *(const f32x4*)p;
    v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
  } else if constexpr (CT == 2) {
    const f32x2 t = *(const f32x2*)p;
    v[0] = t[0]; v[1] = t[1];
  } else {
    v[0] = *p;
  }
}

template <int CT>
__device__ __forceinline__ void vstore(float* __restrict__ p, const float (&v)[CT]) {
  if constexpr (CT == 4) {
    f32x4 t;
    t[0] = v[0]; t[1] = v[1]; t[2] = v[2]; t[3] = v[3];
    *(f32x4*)p = t;
  } else if constexpr (CT == 2) {
    f32x2 t;
    t[0] = v[0]; t[1] = v[1];
    *(f32x2*)p = t;
  } else {
    *p = v[0];
  }
}

template <int MODE, bool ADD, int RT, int U, int NB>
__global__ void __launch_bounds__(kBlock) k_bmm(MmTasks tk, int ntask, GemvOp op,
                                                const int32_t* __restrict__ gidx,
                                                const int64_t* __restrict__ cptr,
                                                const int64_t* __restrict__ cpos,
                                                const float* __restrict__ tb,
                                                const float* __restrict__ M,
                                                const float* __restrict__ in,
                                                float* __restrict__ out,
                                                float* __restrict__ part, int64_t part_rows) {
  static_assert(NB % 16 == 0 && NB <= 64, "column tiles of 16");
  constexpr int CT = NB / 16;
  constexpr int WPB = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  for (int t = __builtin_amdgcn_readfirstlane((int)xcd_block(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6)); t < ntask;
       t += gridDim.x * WPB) {
    const int a = tk.a[t], j0 = tk.j0[t], k0 = tk.k0[t], k1 = tk.k1[t];
    const int nj = op.lj[a];
    const int64_t ib = op.ibase[a];
    const float* __restrict__ m = M + op.moff[a];
    const int64_t ld = mrow(nj, op.pad);
    f32x4 acc[RT][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int q = 0; q < CT; ++q) acc[r][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k = k0; k < k1; k += 4 * U) {
      float av[U][RT], bv[U][CT];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int l = k + 4 * u + g;
        const bool lv = l < k1;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const int jj = j0 + 16 * r + i;
          av[u][r] = (lv && jj < nj) ? m[(int64_t)l * ld + jj] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < CT; ++q) bv[u][q] = 0.f;
        if (lv) {
          const int64_t e = ib + l;
          const int64_t row = MODE == IN_GATHER ? (int64_t)gidx[e] : e;
          vload<CT>(in + row * NB + CT * i, bv[u]);
          if (MODE == IN_TB) {
            for (int64_t p = cptr[e]; p < cptr[e + 1]; ++p) {
              float w[CT];
              vload<CT>(tb + cpos[p] * NB + CT * i, w);
#pragma unroll
              for (int q = 0; q < CT; ++q) bv[u][q] += w[q];
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int q = 0; q < CT; ++q)
            acc[r][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[u][r], bv[u][q], acc[r][q], 0, 0, 0);
    }
    const int slot = tk.slot[t];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = j0 + 16 * r + 4 * g + v;
        if (jj >= nj) continue;
        float o[CT];
#pragma unroll
        for (int q = 0; q < CT; ++q) o[q] = acc[r][q][v];
        if (slot >= 0) {
          vstore<CT>(part + ((int64_t)slot * part_rows + op.obase[a] + jj) * NB + CT * i, o);
        } else {
          float* d = out + (op.obase[a] + jj) * NB + CT * i;
          if (ADD) {
            float w[CT];
            vload<CT>(d, w);
#pragma unroll
            for (int q = 0; q < CT; ++q) o[q] += w[q];
          }
          vstore<CT>(d, o);
        }
      }
  }
}

template <int CT>
__device__ __forceinline__ void vload(const double* __restrict__ p, double (&v)[CT]) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  if constexpr (CT == 4) {
    const d4 t = *(const d4*)p;
    v[0] = t[0]; v[1] = t[1]; v[2] = t[2]; v[3] = t[3];
  } else if constexpr (CT == 2) {
    const d2 t = *(const d2*)p;
    v[0] = t[0]; v[1] = t[1];
  } else {
    v[0] = *p;
  }
}

template <int CT>
__device__ __forceinline__ void vstore(double* __restrict__ p, const double (&v)[CT]) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  if constexpr (CT == 4) {
    d4 t;
    t[0] = v[0]; t[1] = v[1]; t[2] = v[2]; t[3] = v[3];
    *(d4*)p = t;
  } else if constexpr (CT == 2) {
    d2 t;
    t[0] = v[0]; t[1] = v[1];
    *(d2*)p = t;
  } else {
    *p = v[0];
  }
}

// k_bmm in FP64 on the FP64 matrix cores (v_mfma_f64_16x16x4f64): the same
// tasks (aggregate a, 16 RT output rows from j0, the whole loop; no split),
// inputs formed per MODE, columns CT i .. CT i + CT-1 in lane i.  Result
// register v of lane group g holds output row j0 + 16 r + g + 4 v (the FP64
// form's result lanes).
template <int MODE, bool ADD, int RT, int U, int NB>
__global__ void __launch_bounds__(kBlock) k_bmmd(MmTasks tk, int ntask, GemvOp op,
                                                 const int32_t* __restrict__ gidx,
                                                 const int64_t* __restrict__ cptr,
                                                 const int64_t* __restrict__ cpos,
                                                 const double* __restrict__ tb,
                                                 const double* __restrict__ M,
                                                 const double* __restrict__ in,
                                                 double* __restrict__ out) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  static_assert(NB % 16 == 0 && NB <= 64, "column tiles of 16");
  constexpr int CT = NB / 16;
  constexpr int WPB = kBlock / 64;
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, g = lane >> 4;
  for (int t = __builtin_amdgcn_readfirstlane((int)xcd_block(blockIdx.x, gridDim.x) * WPB + (threadIdx.x >> 6)); t < ntask;
       t += gridDim.x * WPB) {
    const int a = tk.a[t], j0 = tk.j0[t], k0 = tk.k0[t], k1 = tk.k1[t];
    const int nj = op.lj[a];
    const int64_t ib = op.ibase[a];
    const double* __restrict__ m = M + op.moff[a];
    const int64_t ld = mrow(nj, op.pad);
    f64x4 acc[RT][CT];
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int q = 0; q < CT; ++q) acc[r][q] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k = k0; k < k1; k += 4 * U) {
      double av[U][RT], bv[U][CT];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int l = k + 4 * u + g;
        const bool lv = l < k1;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const int jj = j0 + 16 * r + i;
          av[u][r] = (lv && jj < nj) ? m[(int64_t)l * ld + jj] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < CT; ++q) bv[u][q] = 0.0;
        if (lv) {
          const int64_t e = ib + l;
          const int64_t row = MODE == IN_GATHER ? (int64_t)gidx[e] : e;
          vload<CT>(in + row * NB + CT * i, bv[u]);
          if (MODE == IN_TB) {
            for (int64_t p = cptr[e]; p < cptr[e + 1]; ++p) {
              double w[CT];
              vload<CT>(tb + cpos[p] * NB + CT * i, w);
#pragma unroll
              for (int q = 0; q < CT; ++q) bv[u][q] += w[q];
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int r = 0; r < RT; ++r)
#pragma unroll
          for (int q = 0; q < CT; ++q)
            acc[r][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][r], bv[u][q], acc[r][q], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int jj = j0 + 16 * r + g + 4 * v;
        if (jj >= nj) continue;
        double o[CT];
#pragma unroll
        for (int q = 0; q < CT; ++q) o[q] = acc[r][q][v];
        double* d = out + (op.obase[a] + jj) * NB + CT * i;
        if (ADD) {
          double w[CT];
          vload<CT>(d, w);
#pragma unroll
          for (int q = 0; q < CT; ++q) o[q] += w[q];
        }
        vstore<CT>(d, o);
      }
  }
}

// k_bmmd on 64 columns with the input rows staged in LDS: a workgroup per
// task (aggregate a, 64 output rows j0 .. j0+63, the whole loop), its four
// waves 16 rows each.  The loop runs in chunks of 32 input rows (formed per
// MODE as in k_bmmd), staged once per workgroup instead of once per wave
// and double-buffered, the next chunk's loads issued before the current
// chunk's MFMAs.  Operands and result lanes as k_bmmd with CT = 4: lane
// (i, g) of wave w feeds A[i][g] = M[k + g][j0 + 16 w + i] and B[g][i] =
// column 4 i + q of input row k + g for column tile q; result register v of
// lane group g holds output row j0 + 16 w + g + 4 v, columns 4 i .. 4 i + 3.
template <int MODE, bool ADD>
__global__ void __launch_bounds__(kBlock) k_bmmd_lds(MmTasks tk, GemvOp op,
                                                     const int32_t* __restrict__ gidx,
                                                     const int64_t* __restrict__ cptr,
                                                     const int64_t* __restrict__ cpos,
                                                     const double* __restrict__ tb,
                                                     const double* __restrict__ M,
                                                     const double* __restrict__ in,
                                                     double* __restrict__ out) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  constexpr int KC = 32, SB = 64 + 2, KS = KC / 4;
  __shared__ __attribute__((aligned(16))) double sB[2][KC * SB];
  const int64_t t = xcd_block(blockIdx.x, gridDim.x);
  const int a = tk.a[t], j0 = tk.j0[t], k0 = tk.k0[t], k1 = tk.k1[t];
  const int nj = op.lj[a];
  const int64_t ib = op.ibase[a];
  const double* __restrict__ m = M + op.moff[a];
  const int64_t ld = mrow(nj, op.pad);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int jr = j0 + 16 * w + i;            // this lane's output row (A operand row)
  const bool jv = jr < nj;
  const int sr = threadIdx.x >> 3, sc = 8 * (threadIdx.x & 7);   // staging: row sr, 8 columns
  const f64x4 zero = {0.0, 0.0, 0.0, 0.0};
  f64x4 acc[4] = {zero, zero, zero, zero};
  f64x2 bst[4];
  double am[KS];
  auto load_chunk = [&](int kb) {
    const int l = kb + sr;
    const f64x2 z2 = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) bst[c] = z2;
    if (l < k1) {
      const int64_t e = ib + l;
      const int64_t row = MODE == IN_GATHER ? (int64_t)gidx[e] : e;
#pragma unroll
      for (int c = 0; c < 4; ++c) bst[c] = *(const f64x2*)(in + row * 64 + sc + 2 * c);
      if (MODE == IN_TB) {
        for (int64_t p = cptr[e]; p < cptr[e + 1]; ++p)
#pragma unroll
          for (int c = 0; c < 4; ++c) bst[c] += *(const f64x2*)(tb + cpos[p] * 64 + sc + 2 * c);
      }
    }
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int lk = kb + 4 * st + g;
      am[st] = (jv && lk < k1) ? m[(int64_t)lk * ld + jr] : 0.0;
    }
  };
  int buf = 0;
  if (k0 < k1) load_chunk(k0);
  for (int kb = k0; kb < k1; kb += KC) {
#pragma unroll
    for (int c = 0; c < 4; ++c) *(f64x2*)(sB[buf] + sr * SB + sc + 2 * c) = bst[c];
    double av[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) av[st] = am[st];
    __syncthreads();
    if (kb + KC < k1) load_chunk(kb + KC);    // in flight during this chunk's MFMAs
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const double* bp = sB[buf] + (4 * st + g) * SB + 4 * i;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[st], bp[q], acc[q], 0, 0, 0);
    }
    buf ^= 1;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int jj = j0 + 16 * w + g + 4 * v;
    if (jj >= nj) continue;
    double* d = out + (op.obase[a] + jj) * 64 + 4 * i;
    f64x2 o0 = {acc[0][v], acc[1][v]}, o1 = {acc[2][v], acc[3][v]};
    if (ADD) {
      o0 += *(const f64x2*)d;
      o1 += *(const f64x2*)(d + 2);
    }
    *(f64x2*)d = o0;
    *(f64x2*)(d + 2) = o1;
  }
}

// k_bmm on 64 columns with the input rows staged in LDS: a workgroup per
// task (aggregate a, 64 output rows j0 .. j0+63, loop range [k0, k1), slot),
// its four waves 16 rows each.  The loop runs in chunks of 32 input rows
// (formed per MODE as in k_bmm: direct, gathered, or plus the staged RAS-T
// rows), staged once per workgroup instead of once per wave and double-
// buffered, the next chunk's loads issued before the current chunk's MFMAs;
// each wave reads its 16 matrix columns from global memory as k_bmm does.
// Output as k_bmm (columns 4i .. 4i+3 in lane i; slot >= 0: partial sums).
template <int MODE, bool ADD>
__global__ void __launch_bounds__(kBlock) k_bmm_lds(MmTasks tk, GemvOp op,
                                                    const int32_t* __restrict__ gidx,
                                                    const int64_t* __restrict__ cptr,
                                                    const int64_t* __restrict__ cpos,
                                                    const float* __restrict__ tb,
                                                    const float* __restrict__ M,
                                                    const float* __restrict__ in,
                                                    float* __restrict__ out,
                                                    float* __restrict__ part, int64_t part_rows) {
  constexpr int KC = 32, SB = 64 + 4, KS = KC / 4;
  __shared__ __attribute__((aligned(16))) float sB[2][KC * SB];
  const int64_t t = xcd_block(blockIdx.x, gridDim.x);
  const int a = tk.a[t], j0 = tk.j0[t], k0 = tk.k0[t], k1 = tk.k1[t], slot = tk.slot[t];
  const int nj = op.lj[a];
  const int64_t ib = op.ibase[a];
  const float* __restrict__ m = M + op.moff[a];
  const int64_t ld = mrow(nj, op.pad);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int jr = j0 + 16 * w + i;            // this lane's output row (A operand row)
  const bool jv = jr < nj;
  const int sr = threadIdx.x >> 3, sc = 8 * (threadIdx.x & 7);
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc[4] = {zero, zero, zero, zero};
  f32x4 bst[2];
  float am[KS];
  auto load_chunk = [&](int kb) {
    const int l = kb + sr;
    bst[0] = zero;
    bst[1] = zero;
    if (l < k1) {
      const int64_t e = ib + l;
      const int64_t row = MODE == IN_GATHER ? (int64_t)gidx[e] : e;
      bst[0] = *(const f32x4*)(in + row * 64 + sc);
      bst[1] = *(const f32x4*)(in + row * 64 + sc + 4);
      if (MODE == IN_TB) {
        for (int64_t p = cptr[e]; p < cptr[e + 1]; ++p) {
          bst[0] += *(const f32x4*)(tb + cpos[p] * 64 + sc);
          bst[1] += *(const f32x4*)(tb + cpos[p] * 64 + sc + 4);
        }
      }
    }
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const int lk = kb + 4 * st + g;
      am[st] = (jv && lk < k1) ? m[(int64_t)lk * ld + jr] : 0.f;
    }
  };
  int buf = 0;
  if (k0 < k1) load_chunk(k0);
  for (int kb = k0; kb < k1; kb += KC) {
    *(f32x4*)(sB[buf] + sr * SB + sc) = bst[0];
    *(f32x4*)(sB[buf] + sr * SB + sc + 4) = bst[1];
    float av[KS];
#pragma unroll
    for (int st = 0; st < KS; ++st) av[st] = am[st];
    __syncthreads();
    if (kb + KC < k1) load_chunk(kb + KC);    // in flight during this chunk's MFMAs
#pragma unroll
    for (int st = 0; st < KS; ++st) {
      const f32x4 b = *(const f32x4*)(sB[buf] + (4 * st + g) * SB + 4 * i);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[st], b[q], acc[q], 0, 0, 0);
    }
    buf ^= 1;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int jj = j0 + 16 * w + 4 * g + v;
    if (jj >= nj) continue;
    f32x4 o = {acc[0][v], acc[1][v], acc[2][v], acc[3][v]};
    if (slot >= 0) {
      *(f32x4*)(part + ((int64_t)slot * part_rows + op.obase[a] + jj) * 64 + 4 * i) = o;
    } else {
      float* d = out + (op.obase[a] + jj) * 64 + 4 * i;
      if (ADD) o += *(const f32x4*)d;
      *(f32x4*)d = o;
    }
  }
}

// Dense level operator on 64 right-hand sides (FP32 MFMA): OUT = M IN with M
// n x n stored row-major with a padded row stride ld (a multiple of 4,
// padding zero; k_pad_rows makes it), and IN, OUT interleaved n x 64.  A workgroup computes
// a 64-row x 64-column output tile over the loop range [k0, k1) of its split
// (blockIdx.y); its four waves take 16 rows each.  The loop runs in chunks of
// KC: the KC input rows of a chunk are staged once in LDS for all four waves,
// and each lane reads KC/4 entries of its own matrix row with 16-byte loads:
// load v of lane group g takes loop indices kb + 16 v + 4 g + e (e < 4), so
// the four lane groups of a row read 64 contiguous bytes per load and a
// wave streams whole row segments of M.  MFMA step 4 v + e takes those four
// loop indices (one per lane group).  The next chunk's loads are
// issued before the current chunk's MFMAs.  Columns 4i+q of a 16-column tile
// q sit in lane i, as in k_bmm.  Splits > 1 write partial sums to
// part[split][row][:] for k_bmm_reduce (an empty loop range writes zeros).
template <int KC>
__global__ void __launch_bounds__(kBlock) k_dense_mm64(int64_t n, int64_t ld, int kchunk,
                                                       const float* __restrict__ M,
                                                       const float* __restrict__ in,
                                                       float* __restrict__ out,
                                                       float* __restrict__ part) {
  static_assert(KC % 32 == 0, "chunks of 32 rows");
  constexpr int SB = 64 + 4;                 // LDS row stride (words)
  constexpr int KL = KC / 4;                 // loop indices per lane group and chunk
  constexpr int SV = KC / 16;                // 16-byte staging loads per thread
  __shared__ __attribute__((aligned(16))) float sB[2][KC * SB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * w;
  const int split = blockIdx.y;
  const int64_t k0 = (int64_t)split * kchunk;
  const int64_t k1 = k0 + kchunk < n ? k0 + kchunk : n;
  const int64_t jr = row0 + i;               // this lane's matrix row (A operand row)
  const float* __restrict__ mrow_p = M + (jr < n ? jr : 0) * ld;
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc[4] = {zero, zero, zero, zero};
  // staging: thread t moves input row kb + (t / 16) + 16 v, columns 4 (t % 16) .. +3
  const int sr = threadIdx.x >> 4, sc = 4 * (threadIdx.x & 15);
  f32x4 bst[SV], am[KL / 4];
  auto load_chunk = [&](int64_t kb) {
#pragma unroll
    for (int v = 0; v < SV; ++v) {
      const int64_t r = kb + sr + 16 * v;
      bst[v] = r < k1 ? *(const f32x4*)(in + r * 64 + sc) : zero;
    }
#pragma unroll
    for (int v = 0; v < KL / 4; ++v) {
      // 4 entries from column c; c < ld covers them all (ld % 4 == 0), and
      // columns >= n inside the row are the zero padding
      const int64_t c = kb + 16 * v + 4 * g;
      am[v] = (jr < n && c < k1) ? *(const f32x4*)(mrow_p + c) : zero;
    }
  };
  int buf = 0;
  if (k0 < k1) load_chunk(k0);
  for (int64_t kb = k0; kb < k1; kb += KC) {
#pragma unroll
    for (int v = 0; v < SV; ++v) *(f32x4*)(sB[buf] + (sr + 16 * v) * SB + sc) = bst[v];
    f32x4 a[KL / 4];
#pragma unroll
    for (int v = 0; v < KL / 4; ++v) a[v] = am[v];
    __syncthreads();
    if (kb + KC < k1) load_chunk(kb + KC);    // in flight during this chunk's MFMAs
#pragma unroll
    for (int st = 0; st < KL; ++st) {
      const f32x4 b = *(const f32x4*)(sB[buf] + (16 * (st / 4) + 4 * g + st % 4) * SB + 4 * i);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[st / 4][st % 4], b[q], acc[q], 0, 0, 0);
    }
    buf ^= 1;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t jj = row0 + 4 * g + v;
    if (jj >= n) continue;
    f32x4 o;
    o[0] = acc[0][v];
    o[1] = acc[1][v];
    o[2] = acc[2][v];
    o[3] = acc[3][v];
    float* dst = (gridDim.y > 1 ? part + (int64_t)split * n * 64 : out) + jj * 64 + 4 * i;
    *(f32x4*)dst = o;
  }
}

// The same dense level operator in FP64 on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: operands as in the FP32 16x16x4 form, lane i + 16 g
// holding A[i][g] and B[g][i]; result register v of lane i + 16 g holds
// D[g + 4 v][i], not D[4 g + v][i] as in the FP32 form): OUT = M IN, M n x n row-major with padded stride ld (a
// multiple of 4, padding zero), IN and OUT interleaved n x 64.  A workgroup
// takes a 64-row x 64-column output tile over the loop range of its split
// (blockIdx.y), 16 rows per wave; the loop runs in chunks of KC input rows
// staged once in LDS (double-buffered), and each lane reads its own matrix
// row in 32-byte pieces: piece v of lane group g holds loop indices
// kb + 16 v + 4 g + e (e < 4), so a row's four lane groups read 128
// contiguous bytes.  The next chunk's loads are in flight during the
// current chunk's MFMAs.  Splits > 1 write partial sums to part[split][row][:]
// for k_dense_reduce64d (an empty loop range writes zeros).
template <int KC>
__global__ void __launch_bounds__(kBlock) k_dense_mm64d(int64_t n, int64_t ld, int kchunk,
                                                        const double* __restrict__ M,
                                                        const double* __restrict__ in,
                                                        double* __restrict__ out,
                                                        double* __restrict__ part) {
  typedef double f64x4 __attribute__((ext_vector_type(4)));
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  static_assert(KC % 16 == 0, "chunks of 16 rows");
  constexpr int SB = 64 + 4;                 // LDS row stride (doubles)
  constexpr int KL = KC / 4;                 // loop indices per lane group and chunk
  constexpr int SV = KC / 8;                 // 16-byte staging loads per thread
  __shared__ __attribute__((aligned(16))) double sB[2][KC * SB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + 16 * w;
  const int split = blockIdx.y;
  const int64_t k0 = (int64_t)split * kchunk;
  const int64_t k1 = k0 + kchunk < n ? k0 + kchunk : n;
  const int64_t jr = row0 + i;               // this lane's matrix row (A operand row)
  const double* __restrict__ mrow_p = M + (jr < n ? jr : 0) * ld;
  const f64x4 zero4 = {0.0, 0.0, 0.0, 0.0};
  const f64x2 zero2 = {0.0, 0.0};
  f64x4 acc[4] = {zero4, zero4, zero4, zero4};
  // staging: thread t moves input row kb + (t / 32) + 8 v, columns 2 (t % 32) .. +1
  const int sr = threadIdx.x >> 5, sc = 2 * (threadIdx.x & 31);
  f64x2 bst[SV];
  f64x4 am[KL / 4];
  auto load_chunk = [&](int64_t kb) {
#pragma unroll
    for (int v = 0; v < SV; ++v) {
      const int64_t r = kb + sr + 8 * v;
      bst[v] = r < k1 ? *(const f64x2*)(in + r * 64 + sc) : zero2;
    }
#pragma unroll
    for (int v = 0; v < KL / 4; ++v) {
      // 4 entries from column c; c < ld covers them all (ld % 4 == 0, and a
      // split's range is a multiple of 4 long), columns >= n are padding
      const int64_t c = kb + 16 * v + 4 * g;
      am[v] = (jr < n && c < k1) ? *(const f64x4*)(mrow_p + c) : zero4;
    }
  };
  int buf = 0;
  if (k0 < k1) load_chunk(k0);
  for (int64_t kb = k0; kb < k1; kb += KC) {
#pragma unroll
    for (int v = 0; v < SV; ++v) *(f64x2*)(sB[buf] + (sr + 8 * v) * SB + sc) = bst[v];
    f64x4 a[KL / 4];
#pragma unroll
    for (int v = 0; v < KL / 4; ++v) a[v] = am[v];
    __syncthreads();
    if (kb + KC < k1) load_chunk(kb + KC);    // in flight during this chunk's MFMAs
#pragma unroll
    for (int st = 0; st < KL; ++st) {
      const f64x4 b = *(const f64x4*)(sB[buf] + (16 * (st / 4) + 4 * g + st % 4) * SB + 4 * i);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st / 4][st % 4], b[q], acc[q], 0, 0, 0);
    }
    buf ^= 1;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t jj = row0 + g + 4 * v;
    if (jj >= n) continue;
    f64x4 o;
    o[0] = acc[0][v];
    o[1] = acc[1][v];
    o[2] = acc[2][v];
    o[3] = acc[3][v];
    double* dst = (gridDim.y > 1 ? part + (int64_t)split * n * 64 : out) + jj * 64 + 4 * i;
    *(f64x4*)dst = o;
  }
}

// out[r][:] = sum over the S slots of part[s][r][:] (64 columns, FP64), in
// slot order
__global__ void __launch_bounds__(kBlock) k_dense_reduce64d(int64_t rows, int S,
                                                            const double* __restrict__ part,
                                                            double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= rows * 64) return;
  double s = 0.0;
  for (int k = 0; k < S; ++k) s += part[(int64_t)k * rows * 64 + e];
  out[e] = s;
}

// dst[j][l] = src[l][j] (j, l < n) with row stride ld >= n, padding zero: the
// row-major copy for k_dense_mm64 / k_dense_mm64d of an operator stored as
// the dense GEMV's M (output j = sum over l of M[l][j] times input l).
// Set-up only.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pad_rows(int64_t n, int64_t ld,
                                                     const T* __restrict__ src,
                                                     T* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * ld) return;
  const int64_t j = e / ld, l = e - j * ld;
  dst[e] = l < n ? src[l * n + j] : T(0);
}

// out[r][:] (=|+=) sum over the S slots of part[s][r][:], in slot order
template <bool ADD, int NB>
__global__ void __launch_bounds__(kBlock) k_bmm_reduce(int64_t rows, int S,
                                                       const float* __restrict__ part,
                                                       float* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= rows * NB) return;
  float s = 0.f;
  for (int k = 0; k < S; ++k) s += part[(int64_t)k * rows * NB + e];
  out[e] = ADD ? out[e] + s : s;
}

// X[j][:] += staged RAS-T contributions (batched k_gather_add)
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bgather_add(int64_t n, const int64_t* __restrict__ cptr,
                                                        const int64_t* __restrict__ cpos,
                                                        const T* __restrict__ tb,
                                                        T* __restrict__ X) {
  const int64_t gid = xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  const int64_t d = wave_row<NB>(gid / NB);
  const int c = (int)(gid % NB);
  if (d >= n) return;
  T s = X[d * NB + c];
  if constexpr (NB == 64)
    s += staged_sum64<T>(cptr[d], cptr[d + 1], cpos, tb, c);
  else
    for (int64_t e = cptr[d]; e < cptr[d + 1]; ++e) s += tb[cpos[e] * NB + c];
  X[d * NB + c] = s;
}

// ---------------------------------------------------------------------------
// Batched FP64 CG.  Column j has its own scalars.  A kernel that produces a
// dot product stores one partial per workgroup and column, column-major
// (part[j * gridDim.x + blockIdx.x], so that a column's partials are
// contiguous); k_bsum adds them in a fixed order into one scalar per column,
// which the consuming kernels read.  active[j] = 0
// freezes a converged column.
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
    part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
  __syncthreads();
}

// out[j] = sum over the np workgroup partials of column j (one workgroup per
// column, coalesced reads; strided partial sums, then a fixed-order tree)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bsum(int np, const double* __restrict__ part,
                                                 double* __restrict__ out) {
  __shared__ double sm[kBlock];
  const int j = blockIdx.x;
  const double* __restrict__ p = part + (int64_t)j * np;
  // eight independent partial sums per thread, so eight loads are in flight
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int b = threadIdx.x;
  for (; b + 7 * kBlock < np; b += 8 * kBlock) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += p[b + u * kBlock];
  }
  for (; b < np; b += kBlock) a[0] += p[b];
  const double s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = sm[0];
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
  for (int64_t d = wave_row<NB>((xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / NB); d < n;
       d += (int64_t)gridDim.x * (kBlock / NB)) {
    double s;
    if constexpr (NB == 64) {
      s = row_dot64<double>(ptr[d], ptr[d + 1], col, val, Y, j);
    } else {
      s = 0;
      for (int64_t e = ptr[d]; e < ptr[d + 1]; ++e) s += val[e] * Y[(int64_t)col[e] * NB + j];
    }
    Q[d * NB + j] = s;
    v += s * P[d * NB + j];
  }
  bwrite_parts<NB>(v, part);
}

// Q = G^T (G P) in one pass (rows of G recomputed, ata_row) and partials of
// P . Q per column
template <int NB, int ME, int MF>
__global__ void __launch_bounds__(kBlock) k_bcg_apq1(int64_t n, const int64_t* __restrict__ gt_ptr,
                                                     const int32_t* __restrict__ gt_col,
                                                     const double* __restrict__ gt_val,
                                                     const int64_t* __restrict__ g_ptr,
                                                     const int32_t* __restrict__ g_col,
                                                     const double* __restrict__ g_val,
                                                     const double* __restrict__ P,
                                                     double* __restrict__ Q,
                                                     double* __restrict__ part) {
  const int j = threadIdx.x % NB;
  double v = 0;
  for (int64_t d = wave_row<NB>((xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / NB); d < n;
       d += (int64_t)gridDim.x * (kBlock / NB)) {
    double acc;
    if constexpr (NB == 64)
      acc = ata_row64<double, ME, MF>(d, gt_ptr, gt_col, gt_val, g_ptr, g_col, g_val, P, j);
    else
      acc = ata_row<double, NB, ME, MF>(d, gt_ptr, gt_col, gt_val, g_ptr, g_col, g_val, P, j);
    Q[d * NB + j] = acc;
    v += acc * P[d * NB + j];
  }
  bwrite_parts<NB>(v, part);
}

// ---------------------------------------------------------------------------
// Tiled one-pass G^T (G X) on 64 columns (finest level, short rows of G).
// The unknowns are cut into tiles of TS consecutive unknowns.  For tile t the
// host lists U_t, the unknowns that the rows of G touching the tile reach
// (ascending), and R_t, those rows (ascending); the entries of each row of R_t
// carry the position in U_t of their column (rli) and their value, padded to
// MF entries with value 0, and each unknown of the tile carries the position
// in R_t of its rows of G (drl) in the order of G^T's row and their values
// (dw), padded to ME with value 0.  A workgroup stages the rows of X listed in
// U_t in LDS, forms y_r = sum_q G[r][c_q] X[c_q] for the rows of R_t into
// LDS (entries in row order), and then sum_k G[r_k][d] y_{r_k} for each
// unknown d (rows in G^T order): the arithmetic of ata_row64, with every X
// row read once per tile instead of once per entry that reaches it.  Each
// wavefront loads the metadata of up to 64 entries with one vector load and
// walks them by lane broadcast; the loads that need no tile list (the
// unknowns' entries, B) are issued first.  The host keeps the rows of a tile
// per wavefront within one metadata load (ceil(|R_t| / 4) * MF <= 64).
//   EPI 0: R = B - G^T G X   (V-cycle residual)
//   EPI 1: R = G^T G X, and partials of B . R per column (B = the CG's P)
// LDS: (umax + rmax) * 64 * sizeof(T) bytes (dynamic).
// ---------------------------------------------------------------------------
struct AtaTiles {
  const int32_t* uptr;    // [ntile + 1] offsets into ucol
  const int32_t* ucol;    // U_t lists
  const int32_t* rptr;    // [ntile + 1] offsets of R_t (rows of the tile order)
  const uint16_t* rli;    // [rows * MF] position in U_t of each row entry's column
  const uint16_t* drl;    // [n * ME] position in R_t of each unknown's rows
  const uint16_t* eli;    // [n * ME * MF] expanded form: position in U_t of entry q of
                          // row k of each unknown (values in ev, row weights in dw)
  int64_t ntile;
  int umax;               // largest |U_t| (LDS stride of the second buffer)
};

template <typename T, int TS, int ME, int MF, int EPI>
__global__ void __launch_bounds__(kBlock) k_bata_tile(int64_t n, AtaTiles tl,
                                                      const T* __restrict__ rv,
                                                      const T* __restrict__ dw,
                                                      const T* __restrict__ X,
                                                      const T* __restrict__ B,
                                                      T* __restrict__ R,
                                                      double* __restrict__ part) {
  constexpr int WPB = kBlock / 64;
  constexpr int DPW = TS / WPB;                    // unknowns per wavefront
  static_assert(TS % WPB == 0 && DPW * ME <= 64 && ME * MF <= 64, "one entry per lane");
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* sX = (T*)lds_raw;
  T* sY = sX + (int64_t)tl.umax * 64;
  constexpr int VPR = 64 * (int)sizeof(T) / 16;   // 16-byte pieces per row of X
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double v = 0;
  for (int64_t t = xcd_block(blockIdx.x, gridDim.x); t < tl.ntile; t += gridDim.x) {
    // loads that need no tile list first: this wavefront's unknowns (their
    // G^T entries, and B)
    const int64_t d0 = t * TS;
    const int nd = (int)(n - d0 < TS ? n - d0 : TS);
    const int db = w * DPW, nwd = nd - db < DPW ? (nd - db > 0 ? nd - db : 0) : DPW;
    int lid = 0;
    T ww = 0;
    T bv[DPW];
    if (nwd > 0) {
      const int cnt = nwd * ME;
      const int64_t e = (d0 + db) * ME + (lane < cnt ? lane : cnt - 1);
      lid = tl.drl[e];
      ww = dw[e];
#pragma unroll
      for (int u = 0; u < DPW; ++u) bv[u] = u < nwd ? B[(d0 + db + u) * 64 + lane] : T(0);
    }
    // the tile's lists, this wavefront's rows of R_t, and the staging of X
    const int u0 = tl.uptr[t], nu = tl.uptr[t + 1] - u0;
    const int r0 = tl.rptr[t], nr = tl.rptr[t + 1] - r0;
    const int per = (nr + WPB - 1) / WPB;            // <= 64 / MF (checked by the host)
    const int rb = w * per, nwr = nr - rb < per ? (nr - rb > 0 ? nr - rb : 0) : per;
    int lir = 0;
    T vv = 0;
    if (nwr > 0) {
      const int cnt = nwr * MF;
      const int64_t e = (int64_t)(r0 + rb) * MF + (lane < cnt ? lane : cnt - 1);
      lir = tl.rli[e];
      vv = rv[e];
    }
    for (int e = threadIdx.x; e < nu * VPR; e += kBlock) {
      const int row = e / VPR, pc = e - row * VPR;
      const int64_t c = tl.ucol[u0 + row];
      *(f32x4*)((char*)(sX + (int64_t)row * 64) + 16 * pc) =
          *(const f32x4*)((const char*)(X + c * 64) + 16 * pc);
    }
    __syncthreads();
    for (int r = 0; r < nwr; ++r) {
      T y = 0;
#pragma unroll
      for (int q = 0; q < MF; ++q)
        y += lane_val(vv, r * MF + q) * sX[(int64_t)lane_val(lir, r * MF + q) * 64 + lane];
      sY[(int64_t)(rb + r) * 64 + lane] = y;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < DPW; ++u) {
      if (u >= nwd) break;
      T acc = 0;
#pragma unroll
      for (int k = 0; k < ME; ++k)
        acc += lane_val(ww, u * ME + k) * sY[(int64_t)lane_val(lid, u * ME + k) * 64 + lane];
      const int64_t o = (d0 + db + u) * 64 + lane;
      if constexpr (EPI == 0) {
        R[o] = bv[u] - acc;
      } else {
        R[o] = acc;
        v += (double)acc * (double)bv[u];
      }
    }
    __syncthreads();                  // LDS is refilled by the next tile
  }
  if constexpr (EPI == 1) bwrite_parts<64>(v, part);
}

// The same one-pass G^T (G X) on 64 columns without the row phase: each
// unknown carries its whole expanded stencil (for each of its rows k of G in
// G^T order, the row's entries q in row order as (position in U_t, value)),
// so a wavefront forms sum_k G[r_k][d] (sum_q G[r_k][c_q] X[c_q]) straight
// from the staged X rows, in the order and arithmetic of ata_row64.  One LDS
// buffer (umax * 64 * sizeof(T)) and one barrier per tile.  EPI as
// k_bata_tile.
template <typename T, int TS, int ME, int MF, int EPI>
__global__ void __launch_bounds__(kBlock) k_bata_tilex(int64_t n, AtaTiles tl,
                                                       const T* __restrict__ ev,
                                                       const T* __restrict__ dw,
                                                       const T* __restrict__ X,
                                                       const T* __restrict__ B,
                                                       T* __restrict__ R,
                                                       double* __restrict__ part) {
  constexpr int WPB = kBlock / 64;
  constexpr int DPW = TS / WPB;                    // unknowns per wavefront
  constexpr int EN = ME * MF;                      // stencil entries per unknown
  static_assert(TS % WPB == 0 && EN <= 64, "one entry per lane");
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* sX = (T*)lds_raw;
  constexpr int VPR = 64 * (int)sizeof(T) / 16;   // 16-byte pieces per row of X
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double v = 0;
  for (int64_t t = xcd_block(blockIdx.x, gridDim.x); t < tl.ntile; t += gridDim.x) {
    const int64_t d0 = t * TS;
    const int nd = (int)(n - d0 < TS ? n - d0 : TS);
    const int db = w * DPW, nwd = nd - db < DPW ? (nd - db > 0 ? nd - db : 0) : DPW;
    // this wavefront's unknowns first: stencils, row weights, B
    int li[DPW];
    T vv[DPW], ww[DPW], bv[DPW];
#pragma unroll
    for (int u = 0; u < DPW; ++u) {
      li[u] = 0;
      vv[u] = ww[u] = bv[u] = T(0);
      if (u < nwd) {
        const int64_t d = d0 + db + u;
        li[u] = tl.eli[d * EN + (lane < EN ? lane : 0)];
        vv[u] = lane < EN ? ev[d * EN + lane] : T(0);
        ww[u] = lane < ME ? dw[d * ME + lane] : T(0);
        bv[u] = B[d * 64 + lane];
      }
    }
    const int u0 = tl.uptr[t], nu = tl.uptr[t + 1] - u0;
    for (int e = threadIdx.x; e < nu * VPR; e += kBlock) {
      const int row = e / VPR, pc = e - row * VPR;
      const int64_t c = tl.ucol[u0 + row];
      *(f32x4*)((char*)(sX + (int64_t)row * 64) + 16 * pc) =
          *(const f32x4*)((const char*)(X + c * 64) + 16 * pc);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < DPW; ++u) {
      if (u >= nwd) break;
      T acc = 0;
#pragma unroll
      for (int k = 0; k < ME; ++k) {
        T y = 0;
#pragma unroll
        for (int q = 0; q < MF; ++q)
          y += lane_val(vv[u], k * MF + q) * sX[(int64_t)lane_val(li[u], k * MF + q) * 64 + lane];
        acc += lane_val(ww[u], k) * y;
      }
      const int64_t o = (d0 + db + u) * 64 + lane;
      if constexpr (EPI == 0) {
        R[o] = bv[u] - acc;
      } else {
        R[o] = acc;
        v += (double)acc * (double)bv[u];
      }
    }
    __syncthreads();                  // LDS is refilled by the next tile
  }
  if constexpr (EPI == 1) bwrite_parts<64>(v, part);
}

// Single right-hand side, one pass: the CG's new direction and its A-apply.
// Over tiles of TS consecutive unknowns (tiles and entry order as for
// k_bata_tile): Pn = Z + beta Po (beta = rz_new / rz_old from the partials
// of the preceding kernels, gridDim.x of them; Pn = Z when rz_old is null) is
// formed for the tile's U_t into LDS, y_r for its rows R_t into LDS, and
// Q[d] = sum_k G[r_k][d] y_{r_k} for its own unknowns, which also store Pn[d];
// partials of Pn . Q per workgroup.  Pn must not alias Po (other tiles still
// read Po for their halos).  One unknown per thread (TS = kBlock).
// LDS: (umax + rmax) doubles (dynamic).
template <int ME, int MF>
__global__ void __launch_bounds__(kBlock) k_cg_tile(int64_t n, AtaTiles tl,
                                                    const double* __restrict__ rv,
                                                    const double* __restrict__ dw,
                                                    const double* __restrict__ rz_new,
                                                    const double* __restrict__ rz_old,
                                                    const double* __restrict__ Z,
                                                    const double* __restrict__ Po,
                                                    double* __restrict__ Pn,
                                                    double* __restrict__ Q,
                                                    double* __restrict__ part) {
  constexpr int TS = kBlock;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  double* sX = (double*)lds_raw;
  double* sY = sX + tl.umax;
  const int np = gridDim.x;
  const bool first = rz_old == nullptr;
  const double beta = first ? 0.0 : sum_parts(rz_new, np) / sum_parts(rz_old, np);
  double v = 0;
  for (int64_t t = xcd_block(blockIdx.x, gridDim.x); t < tl.ntile; t += gridDim.x) {
    const int64_t d = t * TS + threadIdx.x;
    // this thread's unknown: its entries and its new direction first
    int li[ME];
    double w[ME];
    double pd = 0;
    if (d < n) {
#pragma unroll
      for (int k = 0; k < ME; ++k) {
        li[k] = tl.drl[d * ME + k];
        w[k] = dw[d * ME + k];
      }
      pd = first ? Z[d] : Z[d] + beta * Po[d];
    }
    const int u0 = tl.uptr[t], nu = tl.uptr[t + 1] - u0;
    const int r0 = tl.rptr[t], nr = tl.rptr[t + 1] - r0;
    for (int e = threadIdx.x; e < nu; e += kBlock) {
      const int64_t c = tl.ucol[u0 + e];
      sX[e] = first ? Z[c] : Z[c] + beta * Po[c];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nr; r += kBlock) {
      const int64_t e0 = (int64_t)(r0 + r) * MF;
      double y = 0;
#pragma unroll
      for (int q = 0; q < MF; ++q) y += rv[e0 + q] * sX[tl.rli[e0 + q]];
      sY[r] = y;
    }
    __syncthreads();
    if (d < n) {
      double acc = 0;
#pragma unroll
      for (int k = 0; k < ME; ++k) acc += w[k] * sY[li[k]];
      Q[d] = acc;
      Pn[d] = pd;
      v += pd * acc;
    }
    __syncthreads();                  // LDS is refilled by the next tile
  }
  write_part(v, part);
}

// Row-group pass of a coarse level on 64 columns (see k_grp_ata), FP32 on
// the matrix cores: for a task (rows t0 .. t0+nr-1 of group g, nr <= 32;
// support columns t0 .. c-1, w <= wmax of them)
//   Y = R X_S     (nr x 64: y_i = sum_{q >= i} R_g[t0+i][t0+q] X[supp_g[t0+q]])
//   STG[soff + q] = (R^T Y)[q]   (w x 64)
// with R the task's upper-trapezoidal block (local column q of row i at
// val[vstart + i*w - i*(i-1)/2 - i + q], zero for q < i).  One workgroup per
// task; wavefront v owns output columns 16v .. 16v+15 of both products.  X_S
// and the block (dense 32 x w, zero outside the trapezoid, odd row stride so
// that the 16 rows one A operand reads fall in distinct banks) are staged in
// LDS with coalesced loads; Y goes through LDS (32 rows, zero beyond nr)
// between the two products.  v_mfma_f32_16x16x4f32 operand layout as in
// k_bmm: lane i + 16g feeds A[i][g] and B[g][i] and holds D[4g+v][i].
// LDS: ((wmax + 32) * 64 + 32 * (wmax + 1)) * 4 bytes (dynamic).
__global__ void __launch_bounds__(kBlock) k_bgrp_ata64(GrpTasks tk, int wmax,
                                                       const float* __restrict__ val,
                                                       const int32_t* __restrict__ supp,
                                                       const float* __restrict__ X,
                                                       float* __restrict__ stg) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  float* sX = (float*)lds_raw;
  float* sY = sX + (int64_t)wmax * 64;
  float* sR = sY + 32 * 64;
  constexpr int VPR = 16;                   // 16-byte pieces per row of X
  const int64_t task = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, g = lane >> 4;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int col = 16 * wv + i16;
  const int nr = tk.nrow[task], t0 = tk.t0[task], c = tk.c[task];
  const int w = c - t0;
  const int64_t v0 = tk.vstart[task];
  const int32_t* sp = supp + tk.s0[task] + t0;
  const int W1 = w | 1;                     // odd LDS row stride of the block
  for (int e = threadIdx.x; e < 32 * w; e += kBlock) {
    const int i = e / w, q = e - i * w;
    sR[i * W1 + q] = (i < nr && q >= i)
                         ? val[v0 + (int64_t)i * w - (int64_t)i * (i - 1) / 2 - i + q]
                         : 0.f;
  }
  // entry (i, q) of the task's block (i < 32), zero outside the trapezoid
  auto rval = [&](int i, int q) -> float { return q < w ? sR[i * W1 + q] : 0.f; };
  for (int e = threadIdx.x; e < w * VPR; e += kBlock) {
    const int row = e / VPR, pc = e - row * VPR;
    const int64_t cx = sp[row];
    *(f32x4*)((char*)(sX + (int64_t)row * 64) + 16 * pc) =
        *(const f32x4*)((const char*)(X + cx * 64) + 16 * pc);
  }
  __syncthreads();
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  {
    f32x4 acc[2] = {zero, zero};
#pragma unroll 4
    for (int k = 0; k < w; k += 4) {
      const int q = k + g;
      const float bx = q < w ? sX[q * 64 + col] : 0.f;
      acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(rval(i16, q), bx, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(rval(16 + i16, q), bx, acc[1], 0, 0, 0);
    }
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int v = 0; v < 4; ++v) sY[(16 * rt + 4 * g + v) * 64 + col] = acc[rt][v];
  }
  __syncthreads();
  float* dst = stg + tk.soff[task] * 64;
  for (int qt = 0; qt < w; qt += 16) {
    f32x4 acc = zero;
#pragma unroll
    for (int k = 0; k < 32; k += 4) {
      if (k >= nr) break;
      const int i = k + g;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(rval(i, qt + i16), sY[i * 64 + col], acc, 0, 0,
                                                 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = qt + 4 * g + v;
      if (q < w) dst[(int64_t)q * 64 + col] = acc[v];
    }
  }
}

// R = B - (sum of the staged rows of each unknown, in position order), 64
// columns, a wavefront per unknown.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bresid_stg64(int64_t n, const int64_t* __restrict__ cptr,
                                                         const int64_t* __restrict__ cpos,
                                                         const T* __restrict__ stg,
                                                         const T* __restrict__ B,
                                                         T* __restrict__ R) {
  const int lane = threadIdx.x & 63;
  const int64_t d = wave_row<64>((xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) / 64);
  if (d >= n) return;
  const T t = staged_sum64<T>(cptr[d], cptr[d + 1], cpos, stg, lane);
  R[d * 64 + lane] = B[d * 64 + lane] - t;
}

// alpha_j = rho_j / pq_j (0 for inactive columns); X += alpha P; R -= alpha Q;
// R32 = (float) R (if given); partials of R . R
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_update(int64_t n, const double* __restrict__ rz,
                                                       const double* __restrict__ pqs,
                                                       const int* __restrict__ active,
                                                       const double* __restrict__ P,
                                                       const double* __restrict__ Q,
                                                       double* __restrict__ X,
                                                       double* __restrict__ R,
                                                       float* __restrict__ R32,
                                                       double* __restrict__ rr_part) {
  const int j = threadIdx.x % NB;
  bool act = active[j] != 0;
  const double pq = act ? pqs[j] : 0.0;
  act = act && pq != 0.0;
  const double alpha = act ? rz[j] / pq : 0.0;
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

// Z = XV + staged RAS-T contributions (V-cycle precision T); partials of
// R . Z, and with Q given the partials of -(Z . Q) (flexible CG, Q = A P_old)
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_z(int64_t n, const T* __restrict__ XV,
                                                  const int64_t* __restrict__ cptr,
                                                  const int64_t* __restrict__ cpos,
                                                  const T* __restrict__ tb,
                                                  const double* __restrict__ R,
                                                  double* __restrict__ Z,
                                                  double* __restrict__ rz_part,
                                                  const double* __restrict__ Q,
                                                  double* __restrict__ zq_part) {
  const int c = threadIdx.x % NB;
  double v = 0, w = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock) {
    const int64_t d = wave_row<NB>(e / NB);
    T s = XV[e];
    if (cptr) {
      if constexpr (NB == 64)
        s += staged_sum64<T>(cptr[d], cptr[d + 1], cpos, tb, c);
      else
        for (int64_t q = cptr[d]; q < cptr[d + 1]; ++q) s += tb[cpos[q] * NB + c];
    }
    const double zi = (double)s;
    Z[e] = zi;
    v += R[e] * zi;
    if (Q) w += zi * Q[e];
  }
  bwrite_parts<NB>(v, rz_part);
  if (Q) bwrite_parts<NB>(-w, zq_part);
}

// k_bcg_z on 64 columns with four columns per thread: a group of 16 lanes
// takes one unknown (16-byte loads of XV and of each staged row, two of R
// and Z in FP64), so a wavefront carries four unknowns through each memory
// round trip.  Z = (double)(XV + staged sum), the staged rows added in
// position order as in k_bcg_z; partials of R . Z per column and workgroup
// (column-major, as bwrite_parts) summed over the 16 unknown slots in a
// fixed order.  With Q given, also the partials of -(Z . Q) (flexible CG).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_bcg_z64(int64_t n, const T* __restrict__ XV,
                                                    const int64_t* __restrict__ cptr,
                                                    const int64_t* __restrict__ cpos,
                                                    const T* __restrict__ tb,
                                                    const double* __restrict__ R,
                                                    double* __restrict__ Z,
                                                    double* __restrict__ rz_part,
                                                    const double* __restrict__ Q,
                                                    double* __restrict__ zq_part) {
  constexpr int SL = kBlock / 16;          // unknown slots per workgroup
  __shared__ double sm[SL][64];
  const int slot = threadIdx.x >> 4, c4 = 4 * (threadIdx.x & 15);
  double v[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t d = (int64_t)xcd_block(blockIdx.x, gridDim.x) * SL + slot; d < n;
       d += (int64_t)gridDim.x * SL) {
    const int64_t o = d * 64 + c4;
    T s[4];
    load4<T>(XV + o, s);
    if (cptr) {
      const int64_t e1 = cptr[d + 1];
      for (int64_t e = cptr[d]; e < e1; ++e) {
        T t[4];
        load4<T>(tb + cpos[e] * 64 + c4, t);
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += t[k];
      }
    }
    double r[4];
    load4<double>(R + o, r);
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 z01 = {(double)s[0], (double)s[1]}, z23 = {(double)s[2], (double)s[3]};
    *(d2*)(Z + o) = z01;
    *(d2*)(Z + o + 2) = z23;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += r[k] * (double)s[k];
    if (Q) {
      double qv[4];
      load4<double>(Q + o, qv);
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] += (double)s[k] * qv[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) sm[slot][c4 + k] = v[k];
  __syncthreads();
  if (threadIdx.x < 64) {
    double t = 0;
    for (int q = 0; q < SL; ++q) t += sm[q][threadIdx.x];
    rz_part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
  if (!Q) return;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) sm[slot][c4 + k] = w[k];
  __syncthreads();
  if (threadIdx.x < 64) {
    double t = 0;
    for (int q = 0; q < SL; ++q) t += sm[q][threadIdx.x];
    zq_part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = -t;
  }
}

template <typename T>
__device__ __forceinline__ void store4(T* __restrict__ p, const T (&m)[4]);
template <>
__device__ __forceinline__ void store4<float>(float* __restrict__ p, const float (&m)[4]) {
  const f32x4 t = {m[0], m[1], m[2], m[3]};
  *(f32x4*)p = t;
}
template <>
__device__ __forceinline__ void store4<double>(double* __restrict__ p, const double (&m)[4]) {
  typedef double v2 __attribute__((ext_vector_type(2)));
  const v2 t0 = {m[0], m[1]}, t1 = {m[2], m[3]};
  *(v2*)p = t0;
  *(v2*)(p + 2) = t1;
}

// CSR rows on 64 columns with four columns per thread: a group of 16 lanes
// takes one row, so a wavefront works on four rows at once.  The group loads
// 16 entries (index, value) with one load per lane and walks them by lane
// shuffle, four 16-byte row gathers in flight per lane; entries are added in
// row order.  RES: Y = B - A X; else Y = A X.
template <typename T, bool RES>
__global__ void __launch_bounds__(kBlock) k_bspmv4(int64_t nrows, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col,
                                                   const T* __restrict__ val,
                                                   const T* __restrict__ X,
                                                   const T* __restrict__ B, T* __restrict__ Y) {
  const int64_t row = (xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x) >> 4;
  const int j = threadIdx.x & 15, c4 = 4 * j;
  if (row >= nrows) return;            // whole 16-lane groups exit together
  const int64_t e0 = ptr[row], e1 = ptr[row + 1];
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int64_t b = e0; b < e1; b += 16) {
    const int cnt = (int)(e1 - b < 16 ? e1 - b : 16);
    const int64_t e = b + (j < cnt ? j : cnt - 1);
    const int cj = col[e];
    const T vj = val[e];
    int k = 0;
    for (; k + 4 <= cnt; k += 4) {
      T y[4][4];
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = __shfl(cj, k + u, 16);
        v[u] = __shfl(vj, k + u, 16);
        load4<T>(X + (int64_t)c * 64 + c4, y[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += v[u] * y[u][q];
    }
    for (; k < cnt; ++k) {
      const int c = __shfl(cj, k, 16);
      const T v = __shfl(vj, k, 16);
      T y[4];
      load4<T>(X + (int64_t)c * 64 + c4, y);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += v * y[q];
    }
  }
  T out[4];
  if (RES) {
    T bb[4];
    load4<T>(B + row * 64 + c4, bb);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = bb[q] - acc[q];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = acc[q];
  }
  store4<T>(Y + row * 64 + c4, out);
}

// P = Z + beta P, beta_j = rz_new_j / rz_old_j (rz_old == nullptr: P = Z);
// rz_new, rz_old: per-column scalars
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_dir(int64_t n, const double* __restrict__ rz_new,
                                                    const double* __restrict__ rz_old,
                                                    const double* __restrict__ Z,
                                                    double* __restrict__ P) {
  const int j = threadIdx.x % NB;
  double beta = 0.0;
  if (rz_old) {
    const double o = rz_old[j];
    beta = o != 0.0 ? rz_new[j] / o : 0.0;   // an all-zero column stays zero
  }
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock)
    P[e] = rz_old ? Z[e] + beta * P[e] : Z[e];   // first direction: P = Z (P may hold stale data)
}

// partials of ||B - Q||^2 per column (true residual with Q = A X)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bres_parts(int64_t n, const double* __restrict__ B,
                                                       const double* __restrict__ Q,
                                                       double* __restrict__ part) {
  double v = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock) {
    const double d = B[e] - Q[e];
    v += d * d;
  }
  bwrite_parts<NB>(v, part);
}

// CG restart of the masked columns: R = B - Q (Q = A X), R32 = (float) R
// (if given), and rho_old = 0 so that the next direction of such a column is
// P = Z (beta = 0)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_restart(int64_t n, const int* __restrict__ mask,
                                                        const double* __restrict__ B,
                                                        const double* __restrict__ Q,
                                                        double* __restrict__ R,
                                                        float* __restrict__ R32,
                                                        double* __restrict__ rz_old) {
  const int j = threadIdx.x % NB;
  if (!mask[j]) return;
  if (blockIdx.x == 0 && threadIdx.x < NB) rz_old[j] = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock) {
    const double r = B[e] - Q[e];
    R[e] = r;
    if (R32) R32[e] = (float)r;
  }
}

// P = Z on the masked columns only (restart after the next direction of the
// other columns was already formed)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bcg_dir_mask(int64_t n, const int* __restrict__ mask,
                                                         const double* __restrict__ Z,
                                                         double* __restrict__ P) {
  const int j = threadIdx.x % NB;
  if (!mask[j]) return;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n * NB;
       e += (int64_t)gridDim.x * kBlock)
    P[e] = Z[e];
}

// Load ncols user columns (column-major, leading dimension ld) into
// columns j0 .. j0+ncols-1 of the interleaved blocks: B = R = b (internal
// numbering), X = P = 0, R32 = (float) b (if given); other columns untouched
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bload(int64_t n, int j0, int ncols, int64_t ld,
                                                  const int64_t* __restrict__ perm,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ B, double* __restrict__ R,
                                                  double* __restrict__ X, double* __restrict__ P,
                                                  float* __restrict__ R32) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t i = e / ncols;
  const int jj = (int)(e % ncols);
  const double v = b[(int64_t)jj * ld + perm[i]];
  const int64_t o = i * NB + j0 + jj;
  B[o] = v;
  R[o] = v;
  X[o] = 0.0;
  P[o] = 0.0;
  if (R32) R32[o] = (float)v;
}

// Store columns j0 .. j0+ncols-1 of the interleaved X into user columns
// (column-major, leading dimension ld, user numbering)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bstore(int64_t n, int j0, int ncols, int64_t ld,
                                                   const int64_t* __restrict__ perm,
                                                   const double* __restrict__ X,
                                                   double* __restrict__ x) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t i = e / ncols;
  const int jj = (int)(e % ncols);
  x[(int64_t)jj * ld + perm[i]] = X[i * NB + j0 + jj];
}

// rz[j] = 0 on the masked columns (their next direction is P = Z)
template <int NB>
__global__ void __launch_bounds__(kBlock) k_bzero_masked(const int* __restrict__ mask,
                                                         double* __restrict__ rz) {
  const int j = threadIdx.x;
  if (j < NB && mask[j]) rz[j] = 0.0;
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

// ---------------------------------------------------------------------------
// Block CG on 64 interleaved columns (row i of a block: 64 contiguous FP64
// values).  The workgroups take contiguous ranges of rows, staged through
// LDS kBgRows at a time with coalesced loads; a thread owns a 4 x 4 block of
// the 64 x 64 result (rows 4 (t / 16) .., columns 4 (t % 16) ..).
// ---------------------------------------------------------------------------
constexpr int kBgRows = 16;

// part[blk][a * 64 + b] = sum over the workgroup's rows i of A[i][a] B[i][b]
__global__ void __launch_bounds__(kBlock) k_bgram64(int64_t n, const double* __restrict__ A,
                                                    const double* __restrict__ B,
                                                    double* __restrict__ part) {
  __shared__ double sA[kBgRows][64], sB[kBgRows][64];
  const int t = threadIdx.x, a0 = 4 * (t >> 4), b0 = 4 * (t & 15);
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  double acc[4][4] = {};
  for (int64_t rb = r0; rb < r1; rb += kBgRows) {
    const int nr = (int)(r1 - rb < kBgRows ? r1 - rb : kBgRows);
    for (int e = t; e < kBgRows * 64; e += kBlock) {
      const int r = e >> 6, c = e & 63;
      sA[r][c] = r < nr ? A[(rb + r) * 64 + c] : 0.0;
      sB[r][c] = r < nr ? B[(rb + r) * 64 + c] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < nr; ++r) {
      double av[4], bv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        av[k] = sA[r][a0 + k];
        bv[k] = sB[r][b0 + k];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
  double* o = part + (int64_t)blockIdx.x * 4096;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) o[(a0 + i) * 64 + b0 + j] = acc[i][j];
}

// out[e] = sum over the np workgroup partials of entry e (ascending order)
__global__ void __launch_bounds__(kBlock) k_bgram_sum(int np, const double* __restrict__ part,
                                                      double* __restrict__ out) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= 4096) return;
  double v = 0.0;
  for (int b = 0; b < np; ++b) v += part[(int64_t)b * 4096 + e];
  out[e] = v;
}

// X += P C and R -= Q C row by row (C: 64 x 64 row-major), R32 = (float) R
// if given, and the per-column partials of ||R||^2 (column-major over the
// workgroups, as bwrite_parts).  Thread t: row t / 16 of the staged rows,
// columns 4 (t % 16) ...
__global__ void __launch_bounds__(kBlock) k_bupd64(int64_t n, const double* __restrict__ P,
                                                   const double* __restrict__ Q,
                                                   const double* __restrict__ C,
                                                   double* __restrict__ X, double* __restrict__ R,
                                                   float* __restrict__ R32,
                                                   double* __restrict__ rr_part) {
  __shared__ double sC[64][64];
  __shared__ double sP[kBgRows][64], sQ[kBgRows][64];
  __shared__ double sRR[kBgRows][64];
  const int t = threadIdx.x, r = t >> 4, c0 = 4 * (t & 15);
  for (int e = t; e < 4096; e += kBlock) sC[e >> 6][e & 63] = C[e];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  double rr[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t rb = r0; rb < r1; rb += kBgRows) {
    const int nr = (int)(r1 - rb < kBgRows ? r1 - rb : kBgRows);
    for (int e = t; e < kBgRows * 64; e += kBlock) {
      const int rr_ = e >> 6, c = e & 63;
      sP[rr_][c] = rr_ < nr ? P[(rb + rr_) * 64 + c] : 0.0;
      sQ[rr_][c] = rr_ < nr ? Q[(rb + rr_) * 64 + c] : 0.0;
    }
    __syncthreads();
    if (r < nr) {
      double dx[4] = {0.0, 0.0, 0.0, 0.0}, dr[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < 64; ++k) {
        const double pk = sP[r][k], qk = sQ[r][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          dx[j] += pk * sC[k][c0 + j];
          dr[j] += qk * sC[k][c0 + j];
        }
      }
      const int64_t o = (rb + r) * 64 + c0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        X[o + j] += dx[j];
        const double rn = R[o + j] - dr[j];
        R[o + j] = rn;
        if (R32) R32[o + j] = (float)rn;
        rr[j] += rn * rn;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) sRR[r][c0 + j] = rr[j];
  __syncthreads();
  if (t < 64) {
    double v = 0.0;
    for (int q = 0; q < kBgRows; ++q) v += sRR[q][t];
    rr_part[(int64_t)t * gridDim.x + blockIdx.x] = v;
  }
}

// P = Z + P D row by row (D: 64 x 64 row-major); each workgroup stages the
// old rows of its range before writing them
__global__ void __launch_bounds__(kBlock) k_bdir64(int64_t n, const double* __restrict__ Z,
                                                   const double* __restrict__ D,
                                                   double* __restrict__ P) {
  __shared__ double sD[64][64];
  __shared__ double sP[kBgRows][64];
  const int t = threadIdx.x, r = t >> 4, c0 = 4 * (t & 15);
  for (int e = t; e < 4096; e += kBlock) sD[e >> 6][e & 63] = D[e];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  for (int64_t rb = r0; rb < r1; rb += kBgRows) {
    const int nr = (int)(r1 - rb < kBgRows ? r1 - rb : kBgRows);
    for (int e = t; e < kBgRows * 64; e += kBlock) {
      const int rr_ = e >> 6, c = e & 63;
      sP[rr_][c] = rr_ < nr ? P[(rb + rr_) * 64 + c] : 0.0;
    }
    __syncthreads();
    if (r < nr) {
      double d[4] = {0.0, 0.0, 0.0, 0.0};
      for (int k = 0; k < 64; ++k) {
        const double pk = sP[r][k];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] += pk * sD[k][c0 + j];
      }
      const int64_t o = (rb + r) * 64 + c0;
#pragma unroll
      for (int j = 0; j < 4; ++j) P[o + j] = Z[o + j] + d[j];
    }
    __syncthreads();
  }
}

}  // namespace dev
}  // namespace lsamg
