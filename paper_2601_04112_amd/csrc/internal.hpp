// Internal host-side data of the LS-AMG-DD library (not part of the C-ABI).
#pragma once

#include <atomic>
#include <cstdint>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "../../include/lsamg.h"

namespace lsamg {

// Rows of G_l, grouped.  On the finest level every row of the user's G is a
// group of its own.  On coarser levels a group holds all rows of G_l = G_{l-1}
// P_{l-1} that touch the same set of parent aggregates; they share one
// symbolic support (every unknown of those parents), one multiplicity M and
// one set of overlapping aggregates, and are replaced by the R factor of
// their QR factorisation, which leaves every sum of w g^T g unchanged.
struct Groups {
  std::vector<int64_t> sptr;   // [ng+1] support pointer
  std::vector<int32_t> supp;   // support columns, ascending (internal numbering)
  std::vector<int32_t> nrows;  // [ng] rows stored for the group
  std::vector<int64_t> vptr;   // [ng+1] value offset: nrows x |supp| row-major
  std::vector<double> val;
  int64_t ng() const { return (int64_t)nrows.size(); }
  int64_t total_rows() const {
    int64_t s = 0;
    for (int32_t r : nrows) s += r;
    return s;
  }
};

struct Level {
  int64_t n = 0;
  int ndim = 0;
  int ext[3] = {1, 1, 1};          // lattice extent of this level
  std::vector<int32_t> coord;      // [n*ndim] lattice coordinate of each unknown
  std::vector<int64_t> canon;      // canonical index of each internal unknown
  Groups G;
  bool coarsest = false;
  int64_t a_nnz = 0;               // entries of A_l = G_l^T G_l
  // aggregation (non-coarsest)
  int block = 0;
  int64_t nagg = 0;
  int aext[3] = {1, 1, 1};
  std::vector<int64_t> astart;     // [nagg+1] omega_i = [astart[i], astart[i+1])
  std::vector<int64_t> optr;       // [nagg+1]
  std::vector<int32_t> oidx;       // Omega_i = omega_i then Gamma_i (ascending)
  std::vector<int32_t> M;          // multiplicity per group
  int n_color = 0, n_mult = 0;
  double thresh = 0.0;
  std::vector<int32_t> k;          // eigenvectors kept per aggregate
  std::vector<double> mu;          // all local eigenvalues, concatenated by aggregate
  std::vector<int64_t> muptr;      // [nagg+1]
  std::vector<int64_t> zoff;       // [nagg+1] offsets into Z
  std::vector<double> Z;           // A_i^{-1}(omega_i, Omega_i), row-major
  std::vector<int64_t> poff;       // [nagg+1] offsets into Zhat
  std::vector<double> Zhat;        // |omega_i| x k_i row-major
  std::vector<int64_t> cstart;     // [nagg+1] coarse unknowns of aggregate i
  // additive cycle only: the whole A_i^{-1} per aggregate (|Omega_i|^2,
  // symmetric, column-major), at aoff[i]
  std::vector<int64_t> aoff;
  std::vector<double> Ainv_loc;
  int64_t hazards = 0;
  // coarsest
  std::vector<double> Ainv;        // n x n dense inverse
};

struct Hierarchy {
  lsamg_params params;
  int ndim = 0;
  int64_t m0 = 0;                  // rows of the user's G after dropping empty ones
  std::vector<int64_t> row_map;    // kept user rows
  std::vector<Level> levels;
  double setup_seconds = 0.0;
};

// Build the whole hierarchy on the host.  Returns an LSAMG_* code and fills
// msg on error.
int build_hierarchy(const lsamg_csr& G, const lsamg_params& p, Hierarchy& H,
                    std::string& msg);

// Run body(i) for i in [0, n) on a pool of threads (dynamic schedule).
void parallel_for(int64_t n, const std::function<void(int64_t, int)>& body,
                  int nthreads = 0);
int default_threads();

// The dense local problems of nb aggregates on the HIP device `device`
// (setup on the device, csrc/setup_device.hip), every block padded to the
// batch's sizes: R rows of W^{1/2} G_{nz_i}, W unknowns of omega_i, Gm of
// Gamma_i, O of Omega_i.  Inputs (host, column-major, packed per aggregate):
// B (R x (Gm + W)) = W^{1/2} G_{nz_i} with its Gamma_i columns first, then
// its omega_i columns (zero in padded rows and columns); Aww (W x W) = A_ww of
// eq:gevp-S and Ai (O x O) = A(Omega_i, Omega_i), both identity on their
// padded diagonal; nw[b] the true |omega_i|.  Outputs (host): mu (W per
// aggregate) the eigenvalues of S~ u = mu A_ww u ascending, the true ones
// first; U (W x W) their A_ww-orthonormal eigenvectors; Z (O x W) the
// columns A_i^{-1} e_j, j < W; Ainv (O x O, if not null) the whole A_i^{-1};
// rank[b] the singular values of B_Gamma kept in the pseudo-inverse (those
// above rtol times the largest).  phase (7 entries, may be null): seconds
// added per phase (uploads, SVD, Schur products, Cholesky and triangular
// solves, eigensolver, local inverses, downloads), with a synchronisation
// after each.  Returns an LSAMG_* code, msg on error.
int device_local_problems(int device, int nb, int R, int W, int Gm, int O, double rtol,
                          const int32_t* nw, const double* B, const double* Aww, const double* Ai,
                          double* mu, double* U, double* Z, double* Ainv, int32_t* rank,
                          double* phase, std::string& msg);

// Whether the setup of a G with n columns runs its dense local problems on
// the device (setup_device, device): always for LSAMG_SETUP_DEVICE, from
// kAutoDeviceSetupN columns on for LSAMG_SETUP_AUTO, never without a device.
constexpr int64_t kAutoDeviceSetupN = 100000;
bool setup_on_device(const lsamg_params& p, int64_t n);

// Opens rocBLAS and rocSOLVER (whose loading registers their device code
// with the HIP runtime) and makes and releases one rocBLAS handle on
// `device`: done before other threads launch kernels, so that loading never
// overlaps their launches.  Returns an LSAMG_* code, msg on error.
int device_setup_preload(int device, std::string& msg);

// Ainv = A^{-1} for the SPD n x n matrix A (column-major, host) on the HIP
// device `device` (Cholesky factor, then solves against the identity).
int device_spd_inverse(int device, int n, const double* A, double* Ainv, std::string& msg);

// C = G^+ F for the symmetric s x s matrix G and the s x s matrix F (both
// row-major; C row-major): the pseudo-inverse drops the eigenvalues of G at
// or below rtol times the largest.  Returns the rank kept, or -1 if the
// eigen-decomposition does not converge.  (Block CG's small dense step.)
int gram_pinv_apply(int s, const double* G, const double* F, double* C, double rtol);

}  // namespace lsamg
