// FP64 dense linear algebra used by the compression: strided batched GEMM,
// symmetric eigendecomposition (cyclic Jacobi, one workgroup) and the
// Gram-based orthonormalisation / thin SVD built on them.
#pragma once
#include "common.h"

namespace tnb {
namespace la {

// Element (i, j) of batch b lives at p[b*bs + i*rs + j*cs].
struct View {
  const double* p;
  int64_t rs, cs, bs;
};

// Reusable device scratch (grows, never shrinks).
struct Scratch {
  DevBuf<double> buf[9];
  double* get(int slot, size_t n) {
    if (buf[slot].n < n) buf[slot].alloc(n + n / 4 + 64);
    return buf[slot].p;
  }
};

// C[b] (M x N, row-major with leading dimension ldc, batch stride bsc)
//   = alpha * A[b] (M x K) . B[b] (K x N) + beta * C[b].
// Deterministic: K is split into fixed chunks whose partial products are
// summed in chunk order.
void gemm(int batch, int M, int N, int64_t K, View A, View B, double* C, int64_t ldc, int64_t bsc,
          double alpha, double beta, Scratch& ws, hipStream_t s);

// Symmetric eigendecomposition of G (s x s, row-major, overwritten):
// lam[i] descending, V[:, i] (row-major s x s) the eigenvectors.
void eigh(double* G, int s, double* V, double* lam, hipStream_t st);

// Orthonormal basis of the numerical range of Y (n x s, row-major): Q (n x s)
// holds the left singular vectors with singular value > cut * largest,
// remaining columns zero (accurate thin SVD, see thin_svd_tall).
void orth(const double* Y, int64_t n, int s, double cut, double* Q, Scratch& ws, hipStream_t st);

// Thin SVD of a tall M (n x m, m <= 1000): M = U S V^T with the leading t
// triplets kept and sigma <= cut * sigma_max set to 0 (with their vectors).
// A Gram pass gives an orthonormal basis Q of range(M); R = Q^T M is then
// decomposed by one-sided Jacobi, so singular values carry errors of order
// eps * sigma_max, as with a Householder-based SVD.
//   U (n x t) [if not null], S (t), VT (t x m).
void thin_svd_tall(const double* M, int64_t n, int m, int t, double cut, double* U, double* S,
                   double* VT, Scratch& ws, hipStream_t st);

}  // namespace la
}  // namespace tnb

namespace tnb {
namespace la {

// Index map of one operand dimension: i -> (i / n0) * s1 + (i % n0) * s0, or
// i * s0 when n0 == 0.  It lets a GEMM read tensors whose row or column
// index is a pair of tensor indices with unrelated strides.
struct Ix {
  uint32_t n0 = 0;
  int64_t s1 = 0, s0 = 0;
};
struct Operand {
  const double* p = nullptr;
  int64_t bs = 0;  // batch stride
  Ix r, c;         // row and column maps
};

// C(m, n) = alpha * sum_k A(m, k) B(k, n) + beta * C(m, n) for every batch,
// on the FP64 matrix cores (16x16x4 MFMA), in 128 x 64, 128 x 128 or 64 x 64
// output tiles (chosen per shape by the autotuner; defined in gemm_mfma.hip),
// each tile owned by one workgroup and summed over all of K in order, so the
// result is deterministic and the same for every tile choice.
// tag selects a separately named kernel instance (same code): 0 general,
// 1 .. 5 the mediating diagram's G2, out, Y2, W2 and left-transfer products.
void gemm_mfma(int batch, int M, int N, int K, const Operand& A, const Operand& B, double* C, Ix cr, Ix cc,
               int64_t cbs, double alpha, double beta, hipStream_t s, const char* timer = "gemm_mfma", int tag = 0);

}  // namespace la
}  // namespace tnb
