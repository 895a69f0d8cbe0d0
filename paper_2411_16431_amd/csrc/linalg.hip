#include "linalg.h"

namespace tnb {
namespace la {

constexpr int TILE = 16;

// One 16x16 output tile per block, K range [k0, k1) of the chunk blockIdx.z.
__global__ void gemm_kernel(int M, int N, int64_t K, int64_t kchunk, const double* __restrict__ A,
                            int64_t ars, int64_t acs, int64_t abs_, const double* __restrict__ B,
                            int64_t brs, int64_t bcs, int64_t bbs, double* __restrict__ P,
                            int64_t pbs_chunk, int64_t pbs_batch, int nb) {
  __shared__ double As[TILE][TILE + 1];
  __shared__ double Bs[TILE][TILE + 1];
  const int ntj = (N + TILE - 1) / TILE;
  const int ti = int(blockIdx.x / ntj), tj = int(blockIdx.x % ntj);
  const int b = int(blockIdx.y) % nb;
  const int chunk = int(blockIdx.y) / nb;
  const int i = ti * TILE + threadIdx.y;
  const int j = tj * TILE + threadIdx.x;
  const int64_t k0 = int64_t(chunk) * kchunk;
  const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
  const double* Ab = A + b * abs_;
  const double* Bb = B + b * bbs;
  double acc = 0.0;
  for (int64_t kt = k0; kt < k1; kt += TILE) {
    const int64_t ka = kt + threadIdx.x, kb = kt + threadIdx.y;
    const int ia = ti * TILE + threadIdx.y;
    const int jb = tj * TILE + threadIdx.x;
    As[threadIdx.y][threadIdx.x] = (ia < M && ka < k1) ? Ab[ia * ars + ka * acs] : 0.0;
    Bs[threadIdx.y][threadIdx.x] = (kb < k1 && jb < N) ? Bb[kb * brs + jb * bcs] : 0.0;
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TILE; ++kk) acc = fma(As[threadIdx.y][kk], Bs[kk][threadIdx.x], acc);
    __syncthreads();
  }
  if (i < M && j < N) P[chunk * pbs_chunk + b * pbs_batch + int64_t(i) * N + j] = acc;
}

__global__ void gemm_finish_kernel(int nb, int M, int N, int nchunk, const double* __restrict__ P,
                                   int64_t pbs_chunk, int64_t pbs_batch, double* __restrict__ C,
                                   int64_t ldc, int64_t bsc, double alpha, double beta) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(M) * N;
  if (idx >= per * nb) return;
  const int b = int(idx / per);
  const int i = int((idx % per) / N), j = int(idx % N);
  double acc = 0.0;
  for (int c = 0; c < nchunk; ++c) acc += P[c * pbs_chunk + b * pbs_batch + int64_t(i) * N + j];
  double* dst = C + b * bsc + int64_t(i) * ldc + j;
  *dst = beta == 0.0 ? alpha * acc : alpha * acc + beta * *dst;
}

// Small output (M, N <= 64) over a long K chunk on the matrix cores: one
// workgroup per (batch, chunk); wave w takes the k-steps of 4 that are w mod 4
// in the chunk and accumulates the whole output in 16x16 MFMA tiles; the four
// partial outputs are added in LDS in wave order, so the sum is deterministic.
// Without a register cap the accumulators go to AGPRs and the kernel runs one
// wave per SIMD; capped, it fits in VGPRs alone and runs three, with no spill.
typedef double v4d_s __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) gemm_small_kernel(int M, int N, int64_t K, int64_t kchunk,
                                                         const double* __restrict__ A, int64_t ars, int64_t acs,
                                                         int64_t abs_, const double* __restrict__ B, int64_t brs,
                                                         int64_t bcs, int64_t bbs, double* __restrict__ P,
                                                         int64_t pbs_chunk, int64_t pbs_batch, int nb,
                                                         double* __restrict__ C, int64_t ldc, int64_t bsc,
                                                         double alpha, double beta) {
  __shared__ double red[64][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, li = lane & 15, lk = lane >> 4;
  const int b = int(blockIdx.y) % nb, chunk = int(blockIdx.y) / nb;
  const int64_t k0 = int64_t(chunk) * kchunk;
  const int64_t k1 = k0 + kchunk < K ? k0 + kchunk : K;
  const double* Ab = A + b * abs_;
  const double* Bb = B + b * bbs;
  const int mt = (M + 15) >> 4, nt = (N + 15) >> 4;
  v4d_s acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d_s{0.0, 0.0, 0.0, 0.0};
  for (int64_t kb = k0 + 4 * w; kb < k1; kb += 16) {
    const int64_t k = kb + lk;
    const bool kok = k < k1;
    double a[4], bv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = 16 * i + li;
      a[i] = (i < mt && r < M && kok) ? Ab[r * ars + k * acs] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = 16 * j + li;
      bv[j] = (j < nt && c < N && kok) ? Bb[k * brs + c * bcs] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < mt)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < nt) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv[j], acc[i][j], 0, 0, 0);
  }
  for (int src = 0; src < 4; ++src) {
    if (w == src) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * i + 4 * v + lk, c = 16 * j + li;
            red[r][c] = src == 0 ? acc[i][j][v] : red[r][c] + acc[i][j][v];
          }
    }
    __syncthreads();
  }
  if (C) {  // a single K chunk: the result goes straight to C
    for (int i = threadIdx.x; i < M * N; i += blockDim.x) {
      double* dst = C + b * bsc + int64_t(i / N) * ldc + i % N;
      const double v = red[i / N][i % N];
      *dst = beta == 0.0 ? alpha * v : alpha * v + beta * *dst;
    }
    return;
  }
  double* Pb = P + chunk * pbs_chunk + b * pbs_batch;
  for (int i = threadIdx.x; i < M * N; i += blockDim.x) Pb[i] = red[i / N][i % N];
}

static void gemm_part(int batch, int M, int N, int64_t K, View A, View B, double* C, int64_t ldc,
                      int64_t bsc, double alpha, double beta, Scratch& ws, hipStream_t s) {
  const int64_t tiles2d = int64_t((M + TILE - 1) / TILE) * ((N + TILE - 1) / TILE);
  const int64_t tiles = tiles2d * batch;
  int64_t nchunk = 1;
  if (K > 2048 && tiles < 1024) {
    nchunk = (K + 2047) / 2048;
    int64_t cap = (4096 + tiles - 1) / tiles;
    if (nchunk > cap) nchunk = cap;
    if (nchunk * batch > 65535) nchunk = 65535 / batch;
    if (nchunk < 1) nchunk = 1;
  }
  const int64_t kchunk = K > 0 ? (K + nchunk - 1) / nchunk : 0;
  const int64_t per = int64_t(M) * N;
  double* P = ws.get(5, size_t(per * batch * nchunk));
  dim3 grid(unsigned(tiles2d), unsigned(batch * nchunk));
  {
  KTimer _t("gemm", s, 2.0 * M * double(N) * double(K) * batch,
            8.0 * (double(M) * K + double(K) * N + double(M) * N) * batch);
  if (M <= 64 && N <= 64) {
    const bool direct = nchunk == 1;
    hipLaunchKernelGGL(gemm_small_kernel, dim3(1, unsigned(batch * nchunk)), dim3(256), 0, s, M, N, K, kchunk, A.p,
                       A.rs, A.cs, A.bs, B.p, B.rs, B.cs, B.bs, P, per * batch, per, batch, direct ? C : nullptr, ldc,
                       bsc, alpha, beta);
    if (direct) {
      HIPC(hipGetLastError());
      return;
    }
  } else {
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(TILE, TILE), 0, s, M, N, K, kchunk, A.p, A.rs, A.cs,
                       A.bs, B.p, B.rs, B.cs, B.bs, P, per * batch, per, batch);
  }
  HIPC(hipGetLastError());
  }
  const int64_t tot = per * batch;
  hipLaunchKernelGGL(gemm_finish_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, s, batch,
                     M, N, int(nchunk), P, per * batch, per, C, ldc, bsc, alpha, beta);
  HIPC(hipGetLastError());
}


void gemm(int batch, int M, int N, int64_t K, View A, View B, double* C, int64_t ldc, int64_t bsc,
          double alpha, double beta, Scratch& ws, hipStream_t s) {
  if (batch <= 0 || M <= 0 || N <= 0) return;
  // Enough output tiles to fill the chip: the matrix-core kernel, which sums
  // all of K per tile.  Few tiles over a long K (Gram matrices): the split-K
  // vector kernel below.
  const int64_t mt = int64_t((M + 127) / 128) * ((N + 63) / 64) * batch;
  if (mt >= 128 && K < (int64_t(1) << 31)) {
    Operand a{A.p, A.bs, Ix{0, 0, A.rs}, Ix{0, 0, A.cs}};
    Operand b{B.p, B.bs, Ix{0, 0, B.rs}, Ix{0, 0, B.cs}};
    gemm_mfma(batch, M, N, int(K), a, b, C, Ix{0, 0, ldc}, Ix{0, 0, 1}, bsc, alpha, beta, s, "gemm");
    return;
  }
  const int maxb = 32768;
  for (int b0 = 0; b0 < batch; b0 += maxb) {
    const int nb = batch - b0 < maxb ? batch - b0 : maxb;
    View a{A.p + A.bs * b0, A.rs, A.cs, A.bs}, bb{B.p + B.bs * b0, B.rs, B.cs, B.bs};
    gemm_part(nb, M, N, K, a, bb, C + bsc * b0, ldc, bsc, alpha, beta, ws, s);
  }
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi (Golub & Van Loan, Sec. 8.5) with the round-robin ordering:
// each round applies up to s/2 disjoint rotations at once.
// G and V are the working matrices (global memory, or LDS in the _lds
// variant); sh is 2560 doubles of LDS scratch.
__device__ void jacobi_body(double* __restrict__ G, int s, double* __restrict__ V, double* __restrict__ lam,
                            double* __restrict__ sh) {
  double* cs = sh;                 // [m/2] cosines
  double* sn = sh + 512;           // [m/2] sines
  int* pp = reinterpret_cast<int*>(sh + 1024);
  int* qq = pp + 512;
  double* red = sh + 1536;         // [1024]
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = s + (s & 1);       // even number of players (one dummy if odd)
  for (int idx = tid; idx < s * s; idx += nt) V[idx] = (idx / s == idx % s) ? 1.0 : 0.0;
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int idx = tid; idx < s * s; idx += nt) {
      double g = G[idx];
      tot += g * g;
      if (idx / s != idx % s) off += g * g;
    }
    // both sums in one tree (cs and sn, 1024 doubles together, are free here)
    double* red2 = cs;
    red[tid] = off;
    red2[tid] = tot;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[tid] += red[tid + w];
        red2[tid] += red2[tid + w];
      }
      __syncthreads();
    }
    off = red[0];
    tot = red2[0];
    __syncthreads();
    if (!(off > 1e-30 * tot) || tot == 0.0) break;
    for (int round = 0; round < m - 1; ++round) {
      // pair list of this round: player 0 fixed, others rotate
      for (int a = tid; a < m / 2; a += nt) {
        int p1 = (a == 0) ? 0 : 1 + (a - 1 + round) % (m - 1);
        int p2 = 1 + (m - 2 - a + round) % (m - 1);
        int p = p1 < p2 ? p1 : p2, q = p1 < p2 ? p2 : p1;
        double c = 1.0, sv = 0.0;
        if (q < s) {
          double apq = G[p * s + q];
          if (apq != 0.0) {
            double tau = (G[q * s + q] - G[p * s + p]) / (2.0 * apq);
            double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sv = t * c;
          }
        }
        pp[a] = p;
        qq[a] = q;
        cs[a] = c;
        sn[a] = sv;
      }
      __syncthreads();
      // G <- J^T G J and V <- V J in one phase: the pairs are disjoint, so
      // every 2x2 block (rows of pair a, columns of pair b) is updated by one
      // thread, rows first then columns -- the same operations, in the same
      // order, as a row pass followed by a column pass
      const int h = m / 2;
      for (int idx = tid; idx < h * h + h * s; idx += nt) {
        if (idx < h * h) {
          const int a = idx / h, b = idx % h;
          const int pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
          const bool qar = qa < s, qbr = qb < s;
          const bool ra = qar && sn[a] != 0.0, rb = qbr && sn[b] != 0.0;
          if (!ra && !rb) continue;
          double xpp = G[pa * s + pb];
          double xpq = qbr ? G[pa * s + qb] : 0.0;
          double xqp = qar ? G[qa * s + pb] : 0.0;
          double xqq = (qar && qbr) ? G[qa * s + qb] : 0.0;
          if (ra) {
            const double ypp = cs[a] * xpp - sn[a] * xqp, yqp = sn[a] * xpp + cs[a] * xqp;
            const double ypq = cs[a] * xpq - sn[a] * xqq, yqq = sn[a] * xpq + cs[a] * xqq;
            xpp = ypp; xqp = yqp; xpq = ypq; xqq = yqq;
          }
          if (rb) {
            const double zpp = cs[b] * xpp - sn[b] * xpq, zpq = sn[b] * xpp + cs[b] * xpq;
            const double zqp = cs[b] * xqp - sn[b] * xqq, zqq = sn[b] * xqp + cs[b] * xqq;
            xpp = zpp; xpq = zpq; xqp = zqp; xqq = zqq;
          }
          G[pa * s + pb] = xpp;
          if (qbr) G[pa * s + qb] = xpq;
          if (qar) G[qa * s + pb] = xqp;
          if (qar && qbr) G[qa * s + qb] = xqq;
        } else {
          const int jdx = idx - h * h;
          const int a = jdx / s, k = jdx % s;
          const int p = pp[a], q = qq[a];
          if (q >= s || sn[a] == 0.0) continue;
          const double vp = V[k * s + p], vq = V[k * s + q];
          V[k * s + p] = cs[a] * vp - sn[a] * vq;
          V[k * s + q] = sn[a] * vp + cs[a] * vq;
        }
      }
      __syncthreads();
    }
  }
  // sort eigenpairs by descending eigenvalue (ties by index): rank scatter
  double* d = red;  // reuse: diagonal
  for (int i = tid; i < s; i += nt) d[i] = G[i * s + i];
  __syncthreads();
  int* rank = reinterpret_cast<int*>(cs);
  for (int i = tid; i < s; i += nt) {
    int r = 0;
    for (int j = 0; j < s; ++j) r += (d[j] > d[i]) || (d[j] == d[i] && j < i);
    rank[i] = r;
  }
  __syncthreads();
  for (int i = tid; i < s; i += nt) lam[rank[i]] = d[i];
  // permute V columns in place through G as temporary
  for (int idx = tid; idx < s * s; idx += nt) G[idx] = V[idx];
  __syncthreads();
  for (int idx = tid; idx < s * s; idx += nt) {
    int row = idx / s, col = idx % s;
    V[row * s + rank[col]] = G[idx];
  }
}

__global__ void __launch_bounds__(1024) jacobi_kernel(double* __restrict__ G, int s, double* __restrict__ V,
                                                      double* __restrict__ lam) {
  extern __shared__ double sh[];
  jacobi_body(G, s, V, lam, sh);
}

// The same with G and V held in LDS (2 s^2 + 2560 doubles): every rotation
// round reads and writes LDS instead of L2.
__global__ void __launch_bounds__(1024) jacobi_lds_kernel(double* __restrict__ Gg, int s, double* __restrict__ Vg,
                                                          double* __restrict__ lam) {
  extern __shared__ double sh[];
  double* G = sh + 2560;
  double* V = G + s * s;
  for (int i = threadIdx.x; i < s * s; i += blockDim.x) G[i] = Gg[i];
  __syncthreads();
  jacobi_body(G, s, V, lam, sh);
  __syncthreads();
  for (int i = threadIdx.x; i < s * s; i += blockDim.x) Vg[i] = V[i];
}

static bool lds_fits(int m) { return (2560 + 2 * size_t(m) * m) * sizeof(double) <= 163840; }

template <class K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536)
    HIPC(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(bytes)));
}

void eigh(double* G, int s, double* V, double* lam, hipStream_t st) {
  if (s <= 0) return;
  if (s > 1000) fail(TNB_EUNSUPPORTED, "eigensolver limited to 1000 x 1000");
  KTimer _t("eigh", st, 0.0, 16.0 * s * s);
  if (lds_fits(s)) {
    const size_t shm = (2560 + 2 * size_t(s) * s) * sizeof(double);
    allow_lds(jacobi_lds_kernel, shm);
    // G stays in place (the kernel works on an LDS copy), so the launch
    // widths can be timed against each other: 16 or 4 waves
    auto run = [&](int v) {
      hipLaunchKernelGGL(jacobi_lds_kernel, dim3(1), dim3(v == 0 ? 1024 : 256), shm, st, G, s, V, lam);
      HIPC(hipGetLastError());
    };
    char key[64];
    std::snprintf(key, sizeof key, "eigh s%d", s);
    autotune_pick(key, s <= 128 ? 2 : 1, run, st);
  } else {
    hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), 2560 * sizeof(double), st, G, s, V, lam);
  }
  HIPC(hipGetLastError());
}

// W (s x s) = V[:, keep] * diag(1/sqrt(lam)) for lam > thr * lam0, else 0.
__global__ void inv_sqrt_weights_kernel(const double* __restrict__ V, const double* __restrict__ lam,
                                        int s, double rel, double* __restrict__ W) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= s * s) return;
  const int col = idx % s;
  const double l0 = lam[0], l = lam[col];
  W[idx] = (l0 > 0.0 && l > rel * l0) ? V[idx] / sqrt(l) : 0.0;
}

// One-sided Jacobi SVD (Hestenes; Golub & Van Loan Sec. 8.6.3) of a small
// n x m matrix A, overwritten by U*S: rotations orthogonalise the columns
// pairwise, round-robin over disjoint pairs.  Singular values are accurate to
// eps * sigma_max.  Outputs sorted descending: S[m], U (n x m row-major,
// columns of A normalised; zero for sigma = 0), V (m x m row-major).
//
// CM selects the working layout of A and V: column-major with leading
// dimension ld (LDS: a column is contiguous, so the lanes of a pair read
// consecutive words; ld is odd so that the pairs of a wave start on different
// banks), or row-major with ld = m (the global-memory variant).  A needs room
// for max(n, m) rows.  sh is 64 doubles of LDS scratch; nrm and rank hold m
// entries each.
//
// A column pair is owned by a group of L lanes for the whole round: the group
// forms the three dot products (strided partial sums, then a butterfly that
// leaves the same sum on every lane), derives the rotation and applies it to
// the rows it read, so one barrier per round suffices.  Columns whose squared
// norm is at most 1e-28 ||A||_F^2 (rank deficiency: the n < m columns beyond
// the rank, or a rank-deficient R) are left alone and do not count towards
// convergence; their singular values are at the rounding level.
template <bool CM>
__device__ void hestenes_body(double* __restrict__ A, int n, int m, int ld, double* __restrict__ U,
                              double* __restrict__ V, double* __restrict__ S, double* __restrict__ sh,
                              double* __restrict__ nrm, int* __restrict__ rank) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int mm = m + (m & 1), np = mm / 2;
  const int vld = CM ? (m | 1) : m;
  auto at = [&](double* X, int xld, int i, int j) -> double& { return CM ? X[size_t(j) * xld + i] : X[size_t(i) * m + j]; };
  for (int idx = tid; idx < m * m; idx += nt) at(V, vld, idx / m, idx % m) = (idx / m == idx % m) ? 1.0 : 0.0;
  // block reductions through sh: wave partials in sh[0..15], result in sh[32]
  auto block_sum = [&](double x, bool take_max) -> double {
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(x, o, 64);
      x = take_max ? fmax(x, y) : x + y;
    }
    __syncthreads();
    if ((tid & 63) == 0) sh[tid >> 6] = x;
    __syncthreads();
    if (tid == 0) {
      double r = sh[0];
      for (int w = 1; w < (nt + 63) / 64; ++w) r = take_max ? fmax(r, sh[w]) : r + sh[w];
      sh[32] = r;
    }
    __syncthreads();
    return sh[32];
  };
  double f2 = 0.0;
  for (int idx = tid; idx < n * m; idx += nt) {
    const double x = at(A, ld, idx / m, idx % m);
    f2 = fma(x, x, f2);
  }
  const double tiny = 1e-28 * block_sum(f2, false);
  int L = 16;
  while (L > 1 && np * L > nt) L >>= 1;
  const int groups = nt / L;                       // pairs handled at once
  const int iters = (np + groups - 1) / groups;    // the same count on every lane
  const int sub = tid % L;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double worst = 0.0;
    for (int round = 0; round < mm - 1; ++round) {
      for (int it = 0; it < iters; ++it) {
        const int a = it * groups + tid / L;
        const bool act = a < np;
        int p = 0, q = m;
        if (act) {
          const int p1 = (a == 0) ? 0 : 1 + (a - 1 + round) % (mm - 1);
          const int p2 = 1 + (mm - 2 - a + round) % (mm - 1);
          p = p1 < p2 ? p1 : p2;
          q = p1 < p2 ? p2 : p1;
        }
        const bool real = act && q < m;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (real)
          for (int i = sub; i < n; i += L) {
            const double x = at(A, ld, i, p), y = at(A, ld, i, q);
            al = fma(x, x, al);
            be = fma(y, y, be);
            ga = fma(x, y, ga);
          }
        for (int o = L / 2; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, L);
          be += __shfl_xor(be, o, L);
          ga += __shfl_xor(ga, o, L);
        }
        if (real && al > tiny && be > tiny && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), sv = c * t;
          worst = fmax(worst, fabs(ga) / sqrt(al * be));
          for (int i = sub; i < n; i += L) {
            const double x = at(A, ld, i, p), y = at(A, ld, i, q);
            at(A, ld, i, p) = c * x - sv * y;
            at(A, ld, i, q) = sv * x + c * y;
          }
          for (int i = sub; i < m; i += L) {
            const double vx = at(V, vld, i, p), vy = at(V, vld, i, q);
            at(V, vld, i, p) = c * vx - sv * vy;
            at(V, vld, i, q) = sv * vx + c * vy;
          }
        }
      }
      __syncthreads();  // the next round pairs the columns differently
    }
    if (block_sum(worst, true) <= 1e-15) break;
  }
  // column norms, sort descending (ties by index), normalise
  for (int j = tid; j < m; j += nt) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = fma(at(A, ld, i, j), at(A, ld, i, j), acc);
    nrm[j] = sqrt(acc);
  }
  __syncthreads();
  for (int j = tid; j < m; j += nt) {
    int r = 0;
    for (int o = 0; o < m; ++o) r += (nrm[o] > nrm[j]) || (nrm[o] == nrm[j] && o < j);
    rank[j] = r;
  }
  __syncthreads();
  for (int j = tid; j < m; j += nt) S[rank[j]] = nrm[j];
  for (int idx = tid; idx < n * m; idx += nt) {
    const int i = idx / m, j = idx % m;
    U[size_t(i) * m + rank[j]] = nrm[j] > 0.0 ? at(A, ld, i, j) / nrm[j] : 0.0;
  }
  __syncthreads();
  // V columns permuted through A as scratch; V leaves row-major (m x m)
  for (int idx = tid; idx < m * m; idx += nt) A[idx] = at(V, vld, idx / m, idx % m);
  __syncthreads();
  for (int idx = tid; idx < m * m; idx += nt) V[size_t(idx / m) * m + rank[idx % m]] = A[idx];
}

__global__ void __launch_bounds__(1024) hestenes_kernel(double* __restrict__ A, int m, double* __restrict__ U,
                                                        double* __restrict__ V, double* __restrict__ S) {
  __shared__ double sh[64], nrm[1024];
  __shared__ int rank[1024];
  hestenes_body<false>(A, m, m, m, U, V, S, sh, nrm, rank);
}

// The same with A and V held in LDS, column-major with leading dimension
// m | 1, after 64 + 2 m doubles of scratch.
static size_t hestenes_lds_bytes(int m) { return (64 + 2 * size_t(m) + 2 * size_t(m | 1) * m) * sizeof(double); }

__global__ void __launch_bounds__(1024) hestenes_lds_kernel(const double* __restrict__ Ag, int m,
                                                            double* __restrict__ U, double* __restrict__ Vg,
                                                            double* __restrict__ S) {
  extern __shared__ double sh[];
  const int ld = m | 1;
  double* nrm = sh + 64;
  int* rank = reinterpret_cast<int*>(nrm + m);
  double* A = nrm + 2 * m;
  double* V = A + size_t(ld) * m;
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) A[size_t(i % m) * ld + i / m] = Ag[i];
  __syncthreads();
  hestenes_body<true>(A, m, m, ld, U, V, S, sh, nrm, rank);
  __syncthreads();
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) Vg[i] = V[i];
}

static void hestenes(double* A, int m, double* U, double* V, double* S, hipStream_t st) {
  if (m > 1000) fail(TNB_EUNSUPPORTED, "SVD limited to 1000 x 1000");
  KTimer _t("svd_small", st, 0.0, 24.0 * m * m);
  if (hestenes_lds_bytes(m) <= 163840) {
    const size_t shm = hestenes_lds_bytes(m);
    allow_lds(hestenes_lds_kernel, shm);
    // A stays in place (LDS copy): 16 or 4 waves, timed by the autotuner
    auto run = [&](int v) {
      hipLaunchKernelGGL(hestenes_lds_kernel, dim3(1), dim3(v == 0 ? 1024 : 256), shm, st, A, m, U, V, S);
      HIPC(hipGetLastError());
    };
    char key[64];
    std::snprintf(key, sizeof key, "hestenes m%d", m);
    autotune_pick(key, m <= 128 ? 2 : 1, run, st);
  } else {
    hipLaunchKernelGGL(hestenes_kernel, dim3(1), dim3(1024), 0, st, A, m, U, V, S);
  }
  HIPC(hipGetLastError());
}

// Wn[:, j] = V[:, j] for lam_j > rel * lam_0 (unscaled), else 0
__global__ void keep_weights_kernel(const double* __restrict__ V, const double* __restrict__ lam, int m,
                                    double rel, double* __restrict__ W) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int col = idx % m;
  W[idx] = (lam[0] > 0.0 && lam[col] > rel * lam[0]) ? V[idx] : 0.0;
}

// dinv[j] = 1/sqrt(G[j][j]) (0 for an empty column); G <- D^-1/2 G D^-1/2
__global__ void normalise_gram_kernel(double* __restrict__ G, int m, double* __restrict__ dinv) {
  __shared__ double d[1024];
  for (int j = threadIdx.x; j < m; j += blockDim.x) d[j] = G[j * m + j] > 0.0 ? 1.0 / sqrt(G[j * m + j]) : 0.0;
  __syncthreads();
  for (int idx = threadIdx.x; idx < m * m; idx += blockDim.x) G[idx] *= d[idx / m] * d[idx % m];
  for (int j = threadIdx.x; j < m; j += blockDim.x) dinv[j] = d[j];
}

// W2[i][j] = dinv[i] V2[i][j] / sqrt(lam2[j]) for lam2[j] > thr (absolute), else 0
__global__ void ortho_weights_kernel(const double* __restrict__ V2, const double* __restrict__ lam2,
                                     const double* __restrict__ dinv, int m, double thr, double* __restrict__ W) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int i = idx / m, j = idx % m;
  W[idx] = lam2[j] > thr ? dinv[i] * V2[idx] / sqrt(lam2[j]) : 0.0;
}

// Accurate thin SVD of a tall n x m matrix M (m small):
//   (1) eigenvectors V of the Gram matrix M^T M, kept down to
//       lambda/lambda_max = 1e-14 (sigma ratio 1e-7): Q1 = M V,
//   (2) Q1's columns scaled to unit norm (measured, not 1/sqrt(lambda), which
//       is unreliable for small lambda), their Gram matrix diagonalised, and
//       Q = Q1 D^-1/2 V2 L2^-1/2 over eigenvalues above 1e-6 (orthonormal),
//   (3) R = Q^T M by GEMM, (4) one-sided Jacobi SVD R = U_R S V_R^T,
//   (5) M = (Q U_R) S V_R^T.
// Singular values above 1e-7 * sigma_max carry errors of order
// eps * sigma_max, as with a Householder-based SVD.
// Outputs: Uo (n x m) = Q U_R, S (m, descending), Vo (m x m) = V_R.
static void tall_svd(const double* M, int64_t n, int m, double* Uo, double* S, double* Vo, Scratch& ws,
                     hipStream_t st) {
  if (m > 1024) fail(TNB_EUNSUPPORTED, "thin SVD limited to 1024 columns");
  double* G = ws.get(0, size_t(m) * m);
  double* V = ws.get(1, size_t(m) * m);
  double* lam = ws.get(2, size_t(m) + size_t(m));  // lam and dinv
  double* dinv = lam + m;
  double* W = ws.get(3, size_t(m) * m);
  double* Q1 = ws.get(4, size_t(n) * m);
  const unsigned gb = unsigned((m * m + 255) / 256);
  gemm(1, m, m, n, View{M, 1, m, 0}, View{M, m, 1, 0}, G, m, 0, 1.0, 0.0, ws, st);
  eigh(G, m, V, lam, st);
  hipLaunchKernelGGL(keep_weights_kernel, dim3(gb), dim3(256), 0, st, V, lam, m, 1e-14, W);
  gemm(1, int(n), m, m, View{M, m, 1, 0}, View{W, m, 1, 0}, Q1, m, 0, 1.0, 0.0, ws, st);
  gemm(1, m, m, n, View{Q1, 1, m, 0}, View{Q1, m, 1, 0}, G, m, 0, 1.0, 0.0, ws, st);
  hipLaunchKernelGGL(normalise_gram_kernel, dim3(1), dim3(256), 0, st, G, m, dinv);
  eigh(G, m, V, lam, st);
  hipLaunchKernelGGL(ortho_weights_kernel, dim3(gb), dim3(256), 0, st, V, lam, dinv, m, 1e-6, W);
  HIPC(hipGetLastError());
  // Q (into Uo) = Q1 W
  gemm(1, int(n), m, m, View{Q1, m, 1, 0}, View{W, m, 1, 0}, Uo, m, 0, 1.0, 0.0, ws, st);
  // R = Q^T M  (m x m) into G
  gemm(1, m, m, n, View{Uo, 1, m, 0}, View{M, m, 1, 0}, G, m, 0, 1.0, 0.0, ws, st);
  double* UR = W;  // reuse
  hestenes(G, m, UR, Vo, S, st);
  // Uo <- Q U_R  (through Q1 as scratch)
  gemm(1, int(n), m, m, View{Uo, m, 1, 0}, View{UR, m, 1, 0}, Q1, m, 0, 1.0, 0.0, ws, st);
  HIPC(hipMemcpyAsync(Uo, Q1, size_t(n) * m * sizeof(double), hipMemcpyDeviceToDevice, st));
}

// Thin SVD of a small n x m matrix in one workgroup: M is copied to LDS and
// orthogonalised there by the one-sided Jacobi rotations directly (no Gram
// pass), then the leading t triplets are written with those at or below
// cut * sigma_max zeroed together with their vectors: U (n x t), S (t),
// VT (t x m).  One launch instead of the Gram path's twenty, for the many
// tiny blocks of small clusters.  LDS: A (max(n,m) x m), V (m x m), U (n x m)
// and 2560 doubles of scratch.
__global__ void __launch_bounds__(256) small_svd_kernel(const double* __restrict__ M, int n, int m, int t,
                                                        double cut, double* __restrict__ Uo, double* __restrict__ So,
                                                        double* __restrict__ VT) {
  extern __shared__ double sh[];
  const int nr = n > m ? n : m, ld = nr | 1;
  double* nrm = sh + 64;
  int* rank = reinterpret_cast<int*>(nrm + m);
  double* A = nrm + 2 * m;                 // column-major, ld x m
  double* V = A + size_t(ld) * m;          // column-major, (m | 1) x m
  double* U = V + size_t(m | 1) * m;
  double* S = U + size_t(n) * m;
  for (int i = threadIdx.x; i < n * m; i += blockDim.x) A[size_t(i % m) * ld + i / m] = M[i];
  __syncthreads();
  hestenes_body<true>(A, n, m, ld, U, V, S, sh, nrm, rank);
  __syncthreads();
  const double s0 = S[0];
  for (int idx = threadIdx.x; idx < t * m; idx += blockDim.x) {
    const int i = idx / m, col = idx % m;
    const bool keep = i < m && s0 > 0.0 && S[i] > cut * s0;
    VT[idx] = keep ? V[col * m + i] : 0.0;
    if (col == 0) So[i] = keep ? S[i] : 0.0;
  }
  if (Uo)
    for (int idx = threadIdx.x; idx < n * t; idx += blockDim.x) {
      const int r = idx / t, j = idx % t;
      const bool keep = j < m && s0 > 0.0 && S[j] > cut * s0;
      Uo[idx] = keep ? U[r * m + j] : 0.0;
    }
}

static size_t small_svd_lds(int64_t n, int m) {
  const int64_t nr = n > m ? n : m;
  return size_t(64 + 2 * m + (nr | 1) * m + int64_t(m | 1) * m + n * m + m) * sizeof(double);
}
static bool small_svd_fits(int64_t n, int m) { return m <= 64 && n <= 4096 && small_svd_lds(n, m) <= 163840; }

static void small_svd(const double* M, int64_t n, int m, int t, double cut, double* U, double* S, double* VT,
                      hipStream_t st) {
  KTimer _t("svd_small", st, 0.0, 8.0 * (double(n) * m + double(n) * t + double(t) * m));
  const size_t shm = small_svd_lds(n, m);
  if (shm > 65536)
    HIPC(hipFuncSetAttribute(reinterpret_cast<const void*>(small_svd_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(shm)));
  hipLaunchKernelGGL(small_svd_kernel, dim3(1), dim3(256), shm, st, M, int(n), m, t, cut, U, S, VT);
  HIPC(hipGetLastError());
}

// keep columns j with S[j] > cut * S[0]: Q[:, j] = U[:, j] (else 0)
__global__ void keep_cols_kernel(const double* __restrict__ U, const double* __restrict__ S, int64_t n, int m,
                                 double cut, double* __restrict__ Q) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int j = int(idx % m);
  Q[idx] = (S[0] > 0.0 && S[j] > cut * S[0]) ? U[idx] : 0.0;
}

void orth(const double* Y, int64_t n, int s, double cut, double* Q, Scratch& ws, hipStream_t st) {
  if (small_svd_fits(n, s)) {  // Q = U with the dropped columns zeroed
    small_svd(Y, n, s, s, cut, Q, ws.get(7, size_t(s)), ws.get(8, size_t(s) * s), st);
    return;
  }
  double* Ub = ws.get(6, size_t(n) * s);
  double* Sb = ws.get(7, size_t(s));
  double* Vb = ws.get(8, size_t(s) * s);
  tall_svd(Y, n, s, Ub, Sb, Vb, ws, st);
  hipLaunchKernelGGL(keep_cols_kernel, dim3(unsigned((int64_t(n) * s + 255) / 256)), dim3(256), 0, st, Ub,
                     Sb, int64_t(n), s, cut, Q);
  HIPC(hipGetLastError());
}

// S[i] (0 if dropped), Uo columns zeroed if dropped, VT = V[:, :t]^T (zero rows if dropped)
__global__ void svd_trunc_kernel(double* __restrict__ U, int64_t n, int m, int t, double cut,
                                 const double* __restrict__ Sfull, const double* __restrict__ V,
                                 double* __restrict__ Uout, double* __restrict__ S, double* __restrict__ VT) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const bool first = idx < int64_t(t) * m;
  if (first) {
    const int i = int(idx / m), col = int(idx % m);
    const bool keep = Sfull[0] > 0.0 && Sfull[i] > cut * Sfull[0];
    VT[idx] = keep ? V[col * m + i] : 0.0;
    if (col == 0) S[i] = keep ? Sfull[i] : 0.0;
  }
  if (Uout && idx < n * t) {
    const int64_t r = idx / t;
    const int j = int(idx % t);
    const bool keep = Sfull[0] > 0.0 && Sfull[j] > cut * Sfull[0];
    Uout[idx] = keep ? U[r * m + j] : 0.0;
  }
}

void thin_svd_tall(const double* M, int64_t n, int m, int t, double cut, double* U, double* S,
                   double* VT, Scratch& ws, hipStream_t st) {
  if (small_svd_fits(n, m) && t <= m) {
    small_svd(M, n, m, t, cut, U, S, VT, st);
    return;
  }
  double* Ub = ws.get(6, size_t(n) * m);
  double* Sb = ws.get(7, size_t(m));
  double* Vb = ws.get(8, size_t(m) * m);
  tall_svd(M, n, m, Ub, Sb, Vb, ws, st);
  const int64_t tot = std::max<int64_t>(int64_t(n) * t, int64_t(t) * m);
  hipLaunchKernelGGL(svd_trunc_kernel, dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, Ub, int64_t(n), m, t,
                     cut, Sb, Vb, U, S, VT);
  HIPC(hipGetLastError());
}

}  // namespace la
}  // namespace tnb
