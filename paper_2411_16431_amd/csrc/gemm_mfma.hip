#include "linalg.h"

// ---------------------------------------------------------------------------
// FP64 GEMM on the matrix cores.  v_mfma_f64_16x16x4f64 multiplies a 16x4 A
// block by a 4x16 B block: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and receives D[4 v + l / 16][l % 16] in item v.
// A workgroup of four waves (2 x 2) owns a (32 BM) x (32 BN) tile of C; each
// wave a BM x BN grid of 16 x 16 MFMA blocks.  K advances in slices of 16
// staged in LDS, the next slice prefetched into registers while the current
// one is used.  Launch variants: 128 x 64 (BM = 4, BN = 2; registers capped
// at three waves per SIMD, which it fits without spilling), 128 x 128 (twice
// the reuse of each A element, two waves per SIMD) and 64 x 64 (more tiles for
// small outputs); all sum K in the same order, so their results are
// bit-identical and the autotuner picks among them.  Which operand index is
// staged along the unit stride is a template parameter (KF), so each instance
// holds only the staging offsets it uses.  When the k map of both operands
// splits at a multiple of 16 (or not at all), every 16-slice of k lies in one
// block of the map and a staged element's offset is the slice's (uniform)
// base plus a per-thread constant: no integer division in the K loop.
namespace tnb {
namespace la {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GK = 16;

__device__ __forceinline__ int64_t ix_off(uint32_t i, const Ix& x) {
  return x.n0 ? int64_t(i / x.n0) * x.s1 + int64_t(i % x.n0) * x.s0 : int64_t(i) * x.s0;
}

// TAG only names the instance (one per use in the mediating diagram, 0 for
// the rest), so that kernel traces tell the uses apart.  KF bit 0: A is
// staged along k; bit 1: B is; bit 2: the k maps split at multiples of GK.
template <int TAG, int BM, int BN, int KF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BM * BN <= 8 ? 3 : 2)))
gemm_mfma_kernel(int M, int N, int K, Operand A, Operand B, double* __restrict__ C, Ix cr, Ix cc, int64_t cbs,
                 double alpha, double beta, int tiles_n) {
  constexpr bool a_kfast = (KF & 1) != 0, b_kfast = (KF & 2) != 0, fastk = (KF & 4) != 0;
  constexpr int TM = 32 * BM, TN = 32 * BN;          // the workgroup's tile
  constexpr int NA = TM * GK / 256, NB = TN * GK / 256;  // staged elements per thread
  constexpr int SA = 256 / TM, SB = 256 / TN;         // k rows per pass when staging along m / n
  __shared__ double As[GK][TM + 1];
  __shared__ double Bs[GK][TN + 1];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int tm0 = int(blockIdx.x / tiles_n) * TM, tn0 = int(blockIdx.x % tiles_n) * TN;
  const int b = blockIdx.y;
  const double* Ap = A.p + b * A.bs;
  const double* Bp = B.p + b * B.bs;
  // Staging: along the unit-stride index consecutive threads take consecutive
  // elements; the other index of a thread's elements is fixed, so its offsets
  // are computed once.
  double ra[NA], rb[NB];
  // A: kfast -> k = t % 16 fixed, m = t / 16 + 16 i;  else m = t % TM fixed, k = t / TM + SA i
  int64_t a_fixed[NA];
  uint32_t a_ok = 0;
  if (a_kfast) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int gm = tm0 + t / GK + 16 * i;
      a_fixed[i] = gm < M ? ix_off(uint32_t(gm), A.r) : 0;
      a_ok |= uint32_t(gm < M) << i;
    }
  } else {
    const int gm = tm0 + t % TM;
    a_fixed[0] = gm < M ? ix_off(uint32_t(gm), A.r) : 0;
    a_ok = gm < M ? 0xffffu : 0u;
  }
  // B: kfast -> k = t % 16 fixed, n = t / 16 + 16 i;  else n = t % TN fixed, k = t / TN + SB i
  int64_t b_fixed[NB];
  uint32_t b_ok = 0;
  if (b_kfast) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int gn = tn0 + t / GK + 16 * i;
      b_fixed[i] = gn < N ? ix_off(uint32_t(gn), B.c) : 0;
      b_ok |= uint32_t(gn < N) << i;
    }
  } else {
    const int gn = tn0 + t % TN;
    b_fixed[0] = gn < N ? ix_off(uint32_t(gn), B.c) : 0;
    b_ok = gn < N ? 0xffffu : 0u;
  }
  // Offset of k = k0 + dk (dk < GK) in an operand's k map.  With fastk,
  // base and rem hold the offset of k0 and k0 mod n0 for the slice being
  // loaded (slices are loaded in order) and step to the next one by additions.
  int64_t a_base = 0, b_base = 0;
  uint32_t a_rem = 0, b_rem = 0;
  auto koff = [&](int k0, int dk, const Ix& x, int64_t base) -> int64_t {
    return fastk ? base + int64_t(dk) * x.s0 : ix_off(uint32_t(k0 + dk), x);
  };
  auto step = [&](const Ix& x, int64_t& base, uint32_t& rem) {
    rem += GK;
    if (x.n0 && rem == x.n0) {
      rem = 0;
      base += x.s1 - int64_t(x.n0 - GK) * x.s0;
    } else {
      base += GK * x.s0;
    }
  };
  auto load = [&](int k0) {
    if (a_kfast) {
      const int gk = k0 + t % GK;
      const int64_t ko = gk < K ? koff(k0, t % GK, A.c, a_base) : 0;
#pragma unroll
      for (int i = 0; i < NA; ++i) ra[i] = (gk < K && (a_ok >> i & 1)) ? Ap[a_fixed[i] + ko] : 0.0;
    } else {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int dk = t / TM + SA * i, gk = k0 + dk;
        ra[i] = (gk < K && a_ok) ? Ap[a_fixed[0] + koff(k0, dk, A.c, a_base)] : 0.0;
      }
    }
    if (b_kfast) {
      const int gk = k0 + t % GK;
      const int64_t ko = gk < K ? koff(k0, t % GK, B.r, b_base) : 0;
#pragma unroll
      for (int i = 0; i < NB; ++i) rb[i] = (gk < K && (b_ok >> i & 1)) ? Bp[b_fixed[i] + ko] : 0.0;
    } else {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        const int dk = t / TN + SB * i, gk = k0 + dk;
        rb[i] = (gk < K && b_ok) ? Bp[b_fixed[0] + koff(k0, dk, B.r, b_base)] : 0.0;
      }
    }
    if (fastk) {
      step(A.c, a_base, a_rem);
      step(B.r, b_base, b_rem);
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (a_kfast) As[t % GK][t / GK + 16 * i] = ra[i];
      else As[t / TM + SA * i][t % TM] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (b_kfast) Bs[t % GK][t / GK + 16 * i] = rb[i];
      else Bs[t / TN + SB * i][t % TN] = rb[i];
    }
  };
  v4d acc[BM][BN];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  const int li = lane & 15, lk = lane >> 4;
  load(0);
  for (int k0 = 0; k0 < K; k0 += GK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + GK < K) load(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      double a[BM], bv[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) a[i] = As[kk + lk][wm * 16 * BM + i * 16 + li];
#pragma unroll
      for (int j = 0; j < BN; ++j) bv[j] = Bs[kk + lk][wn * 16 * BN + j * 16 + li];
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }
  double* Cb = C + b * cbs;
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int gn = tn0 + wn * 16 * BN + j * 16 + li;
      if (gn >= N) continue;
      const int64_t on = ix_off(uint32_t(gn), cc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = tm0 + wm * 16 * BM + i * 16 + 4 * v + lk;
        if (gm >= M) continue;
        double* dst = Cb + ix_off(uint32_t(gm), cr) + on;
        const double r = alpha * acc[i][j][v];
        *dst = beta == 0.0 ? r : r + beta * *dst;
      }
    }
}

static bool kfast(const Ix& k, const Ix& other) {
  // stage along k when k is the unit-stride index of the operand
  const int64_t sk = k.s0 < 0 ? -k.s0 : k.s0, so = other.s0 < 0 ? -other.s0 : other.s0;
  return sk <= so;
}

template <int TAG, int KF>
static void gemm_launch_kf(int v, dim3 grid, hipStream_t s, int M, int N, int K, const Operand& a, const Operand& b,
                           double* C, Ix cr, Ix cc, int64_t cbs, double alpha, double beta) {
  if (v == 1)
    hipLaunchKernelGGL((gemm_mfma_kernel<TAG, 4, 4, KF>), grid, dim3(256), 0, s, M, N, K, a, b, C, cr, cc, cbs, alpha,
                       beta, (N + 127) / 128);
  else if (v == 2)
    hipLaunchKernelGGL((gemm_mfma_kernel<TAG, 2, 2, KF>), grid, dim3(256), 0, s, M, N, K, a, b, C, cr, cc, cbs, alpha,
                       beta, (N + 63) / 64);
  else
    hipLaunchKernelGGL((gemm_mfma_kernel<TAG, 4, 2, KF>), grid, dim3(256), 0, s, M, N, K, a, b, C, cr, cc, cbs, alpha,
                       beta, (N + 63) / 64);
}

template <int TAG>
static void gemm_launch(int v, dim3 grid, hipStream_t s, int M, int N, int K, const Operand& a, const Operand& b,
                        double* C, Ix cr, Ix cc, int64_t cbs, double alpha, double beta, int akf, int bkf, int fastk) {
  switch (akf | bkf << 1 | fastk << 2) {
#define TNB_GEMM_KF(kf) \
    case kf: gemm_launch_kf<TAG, kf>(v, grid, s, M, N, K, a, b, C, cr, cc, cbs, alpha, beta); break;
    TNB_GEMM_KF(0) TNB_GEMM_KF(1) TNB_GEMM_KF(2) TNB_GEMM_KF(3)
    TNB_GEMM_KF(4) TNB_GEMM_KF(5) TNB_GEMM_KF(6) TNB_GEMM_KF(7)
#undef TNB_GEMM_KF
  }
}

void gemm_mfma(int batch, int M, int N, int K, const Operand& A, const Operand& B, double* C, Ix cr, Ix cc,
               int64_t cbs, double alpha, double beta, hipStream_t s, const char* timer, int tag) {
  if (batch <= 0 || M <= 0 || N <= 0) return;
  static const int TMv[3] = {128, 128, 64}, TNv[3] = {64, 128, 64};
  for (int v = 0; v < 3; ++v) {
    const int64_t tiles = int64_t((M + TMv[v] - 1) / TMv[v]) * ((N + TNv[v] - 1) / TNv[v]);
    if (tiles > 0x7fffffff) fail(TNB_EUNSUPPORTED, "GEMM too large");
  }
  KTimer _t(timer, s, 2.0 * M * double(N) * double(K) * batch,
            8.0 * (double(M) * K + double(K) * N + double(M) * N) * batch);
  const int akf = kfast(A.c, A.r) ? 1 : 0, bkf = kfast(B.r, B.c) ? 1 : 0;
  const int fastk = (A.c.n0 % GK == 0 && B.r.n0 % GK == 0) ? 1 : 0;  // n0 == 0 passes too
  auto run = [&](int v) {
    const int64_t tiles = int64_t((M + TMv[v] - 1) / TMv[v]) * ((N + TNv[v] - 1) / TNv[v]);
    for (int b0 = 0; b0 < batch; b0 += 65535) {
      const int nb = batch - b0 < 65535 ? batch - b0 : 65535;
      Operand a = A, bb = B;
      a.p += A.bs * b0;
      bb.p += B.bs * b0;
      const dim3 grid{unsigned(tiles), unsigned(nb), 1u};
      switch (tag) {
        case 1: gemm_launch<1>(v, grid, s, M, N, K, a, bb, C + cbs * b0, cr, cc, cbs, alpha, beta, akf, bkf, fastk); break;
        case 2: gemm_launch<2>(v, grid, s, M, N, K, a, bb, C + cbs * b0, cr, cc, cbs, alpha, beta, akf, bkf, fastk); break;
        case 3: gemm_launch<3>(v, grid, s, M, N, K, a, bb, C + cbs * b0, cr, cc, cbs, alpha, beta, akf, bkf, fastk); break;
        case 4: gemm_launch<4>(v, grid, s, M, N, K, a, bb, C + cbs * b0, cr, cc, cbs, alpha, beta, akf, bkf, fastk); break;
        case 5: gemm_launch<5>(v, grid, s, M, N, K, a, bb, C + cbs * b0, cr, cc, cbs, alpha, beta, akf, bkf, fastk); break;
        default: gemm_launch<0>(v, grid, s, M, N, K, a, bb, C + cbs * b0, cr, cc, cbs, alpha, beta, akf, bkf, fastk);
      }
    }
    HIPC(hipGetLastError());
  };
  if (beta != 0.0) {  // an accumulating product runs once: no timing trials
    run(0);
    return;
  }
  char key[200];
  std::snprintf(key, sizeof key, "gemm t%d M%d N%d K%d b%d ak%d bk%d", tag, M, N, K, batch, akf, bkf);
  autotune_pick(key, 3, run, s);
}

}  // namespace la
}  // namespace tnb
