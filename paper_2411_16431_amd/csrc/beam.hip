// Branch and bound over cluster variables (Sec. III.A) driven by the
// conditional marginals of the boundary-MPS network (Fig. 6b).
//
// Row r uses Psi_{r+1}.  At the start of a row every parent b gets right
// environments R_b^{(c)}[beta][pi_c] (the contraction of the unfixed
// clusters right of c with their couplings to b's fixed row r-1), built right
// to left in four factorised passes:
//   u[b][x][g]        = A_{2c}[v'(x)] R^{(c)}[:, pi_c(x)]
//   U[b][xh][b'][g]   = sum_{x in (xh, b')} w(x) phi_b(x) u[b][x][g]
//   V[b][xh][a'][be]  = sum_{b', g} U[b][xh][b'][g] A_{2c-1}[a' + da' b'][be][g]   (MFMA GEMM)
//   R^{(c-1)}[b][be][pi] = sum_xh W_h(h(pi), xh) V[b][xh][a'(pi)][be]
// The marginal of (r, c) is then q_b[x] = w phi_b W_h(x_{c-1}^b, x)
// (L_b A_{2c-1}[..] A_{2c}[v'(x)]) . R_b^{(c)}[:, pi_c(x)].
// Candidates are reduced exactly: within a parent, x values that agree on the
// spins facing unfixed clusters share the boundary and only the best is kept;
// across parents, boundaries are equal iff the parents' boundary words are
// equal (class id) and the reduced x agree.  Ordering uses a bitonic sort of
// (boundary key, -score, parent, x): deterministic, no atomics.
#include <cstdio>
#include <cstdlib>
#include <memory>

#include "beam.h"

namespace tnb {


__device__ inline bool cand_less(const Cand& a, const Cand& b) {
  if (a.gkey != b.gkey) return a.gkey < b.gkey;
  if (a.skey != b.skey) return a.skey < b.skey;
  if (a.b != b.b) return a.b < b.b;
  return a.x < b.x;
}

__global__ void bitonic_step(Cand* __restrict__ a, int64_t n, int64_t j, int64_t k) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t l = i ^ j;
  if (l > i) {
    const bool up = (i & k) == 0;
    Cand x = a[i], y = a[l];
    if (up ? cand_less(y, x) : cand_less(x, y)) {
      a[i] = y;
      a[l] = x;
    }
  }
}


// All stages with j < kChunk run inside one workgroup on a kChunk-element
// slice held in LDS: the first kernel performs every stage of k <= kChunk,
// the second the j < kChunk stages of one larger k.  The compare-exchange
// network is the same as the one-launch-per-stage version, so the result is
// identical.
constexpr int kChunk = 2048;

__global__ void __launch_bounds__(1024) bitonic_local(Cand* __restrict__ a, int64_t n, int64_t kfix) {
  __shared__ Cand sh[kChunk];
  const int64_t base = int64_t(blockIdx.x) * kChunk;
  for (int i = threadIdx.x; i < kChunk; i += blockDim.x) sh[i] = a[base + i];
  __syncthreads();
  const int64_t k0 = kfix ? kfix : 2, k1 = kfix ? kfix : kChunk;
  for (int64_t k = k0; k <= k1; k <<= 1) {
    for (int64_t j = (kfix ? kChunk : k) >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < kChunk / 2; t += blockDim.x) {
        const int i = int(2 * j * (t / j) + (t % j));  // lower element of the pair
        const int l = i + int(j);
        const bool up = ((base + i) & k) == 0;
        const Cand x = sh[i], y = sh[l];
        if (up ? cand_less(y, x) : cand_less(x, y)) {
          sh[i] = y;
          sh[l] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < kChunk; i += blockDim.x) a[base + i] = sh[i];
  (void)n;
}

// A whole sort of n <= kChunk elements (a power of two) in one workgroup:
// the network of bitonic_step, stage after stage, on an LDS copy.
__global__ void __launch_bounds__(1024) bitonic_small(Cand* __restrict__ a, int n) {
  __shared__ Cand sh[kChunk];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sh[i] = a[i];
  __syncthreads();
  for (int k = 2; k <= n; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
        const int i = 2 * j * (t / j) + (t % j);
        const int l = i + j;
        const bool up = (i & k) == 0;
        const Cand x = sh[i], y = sh[l];
        if (up ? cand_less(y, x) : cand_less(x, y)) {
          sh[i] = y;
          sh[l] = x;
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = sh[i];
}

void bitonic_sort(Cand* a, int64_t npow2, hipStream_t st) {
  int lg = 0;
  while ((int64_t(1) << lg) < npow2) ++lg;
  KTimer _t("sort", st, 0.0, 2.0 * sizeof(Cand) * double(npow2) * lg * (lg + 1) / 2);
  if (npow2 <= kChunk) {
    if (npow2 > 1) hipLaunchKernelGGL(bitonic_small, dim3(1), dim3(1024), 0, st, a, int(npow2));
    HIPC(hipGetLastError());
    return;
  }
  const unsigned nchunk = unsigned(npow2 / kChunk);
  hipLaunchKernelGGL(bitonic_local, dim3(nchunk), dim3(1024), 0, st, a, npow2, int64_t(0));
  for (int64_t k = 2 * kChunk; k <= npow2; k <<= 1) {
    for (int64_t j = k >> 1; j >= kChunk; j >>= 1)
      hipLaunchKernelGGL(bitonic_step, dim3(nblk(npow2)), dim3(256), 0, st, a, npow2, j, k);
    hipLaunchKernelGGL(bitonic_local, dim3(nchunk), dim3(1024), 0, st, a, npow2, k);
  }
  HIPC(hipGetLastError());
}


// u[b][x][g] = sum_d A2c[vd(x)][g][d] * R[b][d][pi(x)]
__global__ void renv_u_kernel(BCol c, const double* __restrict__ A2c, int Dl, int Dr,
                              const double* __restrict__ R, int nb, double* __restrict__ u) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t d = int64_t(1) << c.k;
  if (idx >= int64_t(nb) * d * Dl) return;
  const int b = int(idx / (d * Dl));
  const uint32_t x = uint32_t((idx / Dl) % d);
  const int g = int(idx % Dl);
  const double* Av = A2c + size_t(pext_dev(x, c.Bvd)) * Dl * Dr + size_t(g) * Dr;
  const double* Rb = R + size_t(b) * Dr * c.dpi;
  const uint32_t pi = pext_dev(x, c.PRR);
  double acc = 0.0;
  for (int e = 0; e < Dr; ++e) acc = fma(Av[e], Rb[size_t(e) * c.dpi + pi], acc);
  u[idx] = acc;
}

// U[b][xh][bd][g] = sum over x in the class of (xh, bd) of w phi u[b][x][g]
__global__ void renv_U_kernel(BCol c, const int32_t* __restrict__ X, int ncell, const double* __restrict__ u,
                              int nb, int Dl, double* __restrict__ U) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(c.dxh) * c.dbd * Dl;
  if (idx >= nb * per) return;
  const int b = int(idx / per);
  const uint32_t xh = uint32_t((idx / (int64_t(c.dbd) * Dl)) % c.dxh);
  const uint32_t bd = uint32_t((idx / Dl) % c.dbd);
  const int g = int(idx % Dl);
  const uint32_t full = c.k ? ((1u << c.k) - 1u) : 0u;
  const uint32_t hx = pdep_dev(xh, c.Bxh), bx = pdep_dev(bd, c.Bbd);
  double acc = 0.0;
  if ((hx & c.Bbd) == (bx & c.Bxh)) {
    const uint32_t base = hx | bx;
    const uint32_t FREE = full & ~(c.Bxh | c.Bbd);
    const int nf = 1 << __builtin_popcount(FREE);
    const int32_t* Xb = X + size_t(b) * ncell;
    const int64_t d = int64_t(1) << c.k;
    for (int f = 0; f < nf; ++f) {
      const uint32_t x = base | pdep_dev(uint32_t(f), FREE);
      acc = fma(wloc(c, x) * phi_of(c, Xb, x), u[(size_t(b) * d + x) * Dl + g], acc);
    }
  }
  U[idx] = acc;
}

// R[b][be][pi] = sum_xh Wh(h(pi), xh) V[b][xh][a(pi)][be]   (pi over PRR_{c-1})
__global__ void renv_R_kernel(BCol c, int dpi_prev, const double* __restrict__ V, int nb, int Dl,
                              double* __restrict__ R) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(Dl) * dpi_prev;
  if (idx >= nb * per) return;
  const int b = int(idx / per);
  const int be = int((idx / dpi_prev) % Dl);
  const uint32_t pi = uint32_t(idx % dpi_prev);
  const uint32_t h = pext_dev(pi, c.pos_h), a2 = pext_dev(pi, c.pos_a);
  double acc = 0.0;
  for (int xh = 0; xh < c.dxh; ++xh)
    acc = fma(c.Wh[h * c.Wh_sp + xh * c.Wh_sq], V[((size_t(b) * c.dxh + xh) * c.da2 + a2) * Dl + be], acc);
  R[idx] = acc;
}

__global__ void normalise_rows_kernel(double* __restrict__ R, int64_t per, int nb, double* __restrict__ logs) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < per; i += blockDim.x) m = fmax(m, fabs(R[b * per + i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double s = red[0] > 0.0 ? 1.0 / red[0] : 1.0;
  for (int64_t i = threadIdx.x; i < per; i += blockDim.x) R[b * per + i] *= s;
  if (logs && threadIdx.x == 0 && red[0] > 0.0) logs[b] += log(red[0]);
}

// T[b][bd][m] = sum_a L[b][a] A[afix(b) + da2*bd][a][m]
__global__ void beam_T_kernel(BCol c, uint32_t Bleft_a, int left_cell, const int32_t* __restrict__ X,
                              int ncell, const double* __restrict__ L, int Ld, const double* __restrict__ A,
                              int Dl, int Dr, int nb, double* __restrict__ T) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(c.dbd) * Dr;
  if (idx >= nb * per) return;
  const int b = int(idx / per);
  const int bd = int((idx / Dr) % c.dbd);
  const int m = int(idx % Dr);
  const uint32_t af = pext_dev(uint32_t(X[size_t(b) * ncell + left_cell]), Bleft_a);
  const double* Ab = A + size_t(af + c.da2 * bd) * Dl * Dr;
  double acc = 0.0;
  for (int a = 0; a < Dl; ++a) acc = fma(L[size_t(b) * Ld + a], Ab[size_t(a) * Dr + m], acc);
  T[idx] = acc;
}

// q[b][x]; T: [b][bd][m] (m over the left bond of A2c), R per ancestor
__global__ void beam_q_kernel(BCol c, int has_left, int left_cell, const int32_t* __restrict__ X,
                              int ncell, const double* __restrict__ T, const double* __restrict__ A2c,
                              int Dl, int Dr, const double* __restrict__ R, const int32_t* __restrict__ rid,
                              int nb, double* __restrict__ q) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t d = int64_t(1) << c.k;
  if (idx >= nb * d) return;
  const int b = int(idx / d);
  const uint32_t x = uint32_t(idx % d);
  const int32_t* Xb = X + size_t(b) * ncell;
  double g = wloc(c, x) * phi_of(c, Xb, x);
  if (has_left)
    g *= c.Wh[pext_dev(uint32_t(Xb[left_cell]), c.Bleft_h) * c.Wh_sp + pext_dev(x, c.Bxh) * c.Wh_sq];
  const double* Tb = T + (size_t(b) * c.dbd + pext_dev(x, c.Bbd)) * Dl;
  const double* Av = A2c + size_t(pext_dev(x, c.Bvd)) * Dl * Dr;
  const double* Rb = R + size_t(rid[b]) * Dr * c.dpi;
  const uint32_t pi = pext_dev(x, c.PRR);
  double acc = 0.0;
  for (int e = 0; e < Dr; ++e) {
    double v = 0.0;
    for (int m = 0; m < Dl; ++m) v = fma(Tb[m], Av[size_t(m) * Dr + e], v);
    acc = fma(v, Rb[size_t(e) * c.dpi + pi], acc);
  }
  q[idx] = g * acc;
}

// per parent: the marginal is a ratio of contractions of one network, so the
// common sign of the approximate environment cancels: sg = sign(sum q),
// Z_b = sum of the positive entries of sg*q, score = logp_b + log(sg*q) - log Z_b
// (entries with sg*q <= 0 get probability 0 and score -inf).
__global__ void beam_score_kernel(const double* __restrict__ q, int64_t d, const double* __restrict__ logp,
                                  double* __restrict__ score, double* __restrict__ prob, int* __restrict__ dead) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += blockDim.x) acc += q[b * d + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double sg = red[0] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  acc = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
    const double v = sg * q[b * d + i];
    acc += v > 0.0 ? v : 0.0;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double Z = red[0];
  const bool alive = Z > 0.0 && isfinite(Z);
  if (threadIdx.x == 0 && !alive) dead[0] = 1;
  const double lZ = alive ? log(Z) : 0.0;
  for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
    const double v = sg * q[b * d + i];
    const bool ok = alive && v > 0.0;
    if (score) score[b * d + i] = ok ? logp[b] + (log(v) - lZ) : -INFINITY;
    if (prob) prob[b * d + i] = ok ? v / Z : 0.0;
  }
}

// packed boundary words of each parent (fixed cells other than the new one)
__global__ void parent_words_kernel(const int32_t* __restrict__ X, int ncell, int nb, const int* __restrict__ kc,
                                    const uint32_t* __restrict__ km, int nk, int W, uint32_t* __restrict__ words) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  uint32_t* wb = words + size_t(b) * W;
  for (int i = 0; i < W; ++i) wb[i] = 0u;
  int pos = 0;
  for (int i = 0; i < nk; ++i) {
    const uint32_t v = pext_dev(uint32_t(X[size_t(b) * ncell + kc[i]]), km[i]);
    const int nbits = __builtin_popcount(km[i]);
    for (int t = 0; t < nbits; ++t, ++pos)
      if ((v >> t) & 1u) wb[pos >> 5] |= 1u << (pos & 31);
  }
}

__global__ void parent_class_kernel(const uint32_t* __restrict__ words, int nb, int W, uint32_t* __restrict__ cls) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  uint32_t c = uint32_t(b);
  for (int o = 0; o < b; ++o) {
    bool eq = true;
    for (int i = 0; i < W && eq; ++i) eq = words[size_t(o) * W + i] == words[size_t(b) * W + i];
    if (eq) { c = uint32_t(o); break; }
  }
  cls[b] = c;
}

// best candidate of every (parent, boundary bits of x); sentinel when none
__global__ void group_kernel(const double* __restrict__ score, int k, uint32_t Un, int nb,
                             const uint32_t* __restrict__ cls, int merge, Cand* __restrict__ out, int64_t nout) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nout) return;
  Cand cnd{~0ull, ~0ull, ~0u, ~0u};
  const int64_t d = int64_t(1) << k;
  if (merge) {
    const int64_t dg = int64_t(1) << __builtin_popcount(Un);
    if (idx < nb * dg) {
      const int b = int(idx / dg);
      const uint32_t xk = uint32_t(idx % dg);
      const uint32_t full = k ? ((1u << k) - 1u) : 0u;
      const uint32_t FREE = full & ~Un;
      const int nf = 1 << __builtin_popcount(FREE);
      const uint32_t base = pdep_dev(xk, Un);
      double best = -INFINITY;
      uint32_t bx = 0;
      for (int f = 0; f < nf; ++f) {
        const uint32_t x = base | pdep_dev(uint32_t(f), FREE);
        const double s = score[b * d + x];
        if (s > best || (s == best && x < bx)) { best = s; bx = x; }
      }
      if (best > -INFINITY) cnd = Cand{uint64_t(cls[b]) * uint64_t(dg) + xk, score_key(best), uint32_t(b), bx};
    }
  } else if (idx < nb * d) {
    const double s = score[idx];
    // no merge (empty boundary): every candidate is its own group
    if (s > -INFINITY) cnd = Cand{uint64_t(idx), score_key(s), uint32_t(idx / d), uint32_t(idx % d)};
  }
  out[idx] = cnd;
}

__global__ void winner_flag_kernel(const Cand* __restrict__ a, int64_t n, int* __restrict__ flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool valid = a[i].gkey != ~0ull;
  flag[i] = (valid && (i == 0 || a[i].gkey != a[i - 1].gkey)) ? 1 : 0;
}

// exclusive scan of flags in one block (n up to a few million: chunked loop)
// Exclusive scan of 0/1 flags in three launches: tile sums (tiles of
// kScanTile flags, read coalesced), a scan of the tile sums in one
// workgroup, then each tile's scan with its offset.  Integer arithmetic, so
// the result does not depend on the decomposition.
constexpr int kScanTile = 4096;

__global__ void __launch_bounds__(256) scan_tiles_kernel(const int* __restrict__ flag, int64_t n,
                                                         int64_t* __restrict__ tsum) {
  __shared__ int64_t red[256];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t s = 0;
  for (int i = threadIdx.x; i < kScanTile; i += 256)
    if (base + i < n) s += flag[base + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) tsum[blockIdx.x] = red[0];
}

__global__ void scan_kernel(const int64_t* __restrict__ x, int64_t n, int64_t* __restrict__ pos,
                            int64_t* __restrict__ total) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int64_t chunk = (n + nt - 1) / nt;
  const int64_t lo = t * chunk, hi = lo + chunk < n ? lo + chunk : n;
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += x[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int i = 0; i < nt; ++i) { int64_t v = part[i]; part[i] = acc; acc += v; }
    *total = acc;
  }
  __syncthreads();
  int64_t acc = part[t];
  for (int64_t i = lo; i < hi; ++i) { pos[i] = acc; acc += x[i]; }
}

// pos[i] = toff[tile] + (flags before i within its tile); 16 flags per thread
__global__ void __launch_bounds__(256) scan_apply_kernel(const int* __restrict__ flag, int64_t n,
                                                         const int64_t* __restrict__ toff,
                                                         int64_t* __restrict__ pos) {
  __shared__ int64_t part[256];
  constexpr int per = kScanTile / 256;
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * per;
  int v[per];
  int64_t s = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    v[q] = base + q < n ? flag[base + q] : 0;
    s += v[q];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  // inclusive Hillis-Steele scan of the 256 thread sums
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t add = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t acc = toff[blockIdx.x] + part[threadIdx.x] - s;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    if (base + q < n) pos[base + q] = acc;
    acc += v[q];
  }
}

__global__ void compact_kernel(const Cand* __restrict__ a, const int* __restrict__ flag, const int64_t* __restrict__ pos,
                               int64_t n, Cand* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  Cand c = a[i];
  c.gkey = 0ull;
  out[pos[i]] = c;
}

__global__ void fill_cand_kernel(Cand* __restrict__ a, int64_t lo, int64_t hi) {
  const int64_t i = lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < hi) a[i] = Cand{~0ull, ~0ull, ~0u, ~0u};
}

// new beam entries from the selected candidates
__global__ void new_beam_kernel(const Cand* __restrict__ sel, int nsel, const int32_t* __restrict__ X, int ncell,
                                int cell, const int32_t* __restrict__ rid, int32_t* __restrict__ Xn,
                                double* __restrict__ logpn, int32_t* __restrict__ ridn) {
  const int i = blockIdx.x;
  if (i >= nsel) return;
  const Cand c = sel[i];
  for (int n = threadIdx.x; n < ncell; n += blockDim.x)
    Xn[size_t(i) * ncell + n] = n == cell ? int32_t(c.x) : X[size_t(c.b) * ncell + n];
  if (threadIdx.x == 0) {
    logpn[i] = key_score(c.skey);
    ridn[i] = rid[c.b];
  }
}

// L'[i][e] = sum_m T[b][bd(x)][m] A2c[vd(x)][m][e], then max-normalised
__global__ void new_left_kernel(BCol c, const Cand* __restrict__ sel, int nsel, const double* __restrict__ T,
                                const double* __restrict__ A2c, int Dl, int Dr, double* __restrict__ Ln) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const Cand cd = sel[i];
  const double* Tb = T + (size_t(cd.b) * c.dbd + pext_dev(cd.x, c.Bbd)) * Dl;
  const double* Av = A2c + size_t(pext_dev(cd.x, c.Bvd)) * Dl * Dr;
  double mx = 0.0;
  for (int e = threadIdx.x; e < Dr; e += blockDim.x) {
    double v = 0.0;
    for (int m = 0; m < Dl; ++m) v = fma(Tb[m], Av[size_t(m) * Dr + e], v);
    Ln[size_t(i) * Dr + e] = v;
    mx = fmax(mx, fabs(v));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double s = red[0] > 0.0 ? 1.0 / red[0] : 1.0;
  for (int e = threadIdx.x; e < Dr; e += blockDim.x) Ln[size_t(i) * Dr + e] *= s;
}

__global__ void export_kernel(const int32_t* __restrict__ X, int ncell, int nfixed, const int32_t* __restrict__ cell_of,
                              const int32_t* __restrict__ bit, int N, int K, int8_t* __restrict__ out,
                              const double* __restrict__ logp, double* __restrict__ lp_out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(K) * N) return;
  const int i = int(idx / N), j = int(idx % N);
  const int n = cell_of[j];
  int8_t v = 0;
  if (n < nfixed) v = ((X[size_t(i) * ncell + n] >> bit[j]) & 1) ? int8_t(1) : int8_t(-1);
  out[idx] = v;
  if (lp_out && j == 0) lp_out[i] = logp[i];
}

// <s_i>_b = sum_x p_b(x) s_i(x) for bit i of the cluster (blockIdx.y), parent
// b = blockIdx.x; s_i(x) = +1 when bit i of x is set.
__global__ void spin_moment_kernel(const double* __restrict__ P, int64_t d, int k, double* __restrict__ out) {
  __shared__ double red[256];
  const int b = blockIdx.x, i = blockIdx.y;
  double acc = 0.0;
  for (int64_t x = threadIdx.x; x < d; x += blockDim.x) {
    const double p = P[b * d + x];
    acc += ((x >> i) & 1) ? p : -p;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[int64_t(b) * k + i] = red[0];
}

// Final selection (the K lowest distinct states).  Candidate j precedes i
// when its energy is lower, or equal with a spin vector that is smaller
// lexicographically (spin 0 first, -1 < +1).
__device__ inline bool sel_less(const int8_t* __restrict__ S, const double* __restrict__ E, int N, int j, int i) {
  if (E[j] != E[i]) return E[j] < E[i];
  const int8_t* a = S + int64_t(j) * N;
  const int8_t* b = S + int64_t(i) * N;
  for (int q = 0; q < N; ++q)
    if (a[q] != b[q]) return a[q] < b[q];
  return false;
}

// dup[i] = 1 when an earlier candidate holds the same spin vector (one
// workgroup per candidate).
__global__ void sel_dup_kernel(const int8_t* __restrict__ S, const double* __restrict__ E, int n, int N,
                               int* __restrict__ dup) {
  __shared__ int found;
  const int i = blockIdx.x;
  if (threadIdx.x == 0) found = 0;
  __syncthreads();
  const int8_t* b = S + int64_t(i) * N;
  for (int j = threadIdx.x; j < i; j += blockDim.x) {
    if (E[j] != E[i]) continue;
    const int8_t* a = S + int64_t(j) * N;
    bool same = true;
    for (int q = 0; q < N && same; ++q) same = a[q] == b[q];
    if (same) found = 1;  // every writer stores the same value
  }
  __syncthreads();
  if (threadIdx.x == 0) dup[i] = found;
}

// Rank of every distinct candidate among the distinct ones; the first K go
// to the output in rank order (one workgroup per candidate).
__global__ void sel_rank_kernel(const int8_t* __restrict__ S, const double* __restrict__ E,
                                const int* __restrict__ dup, int n, int N, int K, int8_t* __restrict__ out_S,
                                double* __restrict__ out_E) {
  __shared__ int cnt[256];
  const int i = blockIdx.x;
  if (dup[i]) return;  // uniform over the workgroup
  int c = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) c += (!dup[j] && sel_less(S, E, N, j, i)) ? 1 : 0;
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) cnt[threadIdx.x] += cnt[threadIdx.x + w];
    __syncthreads();
  }
  const int r = cnt[0];
  if (r >= K) return;
  for (int q = threadIdx.x; q < N; q += blockDim.x) out_S[int64_t(r) * N + q] = S[int64_t(i) * N + q];
  if (threadIdx.x == 0) out_E[r] = E[i];
}

__global__ void fill_d(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void fill_i(int32_t* __restrict__ x, int64_t n, int32_t v, int iota) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = iota ? int32_t(i) : v;
}

}  // namespace tnb

using namespace tnb;


namespace tnb {

void ensure(DevBuf<double>& b, size_t n) { if (b.n < n) b.alloc(n + n / 4 + 16); }

std::vector<BCol> beam_geom(const tnb_clusters* cl, int r) {
  const Lattice& L = cl->lat;
  std::vector<BCol> g(L.C);
  const double* ones = unit_weight();
  for (int c = 0; c < L.C; ++c) {
    BCol& b = g[c];
    b.n = L.cell(r, c);
    b.k = L.k[b.n];
    b.PRR = cl->B(b.n, L.cell(r, c + 1)) | cl->B(b.n, L.cell(r + 1, c + 1));
    b.dpi = 1 << popcount32(b.PRR);
    b.Bvd = cl->B(b.n, L.cell(r + 1, c));
    b.dvd = 1 << popcount32(b.Bvd);
    b.w = cl->w_loc.p + cl->loc_off[b.n];
    for (int dc = -1; dc <= 1; ++dc) {
      int up = L.cell(r - 1, c + dc);
      if (up < 0 || cl->B(b.n, up) == 0) continue;
      UpNb& u = b.up[b.nup++];
      u.cell = up;
      u.Bup_in_up = cl->B(up, b.n);
      u.Bn = cl->B(b.n, up);
      if (!cl->weight_view(up, b.n, &u.W, &u.sp, &u.sq)) fail(TNB_EDEVICE, "missing bond table");
    }
    if (c > 0) {
      int left = L.cell(r, c - 1);
      b.Bxh = cl->B(b.n, left);
      b.dxh = 1 << popcount32(b.Bxh);
      b.Bbd = cl->B(b.n, L.cell(r + 1, c - 1));
      b.dbd = 1 << popcount32(b.Bbd);
      uint32_t la = cl->B(left, L.cell(r + 1, c));
      b.da2 = 1 << popcount32(la);
      const BCol& p = g[c - 1];
      b.pos_h = pext_host(cl->B(left, b.n), p.PRR);
      b.pos_a = pext_host(la, p.PRR);
      b.Bleft_h = cl->B(left, b.n);
      if (!cl->weight_view(left, b.n, &b.Wh, &b.Wh_sp, &b.Wh_sq)) { b.Wh = ones; b.Wh_sp = 0; b.Wh_sq = 0; }
    } else {
      b.Wh = ones;
    }
  }
  return g;
}

void row_step(tnb_beam* bm, const BCol& cc, int c, int nb, const double* Rin, double* Rout, double* logs,
              hipStream_t st) {
  const int r = bm->geo_row;
  const Mps& psi = bm->env->psi[r + 1];
  const Site& A2c = psi.sites[2 * c];
  const Site& A2m = psi.sites[2 * c - 1];
  const int64_t d = int64_t(1) << cc.k;
  ensure(bm->u, size_t(nb) * d * A2c.dl);
  {
  KTimer _tu("renv_u", st, 2.0 * nb * double(d) * A2c.dl * A2c.dr, 8.0 * (double(nb) * d * A2c.dl + A2c.size()));
  hipLaunchKernelGGL(renv_u_kernel, dim3(nblk(int64_t(nb) * d * A2c.dl)), dim3(256), 0, st, cc, A2c.data.p,
                     A2c.dl, A2c.dr, Rin, nb, bm->u.p);
  }
  ensure(bm->U, size_t(nb) * cc.dxh * cc.dbd * A2c.dl);
  {
  KTimer _tU("renv_U", st, 2.0 * nb * double(d) * A2c.dl, 8.0 * (double(nb) * d * A2c.dl));
  hipLaunchKernelGGL(renv_U_kernel, dim3(nblk(int64_t(nb) * cc.dxh * cc.dbd * A2c.dl)), dim3(256), 0, st, cc,
                     bm->X.p, bm->ncell, bm->u.p, nb, A2c.dl, bm->U.p);
  }
  ensure(bm->V, size_t(nb) * cc.da2 * cc.dxh * A2m.dl);
  {
    // V[b][xh][a2][be] = sum_{bd, g} U[b][xh][bd][g] A[a2 + da2 bd][be][g]: rows (b, xh),
    // columns (a2, be), reduction (bd, g) -- one GEMM on the matrix cores
    const int Dl = A2m.dl, Dr = A2m.dr;
    la::Operand Uop{bm->U.p, 0, la::Ix{0, 0, int64_t(cc.dbd) * Dr}, la::Ix{0, 0, 1}};
    la::Operand Aop{A2m.data.p, 0, la::Ix{uint32_t(Dr), int64_t(cc.da2) * Dl * Dr, 1}, la::Ix{0, 0, Dr}};
    const int N = cc.da2 * Dl;
    la::gemm_mfma(1, nb * cc.dxh, N, cc.dbd * Dr, Uop, Aop, bm->V.p, la::Ix{0, 0, N}, la::Ix{0, 0, 1}, 0, 1.0, 0.0,
                  st, "renv_V");
  }
  const int dpi_prev = bm->geo[c - 1].dpi;
  {
  KTimer _tR("renv_R", st, 2.0 * nb * double(A2m.dl) * dpi_prev * cc.dxh,
             8.0 * (double(nb) * cc.da2 * cc.dxh * A2m.dl + double(nb) * A2m.dl * dpi_prev));
  hipLaunchKernelGGL(renv_R_kernel, dim3(nblk(int64_t(nb) * A2m.dl * dpi_prev)), dim3(256), 0, st, cc, dpi_prev,
                     bm->V.p, nb, A2m.dl, Rout);
  }
  hipLaunchKernelGGL(normalise_rows_kernel, dim3(nb), dim3(256), 0, st, Rout, int64_t(A2m.dl) * dpi_prev, nb, logs);
  HIPC(hipGetLastError());
}

void normalise_rows(double* R, int64_t per, int nb, double* logs, hipStream_t st) {
  hipLaunchKernelGGL(normalise_rows_kernel, dim3(nb), dim3(256), 0, st, R, per, nb, logs);
  HIPC(hipGetLastError());
}

// right environments of every current parent for row r
void row_envs(tnb_beam* bm, int r, hipStream_t st) {
  const tnb_clusters* cl = bm->env->cl;
  const Lattice& L = cl->lat;
  const Mps& psi = bm->env->psi[r + 1];
  bm->geo = beam_geom(cl, r);
  bm->geo_row = r;
  const int C = L.C, nb = bm->npar;
  bm->R.clear();
  bm->R.resize(C);
  bm->nanc = nb;
  {
    DevBuf<double>& Rl = bm->R[C - 1];
    Rl.alloc(size_t(nb));
    hipLaunchKernelGGL(fill_d, dim3(nblk(nb)), dim3(256), 0, st, Rl.p, int64_t(nb), 1.0);
  }
  for (int c = C - 1; c >= 1; --c) {
    const Site& A2m = psi.sites[2 * c - 1];
    bm->R[c - 1].alloc(size_t(nb) * A2m.dl * bm->geo[c - 1].dpi);
    row_step(bm, bm->geo[c], c, nb, bm->R[c].p, bm->R[c - 1].p, nullptr, st);
  }
  hipLaunchKernelGGL(fill_i, dim3(nblk(nb)), dim3(256), 0, st, bm->rid.p, int64_t(nb), 0, 1);
  ensure(bm->L, size_t(bm->M) * 1);
  hipLaunchKernelGGL(fill_d, dim3(nblk(nb)), dim3(256), 0, st, bm->L.p, int64_t(nb), 1.0);
  bm->Ld = 1;
}

// q[b][x] for the current step (row environments must be in place)
void compute_q(tnb_beam* bm, hipStream_t st) {
  const tnb_clusters* cl = bm->env->cl;
  const Lattice& L = cl->lat;
  const int r = bm->step / L.C, c = bm->step % L.C;
  if (bm->geo_row != r || c == 0) row_envs(bm, r, st);
  const Mps& psi = bm->env->psi[r + 1];
  const BCol& cc = bm->geo[c];
  const Site& A2c = psi.sites[2 * c];
  const int nb = bm->npar;
  const int64_t d = int64_t(1) << cc.k;
  // T[b][bd][m]
  ensure(bm->T, size_t(nb) * cc.dbd * A2c.dl);
  if (c == 0) {
    hipLaunchKernelGGL(fill_d, dim3(nblk(nb)), dim3(256), 0, st, bm->T.p, int64_t(nb), 1.0);
  } else {
    const Site& A2m = psi.sites[2 * c - 1];
    const int left = L.cell(r, c - 1);
    uint32_t la = cl->B(left, L.cell(r + 1, c));
    hipLaunchKernelGGL(beam_T_kernel, dim3(nblk(int64_t(nb) * cc.dbd * A2m.dr)), dim3(256), 0, st, cc, la, left,
                       bm->X.p, bm->ncell, bm->L.p, bm->Ld, A2m.data.p, A2m.dl, A2m.dr, nb, bm->T.p);
  }
  ensure(bm->q, size_t(nb) * d);
  q_against(bm, cc, bm->R[c].p, bm->rid.p, bm->q.p, st);
}

void q_against(tnb_beam* bm, const BCol& cc, const double* Rc, const int32_t* rid, double* q, hipStream_t st) {
  const tnb_clusters* cl = bm->env->cl;
  const Lattice& L = cl->lat;
  const int r = bm->step / L.C, c = bm->step % L.C;
  const Mps& psi = bm->env->psi[r + 1];
  const Site& A2c = psi.sites[2 * c];
  const int nb = bm->npar;
  const int64_t d = int64_t(1) << cc.k;
  const int left = c > 0 ? L.cell(r, c - 1) : 0;
  {
  KTimer _tq("beam_q", st, double(nb) * d * (2.0 * A2c.dl * A2c.dr + 2.0 * A2c.dr),
             8.0 * (double(nb) * d + A2c.size() + double(bm->nanc) * A2c.dr * cc.dpi + double(nb) * cc.dbd * A2c.dl));
  hipLaunchKernelGGL(beam_q_kernel, dim3(nblk(int64_t(nb) * d)), dim3(256), 0, st, cc, c > 0 ? 1 : 0, left,
                     bm->X.p, bm->ncell, bm->T.p, A2c.data.p, A2c.dl, A2c.dr, Rc, rid, nb, q);
  }
  HIPC(hipGetLastError());
}

}  // namespace tnb

extern "C" tnb_status tnb_beam_create(tnb_env* env, int32_t M, tnb_beam** out) {
  return guarded([&] {
    if (!out) fail(TNB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!env || env->kind != KIND_ENV) fail(TNB_EINVAL, "not an env handle");
    if (M < 1 || M > (1 << 16)) fail(TNB_EINVAL, "M must be in [1, 65536]");
    auto bm = std::make_unique<tnb_beam>();
    bm->env = env;
    bm->M = M;
    const Lattice& L = env->cl->lat;
    bm->ncell = L.cells();
    bm->X.alloc(size_t(M) * bm->ncell);
    bm->Xn.alloc(size_t(M) * bm->ncell);
    bm->rid.alloc(size_t(M));
    bm->ridn.alloc(size_t(M));
    bm->logp.alloc(size_t(M));
    bm->logpn.alloc(size_t(M));
    HIPC(hipMemset(bm->X.p, 0, sizeof(int32_t) * size_t(M) * bm->ncell));
    HIPC(hipMemset(bm->logp.p, 0, sizeof(double) * size_t(M)));
    HIPC(hipMemset(bm->rid.p, 0, sizeof(int32_t) * size_t(M)));
    bm->cell_of.upload(L.cell_of, nullptr);
    std::vector<int32_t> bits(L.bit.begin(), L.bit.end());
    bm->bit.upload(bits, nullptr);
    bm->dead.alloc(1);
    HIPC(hipDeviceSynchronize());
    *out = bm.release();
  });
}

extern "C" tnb_status tnb_beam_info(const tnb_beam* bm, int32_t* step, int32_t* npar, int32_t* d) {
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (step) *step = bm->step;
    if (npar) *npar = bm->npar;
    if (d) *d = bm->step < bm->ncell ? (1 << bm->env->cl->lat.k[bm->step]) : 0;
  });
}

extern "C" tnb_status tnb_row_moments(tnb_beam* bm, double* d_m1, int64_t m1_len, double* d_m2, int64_t m2_len,
                                      tnb_stream stream);

extern "C" tnb_status tnb_marginals(tnb_beam* bm, int32_t mode, double* d_out, int64_t out_len, tnb_stream stream) {
  if (mode == TNB_MARG_ADJOINT) return tnb_row_moments(bm, d_out, out_len, nullptr, 0, stream);
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (mode != TNB_MARG_VECTOR && mode != TNB_MARG_SPIN) fail(TNB_EINVAL, "unknown marginal mode");
    if (bm->step >= bm->ncell) fail(TNB_EINVAL, "every cluster is fixed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int kbits = bm->env->cl->lat.k[bm->step];
    const int64_t d = int64_t(1) << kbits;
    const int64_t need = mode == TNB_MARG_VECTOR ? bm->npar * d : int64_t(bm->npar) * kbits;
    if (!d_out || out_len < need) fail(TNB_EINVAL, "output too small");
    double* P = d_out;
    if (mode == TNB_MARG_SPIN) {
      ensure(bm->U, size_t(bm->npar) * d);  // p_b(x) before the moments
      P = bm->U.p;
    }
    compute_q(bm, st);
    if (std::getenv("TNB_DEBUG")) {
      std::vector<double> hq(std::min<int64_t>(d, 4));
      HIPC(hipMemcpy(hq.data(), bm->q.p, hq.size() * sizeof(double), hipMemcpyDeviceToHost));
      std::fprintf(stderr, "[tnb] step %d q[0][0..] =", bm->step);
      for (double v : hq) std::fprintf(stderr, " %.6e", v);
      std::fprintf(stderr, "\n");
      for (int c = bm->env->cl->lat.C - 1; c >= 0; --c) {
        std::vector<double> hr(std::min<size_t>(bm->R[c].n, 6));
        HIPC(hipMemcpy(hr.data(), bm->R[c].p, hr.size() * sizeof(double), hipMemcpyDeviceToHost));
        std::fprintf(stderr, "[tnb]   R[%d] (%zu entries) head:", c, bm->R[c].n);
        for (double v : hr) std::fprintf(stderr, " %.3e", v);
        std::fprintf(stderr, "\n");
      }
    }
    HIPC(hipMemsetAsync(bm->dead.p, 0, sizeof(int), st));
    hipLaunchKernelGGL(beam_score_kernel, dim3(bm->npar), dim3(256), 0, st, bm->q.p, d, bm->logp.p, nullptr, P,
                       bm->dead.p);
    if (mode == TNB_MARG_SPIN && kbits > 0)
      hipLaunchKernelGGL(spin_moment_kernel, dim3(bm->npar, kbits), dim3(256), 0, st, P, d, kbits, d_out);
    HIPC(hipGetLastError());
    int dead = 0;
    HIPC(hipMemcpyAsync(&dead, bm->dead.p, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    if (dead) fail(TNB_ENUMERIC, "a parent has no positive marginal at step " + std::to_string(bm->step));
  });
}

extern "C" tnb_status tnb_branch_step(tnb_beam* bm, double* p_disc_log, tnb_stream stream) {
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (bm->step >= bm->ncell) fail(TNB_EINVAL, "every cluster is fixed");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const tnb_clusters* cl = bm->env->cl;
    const Lattice& L = cl->lat;
    const int n = bm->step, r = n / L.C, c = n % L.C;
    const int nb = bm->npar;
    const int k = L.k[n];
    const int64_t d = int64_t(1) << k;
    compute_q(bm, st);
    ensure(bm->score, size_t(nb) * d);
    HIPC(hipMemsetAsync(bm->dead.p, 0, sizeof(int), st));
    hipLaunchKernelGGL(beam_score_kernel, dim3(nb), dim3(256), 0, st, bm->q.p, d, bm->logp.p, bm->score.p, nullptr,
                       bm->dead.p);
    // boundary after fixing n: (fixed cell, mask facing unfixed cells)
    uint32_t Un = 0;
    std::vector<int> kcells;
    std::vector<uint32_t> kmasks;
    for (int kk = 0; kk <= n; ++kk) {
      uint32_t U = 0;
      int rr = kk / L.C, ccol = kk % L.C;
      for (int dr = -1; dr <= 1; ++dr)
        for (int dc = -1; dc <= 1; ++dc) {
          int l = L.cell(rr + dr, ccol + dc);
          if (l > n) U |= cl->B(kk, l);
        }
      if (kk == n) Un = U;
      else if (U) { kcells.push_back(kk); kmasks.push_back(U); }
    }
    // merge by boundary (Eq. 8) while some fixed cluster still couples to an
    // unfixed one; with an empty boundary (the last cluster, or only
    // uncoupled clusters left) every candidate is its own group
    const bool last = Un == 0 && kmasks.empty();
    int totbits = 0;
    for (auto m : kmasks) totbits += popcount32(m);
    const int W = std::max(1, (totbits + 31) / 32);
    int64_t ncand;
    if (!last) {
      if (bm->words.n < size_t(nb) * W) bm->words.alloc(size_t(nb) * W);
      if (bm->cls.n < size_t(nb)) bm->cls.alloc(size_t(nb));
      bm->kc.upload(kcells.empty() ? std::vector<int>{0} : kcells, st);
      bm->km.upload(kmasks.empty() ? std::vector<uint32_t>{0u} : kmasks, st);
      hipLaunchKernelGGL(parent_words_kernel, dim3(nblk(nb)), dim3(256), 0, st, bm->X.p, bm->ncell, nb, bm->kc.p,
                         bm->km.p, int(kcells.size()), W, bm->words.p);
      hipLaunchKernelGGL(parent_class_kernel, dim3(nblk(nb)), dim3(256), 0, st, bm->words.p, nb, W, bm->cls.p);
      ncand = int64_t(nb) << popcount32(Un);
    } else {
      ncand = int64_t(nb) * d;
    }
    int64_t np2 = 1;
    while (np2 < ncand) np2 <<= 1;
    if (bm->cand.n < size_t(np2)) bm->cand.alloc(size_t(np2));
    if (bm->win.n < size_t(np2)) bm->win.alloc(size_t(np2));
    hipLaunchKernelGGL(group_kernel, dim3(nblk(np2)), dim3(256), 0, st, bm->score.p, k, Un, nb,
                       last ? nullptr : bm->cls.p, last ? 0 : 1, bm->cand.p, np2);
    bitonic_sort(bm->cand.p, np2, st);
    if (bm->flag.n < size_t(np2)) bm->flag.alloc(size_t(np2));
    if (bm->pos.n < size_t(np2)) bm->pos.alloc(size_t(np2));
    if (bm->total.n < 1) bm->total.alloc(1);
    hipLaunchKernelGGL(winner_flag_kernel, dim3(nblk(np2)), dim3(256), 0, st, bm->cand.p, np2, bm->flag.p);
    {
      const int64_t ntile = (np2 + kScanTile - 1) / kScanTile;
      if (bm->tsum.n < size_t(2 * ntile)) bm->tsum.alloc(size_t(2 * ntile));
      hipLaunchKernelGGL(scan_tiles_kernel, dim3(unsigned(ntile)), dim3(256), 0, st, bm->flag.p, np2, bm->tsum.p);
      hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, bm->tsum.p, ntile, bm->tsum.p + ntile,
                         bm->total.p);
      hipLaunchKernelGGL(scan_apply_kernel, dim3(unsigned(ntile)), dim3(256), 0, st, bm->flag.p, np2,
                         bm->tsum.p + ntile, bm->pos.p);
    }
    int64_t nw = 0;
    HIPC(hipMemcpyAsync(&nw, bm->total.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    int64_t wp2 = 1;
    while (wp2 < nw) wp2 <<= 1;
    if (std::getenv("TNB_DEBUG")) {
      std::vector<uint32_t> hc(nb);
      if (!last) HIPC(hipMemcpy(hc.data(), bm->cls.p, nb * sizeof(uint32_t), hipMemcpyDeviceToHost));
      std::vector<Cand> hcand(std::min<int64_t>(np2, 64));
      HIPC(hipMemcpy(hcand.data(), bm->cand.p, hcand.size() * sizeof(Cand), hipMemcpyDeviceToHost));
      std::fprintf(stderr, "[tnb] step %d nb %d Un %x ncand %lld np2 %lld nw %lld W %d cls:", n, nb, Un,
                   (long long)ncand, (long long)np2, (long long)nw, W);
      for (auto v : hc) std::fprintf(stderr, " %u", v);
      std::fprintf(stderr, "\n  sorted gkeys:");
      for (auto& c : hcand) std::fprintf(stderr, " %llx/%u/%u", (unsigned long long)c.gkey, c.b, c.x);
      std::fprintf(stderr, "\n");
    }
    hipLaunchKernelGGL(fill_cand_kernel, dim3(nblk(wp2)), dim3(256), 0, st, bm->win.p, int64_t(0), wp2);
    hipLaunchKernelGGL(compact_kernel, dim3(nblk(np2)), dim3(256), 0, st, bm->cand.p, bm->flag.p, bm->pos.p, np2,
                       bm->win.p);
    bitonic_sort(bm->win.p, wp2, st);
    const int nsel = int(std::min<int64_t>(nw, bm->M));
    if (nsel == 0) fail(TNB_ENUMERIC, "no candidate with positive probability at step " + std::to_string(n));
    if (nw > bm->M) {
      Cand loser;
      HIPC(hipMemcpyAsync(&loser, bm->win.p + bm->M, sizeof(Cand), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      bm->pd_log = std::max(bm->pd_log, key_score(loser.skey));
    }
    hipLaunchKernelGGL(new_beam_kernel, dim3(nsel), dim3(64), 0, st, bm->win.p, nsel, bm->X.p, bm->ncell, n, bm->rid.p,
                       bm->Xn.p, bm->logpn.p, bm->ridn.p);
    if (bm->dopt.max_droplets > 0) droplet_step(bm, n, Un, !last, nb, nsel, st);
    // left vectors over the bond right of Psi site 2c
    const Mps& psi = bm->env->psi[r + 1];
    const Site& A2c = psi.sites[2 * c];
    ensure(bm->Ln, size_t(bm->M) * A2c.dr);
    hipLaunchKernelGGL(new_left_kernel, dim3(nsel), dim3(256), 0, st, bm->geo[c], bm->win.p, nsel, bm->T.p,
                       A2c.data.p, A2c.dl, A2c.dr, bm->Ln.p);
    HIPC(hipGetLastError());
    std::swap(bm->X, bm->Xn);
    std::swap(bm->logp, bm->logpn);
    std::swap(bm->rid, bm->ridn);
    std::swap(bm->L, bm->Ln);
    if (bm->dopt.max_droplets > 0) {
      std::swap(bm->Ep, bm->Epn);
      std::swap(bm->dcnt, bm->dcntn);
      std::swap(bm->dlen, bm->dlenn);
      std::swap(bm->dEv, bm->dEvn);
      std::swap(bm->dcell, bm->dcelln);
      std::swap(bm->dmask, bm->dmaskn);
    }
    bm->Ld = A2c.dr;
    bm->npar = nsel;
    bm->step = n + 1;
    if (p_disc_log) *p_disc_log = bm->pd_log;
    HIPC(hipStreamSynchronize(st));
  });
}

extern "C" tnb_status tnb_beam_export(const tnb_beam* bm, int32_t K, int8_t* d_states, double* d_logp,
                                      int32_t* count, tnb_stream stream) {
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (K < 0 || !d_states) fail(TNB_EINVAL, "bad output");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int k = std::min(K, bm->npar);
    const Lattice& L = bm->env->cl->lat;
    if (k > 0)
      hipLaunchKernelGGL(export_kernel, dim3(nblk(int64_t(k) * L.N)), dim3(256), 0, st, bm->X.p, bm->ncell, bm->step,
                         bm->cell_of.p, bm->bit.p, L.N, k, d_states, bm->logp.p, d_logp);
    HIPC(hipGetLastError());
    if (count) *count = k;
    HIPC(hipStreamSynchronize(st));
  });
}

extern "C" tnb_status tnb_beam_lowest(tnb_beam* bm, int32_t K, int8_t* d_states, double* d_E, int32_t* count,
                                      tnb_stream stream) {
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (K < 0 || (K > 0 && (!d_states || !d_E))) fail(TNB_EINVAL, "bad output");
    if (bm->step != bm->ncell) fail(TNB_EINVAL, "the beam has unfixed clusters");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const tnb_clusters* cl = bm->env->cl;
    const Lattice& L = cl->lat;
    const int n = bm->npar, N = L.N;
    int found = 0;
    if (n > 0 && K > 0) {
      if (bm->sel_states.n < size_t(n) * N) bm->sel_states.alloc(size_t(n) * N);
      if (bm->sel_E.n < size_t(n)) bm->sel_E.alloc(size_t(n));
      if (bm->sel_dup.n < size_t(n)) bm->sel_dup.alloc(size_t(n));
      hipLaunchKernelGGL(export_kernel, dim3(nblk(int64_t(n) * N)), dim3(256), 0, st, bm->X.p, bm->ncell, bm->step,
                         bm->cell_of.p, bm->bit.p, N, n, bm->sel_states.p, bm->logp.p, nullptr);
      hipLaunchKernelGGL(ising_energy_kernel, dim3(nblk(n, 128)), dim3(128), 0, st, bm->sel_states.p, int64_t(n), N,
                         L.E, cl->d_ei.p, cl->d_ej.p, cl->d_J.p, cl->d_h.p, bm->sel_E.p);
      hipLaunchKernelGGL(sel_dup_kernel, dim3(n), dim3(256), 0, st, bm->sel_states.p, bm->sel_E.p, n, N,
                         bm->sel_dup.p);
      hipLaunchKernelGGL(sel_rank_kernel, dim3(n), dim3(256), 0, st, bm->sel_states.p, bm->sel_E.p, bm->sel_dup.p, n,
                         N, K, d_states, d_E);
      HIPC(hipGetLastError());
      std::vector<int> dup(n);
      HIPC(hipMemcpyAsync(dup.data(), bm->sel_dup.p, size_t(n) * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      for (int v : dup) found += v ? 0 : 1;
    }
    if (count) *count = std::min(K, found);
  });
}

extern "C" tnb_status tnb_select_lowest(const int8_t* d_states, const double* d_E, int64_t n, int32_t n_spins,
                                        int32_t K, int8_t* d_out, double* d_E_out, int32_t* count,
                                        tnb_stream stream) {
  return guarded([&] {
    if (n < 0 || n > (int64_t(1) << 30) || n_spins < 1 || K < 0) fail(TNB_EINVAL, "bad sizes");
    if (n > 0 && (!d_states || !d_E)) fail(TNB_EINVAL, "NULL input");
    if (K > 0 && n > 0 && (!d_out || !d_E_out)) fail(TNB_EINVAL, "NULL output");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int found = 0;
    if (n > 0 && K > 0) {
      DevBuf<int> dup{static_cast<size_t>(n)};
      hipLaunchKernelGGL(sel_dup_kernel, dim3(unsigned(n)), dim3(256), 0, st, d_states, d_E, int(n), n_spins, dup.p);
      hipLaunchKernelGGL(sel_rank_kernel, dim3(unsigned(n)), dim3(256), 0, st, d_states, d_E, dup.p, int(n), n_spins, K,
                         d_out, d_E_out);
      HIPC(hipGetLastError());
      std::vector<int> h(static_cast<size_t>(n));
      HIPC(hipMemcpyAsync(h.data(), dup.p, size_t(n) * sizeof(int), hipMemcpyDeviceToHost, st));
      HIPC(hipStreamSynchronize(st));
      for (int v : h) found += v ? 0 : 1;
    }
    if (count) *count = std::min<int64_t>(K, found);
  });
}

extern "C" void tnb_destroy(void* handle) {
  if (!handle) return;
  uint32_t kind = *static_cast<uint32_t*>(handle);
  (void)hipDeviceSynchronize();
  if (kind == KIND_CLUSTERS) delete static_cast<tnb_clusters*>(handle);
  else if (kind == KIND_ENV) delete static_cast<tnb_env*>(handle);
  else if (kind == KIND_BEAM) delete static_cast<tnb_beam*>(handle);
}
