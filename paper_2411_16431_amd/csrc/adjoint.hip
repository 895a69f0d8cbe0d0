// Row moments of a beam state: <s_i>_b and <s_i s_j>_b for every spin and
// intra-cluster coupling of the unfixed clusters of the current row, for every
// parent b, with the boundary MPS below the row held fixed (Eq. 9-10, Fig. 6b).
//
// log Z_b of the conditioned row is a chain of linear maps over the columns;
// its derivative with respect to the local weights of column c' is the
// product of everything left of c' (the left environment Lambda) and
// everything right of it (the right environment R of the forward pass):
//   q'_b[x] = d Z_b / d log w_{c'}[x]
//           = w phi_b(x) (V'_b[xh(x)][b'(x)] . A_{2c'}[v'(x)]) . R_b^{(c')}[:, pi(x)]
// and <f>_b = sum_x q'_b[x] f(x) / sum_x q'_b[x] for f = s_i or s_i s_j.
// The backward sweep runs left to right, transposing the forward passes:
//   Lh[b][xh][a'][be] = sum_{pi: a'(pi) = a'} Lambda[b][be][pi] W_h(h(pi), xh)
//   V'[b][xh][b'][g]  = sum_{a', be} Lh[b][xh][a'][be] A_{2c'-1}[a' + da' b'][be][g]
//   Lambda'[b][e][pi] = sum_{x: pi(x) = pi} w phi_b(x) (V'[b][xh(x)][b'(x)] . A_{2c'}[v'(x)])[e]
// The right environments R^{(c')} are the checkpoints kept from the forward
// pass; the per-x products are recomputed rather than stored.
//
// The plain alternative, one contraction per branch s_i = +1 and s_i = -1 of
// every spin, reuses the stored R^{(c_i)} and sweeps the clamped column and
// those between it and the current column again for each branch.
#include <algorithm>
#include <cstdio>

#include "beam.h"

namespace tnb {

// Items of the moments reduction: kind 0 = <s_bi>, 1 = <s_bi s_bj>; out is the
// column of m1 (kind 0) or m2 (kind 1).
struct Item {
  int32_t kind, bi, bj, out;
};
static_assert(sizeof(Item) == 4 * sizeof(int32_t), "Item layout");

// V'[b][xh][b'][g] at the current column: the parent's fixed left part.
__global__ void adj_v0_kernel(BCol c, int has_left, int left_cell, const int32_t* __restrict__ X, int ncell,
                              const double* __restrict__ T, int Dl, int nb, double* __restrict__ Vp) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(c.dxh) * c.dbd * Dl;
  if (idx >= nb * per) return;
  const int b = int(idx / per);
  const uint32_t xh = uint32_t((idx / (int64_t(c.dbd) * Dl)) % c.dxh);
  const int bd = int((idx / Dl) % c.dbd);
  const int g = int(idx % Dl);
  double f = 1.0;
  if (has_left) f = c.Wh[pext_dev(uint32_t(X[size_t(b) * ncell + left_cell]), c.Bleft_h) * c.Wh_sp + xh * c.Wh_sq];
  Vp[idx] = f * T[(size_t(b) * c.dbd + bd) * Dl + g];
}

// q[b][x] = w phi_b(x) sum_e (V'[b][xh][b'] . A2c[v'(x)])[e] R[rid b][e][pi(x)]
__global__ void adj_q_kernel(BCol c, const int32_t* __restrict__ X, int ncell, const double* __restrict__ Vp,
                             const double* __restrict__ A2c, int Dl, int Dr, const double* __restrict__ R,
                             const int32_t* __restrict__ rid, int nb, double* __restrict__ q) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t d = int64_t(1) << c.k;
  if (idx >= nb * d) return;
  const int b = int(idx / d);
  const uint32_t x = uint32_t(idx % d);
  const double g = wloc(c, x) * phi_of(c, X + size_t(b) * ncell, x);
  if (g == 0.0) {
    q[idx] = 0.0;
    return;
  }
  const double* Vb = Vp + ((size_t(b) * c.dxh + pext_dev(x, c.Bxh)) * c.dbd + pext_dev(x, c.Bbd)) * Dl;
  const double* Av = A2c + size_t(pext_dev(x, c.Bvd)) * Dl * Dr;
  const double* Rb = R + size_t(rid[b]) * Dr * c.dpi;
  const uint32_t pi = pext_dev(x, c.PRR);
  double acc = 0.0;
  for (int e = 0; e < Dr; ++e) {
    double v = 0.0;
    for (int m = 0; m < Dl; ++m) v = fma(Vb[m], Av[size_t(m) * Dr + e], v);
    acc = fma(v, Rb[size_t(e) * c.dpi + pi], acc);
  }
  q[idx] = g * acc;
}

// adj_q on the matrix cores (Dl, Dr <= 16): one wave per cluster value x.
// For the parents in tiles of 16, Y = V'_x (16 x Dl) . A2c[v'(x)] (Dl x Dr)
// runs on v_mfma_f64_16x16x4f64; lane l then holds Y[b][e] with e = l % 16,
// multiplies it by R[b][e][pi(x)] (RT: R transposed to [anc][pi][e]) and the
// 16 lanes of one row sum over e with a fixed butterfly.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) adj_q_mfma(BCol c, const int32_t* __restrict__ X, int ncell,
                                                  const double* __restrict__ Vp, const double* __restrict__ A2c,
                                                  int Dl, int Dr, const double* __restrict__ RT,
                                                  const int32_t* __restrict__ rid, int nb, double* __restrict__ q) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int64_t d = int64_t(1) << c.k;
  const int64_t xw = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (xw >= d) return;  // x is uniform over the wave
  const uint32_t x = uint32_t(xw);
  const uint32_t xh = pext_dev(x, c.Bxh), bd = pext_dev(x, c.Bbd), pi = pext_dev(x, c.PRR);
  const double w0 = wloc(c, x);
  const double* Av = A2c + size_t(pext_dev(x, c.Bvd)) * Dl * Dr;
  double bv[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int m = 4 * kk + lk;
    bv[kk] = (m < Dl && li < Dr) ? Av[m * Dr + li] : 0.0;
  }
  const int64_t vstride = int64_t(c.dxh) * c.dbd * Dl;
  const double* Vx = Vp + (size_t(xh) * c.dbd + bd) * Dl;
  for (int b0 = 0; b0 < nb; b0 += 16) {
    v4d y = v4d{0.0, 0.0, 0.0, 0.0};
    const int b = b0 + li;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int m = 4 * kk + lk;
      const double a = (b < nb && m < Dl) ? Vx[b * vstride + m] : 0.0;
      y = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[kk], y, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int bb = b0 + 4 * v + lk;  // row of item v; column e = li
      double t = 0.0;
      if (bb < nb && li < Dr) t = y[v] * RT[(size_t(rid[bb]) * c.dpi + pi) * Dr + li];
      for (int o = 8; o > 0; o >>= 1) t += __shfl_xor(t, o, 16);
      if (li == 0 && bb < nb) {
        const double g = w0 == 0.0 ? 0.0 : w0 * phi_of(c, X + size_t(bb) * ncell, x);
        q[size_t(bb) * d + x] = g * t;
      }
    }
  }
}

// Lambda' on the matrix cores (Dl, Dr <= 16): one wave per pi, summing over
// the cluster values x of the class; Y = V'_x A2c[v'(x)] for 16 parents per
// MFMA tile, weighted by w phi_b(x), written [b][pi][e] (e along the lanes).
__global__ void __launch_bounds__(256) adj_lam_mfma(BCol c, const int32_t* __restrict__ X, int ncell,
                                                    const double* __restrict__ Vp, const double* __restrict__ A2c,
                                                    int Dl, int Dr, int nb, double* __restrict__ LamT) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  const int64_t pw = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (pw >= c.dpi) return;  // pi is uniform over the wave
  const uint32_t pi = uint32_t(pw);
  const uint32_t full = c.k ? ((1u << c.k) - 1u) : 0u;
  const uint32_t FREE = full & ~c.PRR;
  const int nf = 1 << __builtin_popcount(FREE);
  const uint32_t base = pdep_dev(pi, c.PRR);
  const int64_t vstride = int64_t(c.dxh) * c.dbd * Dl;
  for (int b0 = 0; b0 < nb; b0 += 16) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int b = b0 + li;
    for (int f = 0; f < nf; ++f) {
      const uint32_t x = base | pdep_dev(uint32_t(f), FREE);
      const double w0 = wloc(c, x);
      if (w0 == 0.0) continue;
      const double* Av = A2c + size_t(pext_dev(x, c.Bvd)) * Dl * Dr;
      const double* Vx = Vp + (size_t(pext_dev(x, c.Bxh)) * c.dbd + pext_dev(x, c.Bbd)) * Dl;
      v4d y = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int m = 4 * kk + lk;
        const double a = (b < nb && m < Dl) ? Vx[b * vstride + m] : 0.0;
        const double bvv = (m < Dl && li < Dr) ? Av[m * Dr + li] : 0.0;
        y = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bvv, y, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int bb = b0 + 4 * v + lk;
        if (bb < nb) acc[v] = fma(w0 * phi_of(c, X + size_t(bb) * ncell, x), y[v], acc[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int bb = b0 + 4 * v + lk;
      if (bb < nb && li < Dr) LamT[(size_t(bb) * c.dpi + pi) * Dr + li] = acc[v];
    }
  }
}

// out[a][j][i] = in[a][i][j] for a < count (per-item transpose of r x c blocks)
__global__ void adj_transpose_kernel(const double* __restrict__ in, int64_t count, int r, int c,
                                     double* __restrict__ out) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= count * r * c) return;
  const int64_t n = idx / (int64_t(r) * c);
  const int64_t rc = idx % (int64_t(r) * c);
  const int64_t i = rc / c, j = rc % c;
  out[(n * c + j) * r + i] = in[idx];
}

// Lambda'[b][e][pi] = sum_{x: pi(x) = pi} w phi_b(x) (V'[b][xh(x)][b'(x)] . A2c[v'(x)])[e],
// stored [b][pi][e]
__global__ void adj_lam_kernel(BCol c, const int32_t* __restrict__ X, int ncell, const double* __restrict__ Vp,
                               const double* __restrict__ A2c, int Dl, int Dr, int nb, double* __restrict__ Lam) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(Dr) * c.dpi;
  if (idx >= nb * per) return;
  const int b = int(idx / per);
  const int e = int((idx / c.dpi) % Dr);
  const uint32_t pi = uint32_t(idx % c.dpi);
  const uint32_t full = c.k ? ((1u << c.k) - 1u) : 0u;
  const uint32_t FREE = full & ~c.PRR;
  const int nf = 1 << __builtin_popcount(FREE);
  const uint32_t base = pdep_dev(pi, c.PRR);
  const int32_t* Xb = X + size_t(b) * ncell;
  double acc = 0.0;
  for (int f = 0; f < nf; ++f) {
    const uint32_t x = base | pdep_dev(uint32_t(f), FREE);
    const double g = wloc(c, x) * phi_of(c, Xb, x);
    if (g == 0.0) continue;
    const double* Vb = Vp + ((size_t(b) * c.dxh + pext_dev(x, c.Bxh)) * c.dbd + pext_dev(x, c.Bbd)) * Dl;
    const double* Av = A2c + size_t(pext_dev(x, c.Bvd)) * Dl * Dr + e;
    double v = 0.0;
    for (int m = 0; m < Dl; ++m) v = fma(Vb[m], Av[size_t(m) * Dr], v);
    acc = fma(g, v, acc);
  }
  Lam[(size_t(b) * c.dpi + pi) * Dr + e] = acc;  // [b][pi][e]
}

// Lh[b][xh][a'][be] = sum_{pi: a'(pi) = a'} Lambda[b][be][pi] W_h(h(pi), xh)
// (c: geometry of column c'; pi runs over PRR of column c'-1; Lambda stored [b][pi][be])
__global__ void adj_lh_kernel(BCol c, int dpi_prev, const double* __restrict__ Lam, int nb, int Dl,
                              double* __restrict__ Lh) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t per = int64_t(c.da2) * c.dxh * Dl;
  if (idx >= nb * per) return;
  const int b = int(idx / per);
  const uint32_t xh = uint32_t((idx / (int64_t(c.da2) * Dl)) % c.dxh);
  const uint32_t a2 = uint32_t((idx / Dl) % c.da2);
  const int be = int(idx % Dl);
  const uint32_t FREEh = c.pos_h & ~c.pos_a;
  const int nf = 1 << __builtin_popcount(FREEh);
  const uint32_t base = pdep_dev(a2, c.pos_a);
  const double* Lb = Lam + size_t(b) * dpi_prev * Dl + be;  // Lambda stored [b][pi][be]
  double acc = 0.0;
  for (int f = 0; f < nf; ++f) {
    const uint32_t pi = base | pdep_dev(uint32_t(f), FREEh);
    acc = fma(Lb[size_t(pi) * Dl], c.Wh[pext_dev(pi, c.pos_h) * c.Wh_sp + xh * c.Wh_sq], acc);
  }
  Lh[idx] = acc;
}

// Per parent b (blockIdx.x) and a chunk of up to 8 items (blockIdx.y):
// Z = sum_x q[b][x] and <f>_b = sum_x q[b][x] f(x) / Z.
constexpr int kItemsPerBlock = 8;
__global__ void adj_moments_kernel(const double* __restrict__ q, int64_t d, const Item* __restrict__ items,
                                   int n_items, int ld1, int ld2, double* __restrict__ m1, double* __restrict__ m2,
                                   int* __restrict__ bad) {
  __shared__ double red[kItemsPerBlock + 1][256];
  const int b = blockIdx.x;
  const int i0 = blockIdx.y * kItemsPerBlock;
  const int ni = min(kItemsPerBlock, n_items - i0);
  Item it[kItemsPerBlock];
  for (int j = 0; j < kItemsPerBlock; ++j) it[j] = j < ni ? items[i0 + j] : Item{0, 0, 0, 0};
  double z = 0.0, acc[kItemsPerBlock];
  for (int j = 0; j < kItemsPerBlock; ++j) acc[j] = 0.0;
  for (int64_t xi = threadIdx.x; xi < d; xi += blockDim.x) {
    const double v = q[size_t(b) * d + xi];
    const uint32_t x = uint32_t(xi);
    z += v;
    for (int j = 0; j < kItemsPerBlock; ++j) {
      const uint32_t s = it[j].kind == 0 ? ((x >> it[j].bi) & 1u) : (((x >> it[j].bi) ^ (x >> it[j].bj) ^ 1u) & 1u);
      acc[j] += s ? v : -v;
    }
  }
  red[0][threadIdx.x] = z;
  for (int j = 0; j < kItemsPerBlock; ++j) red[j + 1][threadIdx.x] = acc[j];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j <= kItemsPerBlock; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < ni) {
    const int j = threadIdx.x;
    const double Z = red[0][0];
    const double v = red[j + 1][0] / Z;
    if (!(Z != 0.0) || !isfinite(v)) bad[0] = 1;
    if (it[j].kind == 0) m1[size_t(b) * ld1 + it[j].out] = v;
    else if (m2) m2[size_t(b) * ld2 + it[j].out] = v;
  }
}

// zs[b] = sum_x q[b][x]
__global__ void adj_rowsum_kernel(const double* __restrict__ q, int64_t d, double* __restrict__ zs) {
  __shared__ double red[256];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += blockDim.x) acc += q[size_t(b) * d + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) zs[b] = red[0];
}

// m1[b][out] = (Z+ - Z-) / (Z+ + Z-), Z = zs exp(zl), both branches per parent
__global__ void adj_branch_ratio_kernel(const double* __restrict__ zs, const double* __restrict__ zl, int nb, int out,
                                        int ld1, double* __restrict__ m1, int* __restrict__ bad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const double lp = zl[b], lm = zl[nb + b];
  const double top = fmax(lp, lm);
  const double zp = zs[b] * exp(lp - top), zm = zs[nb + b] * exp(lm - top);
  const double v = (zp - zm) / (zp + zm);
  if (!(zp + zm != 0.0) || !isfinite(v)) bad[0] = 1;
  m1[size_t(b) * ld1 + out] = v;
}

__global__ void adj_gather_rows_kernel(const double* __restrict__ src, const int32_t* __restrict__ rid, int64_t per,
                                       int nb, double* __restrict__ dst) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= nb * per) return;
  dst[idx] = src[size_t(rid[idx / per]) * per + idx % per];
}

__global__ void adj_fill_kernel(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void adj_iota_kernel(int32_t* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

// Spins and intra-cluster couplings of the unfixed clusters of the current
// row, and the reduction items per column.
static void row_layout(tnb_beam* bm) {
  if (bm->lay_step == bm->step) return;
  const Lattice& L = bm->env->cl->lat;
  const int r = bm->step / L.C, c = bm->step % L.C;
  bm->lay_spins.clear();
  bm->lay_edges.clear();
  bm->lay_items.clear();
  bm->lay_off.clear();
  int nitems = 0;
  for (int cc = c; cc < L.C; ++cc) {
    const int n = L.cell(r, cc);
    bm->lay_off.push_back(nitems);
    for (int s : L.spins[n]) {
      bm->lay_items.insert(bm->lay_items.end(), {0, L.bit[s], 0, int32_t(bm->lay_spins.size())});
      bm->lay_spins.push_back(s);
      ++nitems;
    }
    for (int e = 0; e < L.E; ++e) {
      if (L.cell_of[L.ei[e]] != n || L.cell_of[L.ej[e]] != n) continue;
      bm->lay_items.insert(bm->lay_items.end(), {1, L.bit[L.ei[e]], L.bit[L.ej[e]], int32_t(bm->lay_edges.size())});
      bm->lay_edges.push_back(e);
      ++nitems;
    }
  }
  bm->lay_off.push_back(nitems);
  bm->items.upload(bm->lay_items, nullptr);
  HIPC(hipDeviceSynchronize());
  bm->lay_step = bm->step;
}

static void moments_of(tnb_beam* bm, const double* q, int64_t d, int col, double* m1, double* m2, hipStream_t st) {
  const int i0 = bm->lay_off[col], i1 = bm->lay_off[col + 1];
  if (i1 == i0) return;
  const Item* items = reinterpret_cast<const Item*>(bm->items.p) + i0;
  const int nch = (i1 - i0 + kItemsPerBlock - 1) / kItemsPerBlock;
  KTimer _t("adj_moments", st, 2.0 * bm->npar * double(d) * (i1 - i0 + 1), 8.0 * bm->npar * double(d) * nch);
  hipLaunchKernelGGL(adj_moments_kernel, dim3(bm->npar, nch), dim3(256), 0, st, q, d, items, i1 - i0,
                     int(bm->lay_spins.size()), int(bm->lay_edges.size()), m1, m2, bm->dead.p);
  HIPC(hipGetLastError());
}

static void check_args(tnb_beam* bm, double* m1, int64_t m1_len, double* m2, int64_t m2_len) {
  if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
  if (bm->step >= bm->ncell) fail(TNB_EINVAL, "every cluster is fixed");
  row_layout(bm);
  if (!m1 || m1_len < int64_t(bm->npar) * int64_t(bm->lay_spins.size())) fail(TNB_EINVAL, "m1 too small");
  if (m2 && m2_len < int64_t(bm->npar) * int64_t(bm->lay_edges.size())) fail(TNB_EINVAL, "m2 too small");
}

static void finish(tnb_beam* bm, hipStream_t st, const char* what) {
  int bad = 0;
  HIPC(hipMemcpyAsync(&bad, bm->dead.p, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  if (bad) fail(TNB_ENUMERIC, std::string(what) + ": zero or non-finite contraction at step " + std::to_string(bm->step));
}

}  // namespace tnb

using namespace tnb;

extern "C" tnb_status tnb_row_layout(const tnb_beam* beam, int32_t* n_spins, int32_t* n_edges, int32_t* spins,
                                     int32_t* edges, int32_t cap) {
  return guarded([&] {
    tnb_beam* bm = const_cast<tnb_beam*>(beam);
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (bm->step >= bm->ncell) fail(TNB_EINVAL, "every cluster is fixed");
    row_layout(bm);
    if (n_spins) *n_spins = int32_t(bm->lay_spins.size());
    if (n_edges) *n_edges = int32_t(bm->lay_edges.size());
    if (spins) std::copy_n(bm->lay_spins.begin(), std::min<size_t>(std::max(cap, 0), bm->lay_spins.size()), spins);
    if (edges) std::copy_n(bm->lay_edges.begin(), std::min<size_t>(std::max(cap, 0), bm->lay_edges.size()), edges);
  });
}

extern "C" tnb_status tnb_row_moments(tnb_beam* bm, double* d_m1, int64_t m1_len, double* d_m2, int64_t m2_len,
                                      tnb_stream stream) {
  return guarded([&] {
    check_args(bm, d_m1, m1_len, d_m2, m2_len);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Lattice& L = bm->env->cl->lat;
    const int r = bm->step / L.C, c = bm->step % L.C, C = L.C;
    const int nb = bm->npar;
    compute_q(bm, st);  // right environments (checkpoints), T and q of column c
    const Mps& psi = bm->env->psi[r + 1];
    HIPC(hipMemsetAsync(bm->dead.p, 0, sizeof(int), st));
    moments_of(bm, bm->q.p, int64_t(1) << bm->geo[c].k, 0, d_m1, d_m2, st);
    if (c + 1 < C) {
      // V' of the current column from the parent's left vector
      const BCol& g0 = bm->geo[c];
      const Site& A0 = psi.sites[2 * c];
      ensure(bm->vp, size_t(nb) * g0.dxh * g0.dbd * A0.dl);
      hipLaunchKernelGGL(adj_v0_kernel, dim3(nblk(int64_t(nb) * g0.dxh * g0.dbd * A0.dl)), dim3(256), 0, st, g0,
                         c > 0 ? 1 : 0, c > 0 ? L.cell(r, c - 1) : 0, bm->X.p, bm->ncell, bm->T.p, A0.dl, nb,
                         bm->vp.p);
      for (int cp = c; cp + 1 < C; ++cp) {
        const BCol& gc = bm->geo[cp];
        const Site& Ac = psi.sites[2 * cp];
        ensure(bm->lam, size_t(nb) * Ac.dr * gc.dpi);
        {
          KTimer _t("adj_lam", st, 2.0 * nb * double(int64_t(1) << gc.k) * Ac.dl * Ac.dr,
                    8.0 * (double(nb) * Ac.dr * gc.dpi + double(nb) * gc.dxh * gc.dbd * Ac.dl + Ac.size()));
          if (Ac.dl <= 16 && Ac.dr <= 16) {
            hipLaunchKernelGGL(adj_lam_mfma, dim3(unsigned((gc.dpi + 3) / 4)), dim3(256), 0, st, gc, bm->X.p,
                               bm->ncell, bm->vp.p, Ac.data.p, Ac.dl, Ac.dr, nb, bm->lam.p);
          } else {
            hipLaunchKernelGGL(adj_lam_kernel, dim3(nblk(int64_t(nb) * Ac.dr * gc.dpi)), dim3(256), 0, st, gc,
                               bm->X.p, bm->ncell, bm->vp.p, Ac.data.p, Ac.dl, Ac.dr, nb, bm->lam.p);
          }
        }
        normalise_rows(bm->lam.p, int64_t(Ac.dr) * gc.dpi, nb, nullptr, st);
        // next column
        const int cn = cp + 1;
        const BCol& gn = bm->geo[cn];
        const Site& Am = psi.sites[2 * cn - 1];
        const Site& An = psi.sites[2 * cn];
        ensure(bm->lh, size_t(nb) * gn.da2 * gn.dxh * Am.dl);
        {
          KTimer _t("adj_lh", st, 2.0 * nb * double(Am.dl) * gc.dpi * gn.dxh,
                    8.0 * (double(nb) * Am.dl * gc.dpi + double(nb) * gn.da2 * gn.dxh * Am.dl));
          hipLaunchKernelGGL(adj_lh_kernel, dim3(nblk(int64_t(nb) * gn.da2 * gn.dxh * Am.dl)), dim3(256), 0, st, gn,
                             gc.dpi, bm->lam.p, nb, Am.dl, bm->lh.p);
        }
        ensure(bm->vp, size_t(nb) * gn.dxh * gn.dbd * Am.dr);
        {
          // V'[b][xh][b'][g] = sum_{a', be} Lh[b][xh][a'][be] A_{2c'-1}[a' + da' b'][be][g]: rows
          // (b, xh), columns (b', g), reduction (a', be) -- one GEMM on the matrix cores
          const int Dl = Am.dl, Dr = Am.dr;
          const int Kd = gn.da2 * Dl, N = gn.dbd * Dr;
          la::Operand Lop{bm->lh.p, 0, la::Ix{0, 0, Kd}, la::Ix{0, 0, 1}};
          la::Operand Aop{Am.data.p, 0, la::Ix{0, 0, Dr}, la::Ix{uint32_t(Dr), int64_t(gn.da2) * Dl * Dr, 1}};
          la::gemm_mfma(1, nb * gn.dxh, N, Kd, Lop, Aop, bm->vp.p, la::Ix{0, 0, N}, la::Ix{0, 0, 1}, 0, 1.0, 0.0,
                        st, "adj_v");
        }
        const int64_t dn = int64_t(1) << gn.k;
        ensure(bm->qa, size_t(nb) * dn);
        {
          KTimer _t("adj_q", st, double(nb) * dn * (2.0 * An.dl * An.dr + 2.0 * An.dr),
                    8.0 * (double(nb) * dn + An.size() + double(bm->nanc) * An.dr * gn.dpi));
          if (An.dl <= 16 && An.dr <= 16) {
            // R^{(c')} transposed to [anc][pi][e] for the e-contiguous reads of adj_q_mfma
            const int64_t nr = int64_t(bm->nanc) * An.dr * gn.dpi;
            ensure(bm->rt0, size_t(nr));
            hipLaunchKernelGGL(adj_transpose_kernel, dim3(nblk(nr)), dim3(256), 0, st, bm->R[cn].p,
                               int64_t(bm->nanc), An.dr, gn.dpi, bm->rt0.p);
            hipLaunchKernelGGL(adj_q_mfma, dim3(unsigned((dn + 3) / 4)), dim3(256), 0, st, gn, bm->X.p, bm->ncell,
                               bm->vp.p, An.data.p, An.dl, An.dr, bm->rt0.p, bm->rid.p, nb, bm->qa.p);
          } else {
            hipLaunchKernelGGL(adj_q_kernel, dim3(nblk(int64_t(nb) * dn)), dim3(256), 0, st, gn, bm->X.p,
                               bm->ncell, bm->vp.p, An.data.p, An.dl, An.dr, bm->R[cn].p, bm->rid.p, nb, bm->qa.p);
          }
        }
        HIPC(hipGetLastError());
        moments_of(bm, bm->qa.p, dn, cn - c, d_m1, d_m2, st);
      }
    }
    finish(bm, st, "row moments");
  });
}

extern "C" tnb_status tnb_row_moments_per_branch(tnb_beam* bm, double* d_m1, int64_t m1_len, tnb_stream stream) {
  return guarded([&] {
    check_args(bm, d_m1, m1_len, nullptr, 0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Lattice& L = bm->env->cl->lat;
    const int r = bm->step / L.C, c = bm->step % L.C, C = L.C;
    const int nb = bm->npar;
    compute_q(bm, st);
    const Mps& psi = bm->env->psi[r + 1];
    HIPC(hipMemsetAsync(bm->dead.p, 0, sizeof(int), st));
    ensure(bm->zs, size_t(2) * nb);
    ensure(bm->zl, size_t(2) * nb);
    if (bm->iota.n < size_t(nb)) bm->iota.alloc(size_t(bm->M));
    hipLaunchKernelGGL(adj_iota_kernel, dim3(nblk(nb)), dim3(256), 0, st, bm->iota.p, nb);
    size_t rmax = 1;
    for (int cc = c; cc < C; ++cc) rmax = std::max(rmax, bm->R[cc].n / std::max(bm->nanc, 1));
    ensure(bm->rt0, size_t(nb) * rmax);
    ensure(bm->rt1, size_t(nb) * rmax);
    int out = 0;
    for (int ci = c; ci < C; ++ci) {
      const BCol& base = bm->geo[ci];
      for (int bit = 0; bit < base.k; ++bit, ++out) {
        for (int br = 0; br < 2; ++br) {
          BCol gcl = base;
          gcl.cmask = 1u << bit;
          gcl.cval = br == 0 ? gcl.cmask : 0u;
          double* zl = bm->zl.p + size_t(br) * nb;
          hipLaunchKernelGGL(adj_fill_kernel, dim3(nblk(nb)), dim3(256), 0, st, zl, int64_t(nb), 0.0);
          const int64_t d = int64_t(1) << bm->geo[c].k;
          ensure(bm->qa, size_t(nb) * d);
          if (ci == c) {
            q_against(bm, gcl, bm->R[c].p, bm->rid.p, bm->qa.p, st);
          } else {
            const int64_t per = int64_t(bm->R[ci].n / bm->nanc);
            hipLaunchKernelGGL(adj_gather_rows_kernel, dim3(nblk(int64_t(nb) * per)), dim3(256), 0, st, bm->R[ci].p,
                               bm->rid.p, per, nb, bm->rt0.p);
            double* cur = bm->rt0.p;
            double* nxt = bm->rt1.p;
            for (int cc = ci; cc > c; --cc) {
              row_step(bm, cc == ci ? gcl : bm->geo[cc], cc, nb, cur, nxt, zl, st);
              std::swap(cur, nxt);
            }
            q_against(bm, bm->geo[c], cur, bm->iota.p, bm->qa.p, st);
          }
          hipLaunchKernelGGL(adj_rowsum_kernel, dim3(nb), dim3(256), 0, st, bm->qa.p, d, bm->zs.p + size_t(br) * nb);
        }
        hipLaunchKernelGGL(adj_branch_ratio_kernel, dim3(nblk(nb)), dim3(256), 0, st, bm->zs.p, bm->zl.p, nb, out,
                           int(bm->lay_spins.size()), d_m1, bm->dead.p);
        HIPC(hipGetLastError());
      }
    }
    finish(bm, st, "per-branch row moments");
  });
}
