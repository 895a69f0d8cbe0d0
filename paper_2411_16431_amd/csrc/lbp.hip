// Local dimensional reduction (Sec. IV, Fig. 9): loopy belief propagation
// over the cluster graph with messages on projected states (Eq. 4), cluster
// beliefs, and the reduction of every cluster to its most probable states.
//
// One synchronous iteration, for every directed bond m -> n:
//   mu[m->n](xbar_m) = sum_{x_m : P^{mn} x_m = xbar_m} w_m(x_m) prod_{m' in N(m)\n} nu[m'->m](P^{mm'} x_m)
//   nu[m->n](xbar_n) = sum_{xbar_m} W_mn(xbar_m, xbar_n) mu[m->n](xbar_m),   normalised to sum 1
// from the previous iteration's messages (uniform at the start).  Beliefs:
//   p_n(x) ~ w_n(x) prod_{m in N(n)} nu[m->n](P^{nm} x).
// Every sum is a fixed-order block reduction, so results do not depend on
// scheduling.  The reduction keeps, per cluster, the `keep` states of largest
// belief (ties: smaller x) and sets the local weight of the others to zero,
// so every later contraction and search on the handle runs on the reduced
// state space (the kernels still index the full 2^k range).
#include "beam.h"
#include "model.h"

namespace tnb {

constexpr int LBP_NIN = 8;  // king neighbours

struct LbpBond {
  int m, n, dm, dn, nf;       // nf: values of m's spins outside P^{mn}
  uint32_t Bmn, FREE;
  int64_t msg, mu;            // offsets of nu[m->n] (dn) and mu[m->n] (dm)
  const double* W;            // W(xbar_m, xbar_n) = W[xbar_m * sp + xbar_n * sq]
  int64_t sp, sq;
  int64_t wm;                 // offset of m's local table
  int nin;                    // incoming messages to m other than from n
  int64_t in_msg[LBP_NIN];
  uint32_t in_mask[LBP_NIN];
};

struct LbpCell {
  int64_t w;                  // offset of the local table (and of the beliefs)
  int k, nin;
  int64_t in_msg[LBP_NIN];
  uint32_t in_mask[LBP_NIN];
};

__device__ inline double block_sum256(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// mu[e][xbar] for bond e = blockIdx.y, xbar = blockIdx.x
__global__ void __launch_bounds__(256) lbp_mu_kernel(const LbpBond* __restrict__ bonds, const double* __restrict__ w,
                                                     const double* __restrict__ nu, double* __restrict__ mu) {
  __shared__ double red[256];
  const LbpBond& e = bonds[blockIdx.y];
  const uint32_t xb = blockIdx.x;
  if (int(xb) >= e.dm) return;  // uniform over the workgroup
  const uint32_t base = pdep_dev(xb, e.Bmn);
  double acc = 0.0;
  for (int f = threadIdx.x; f < e.nf; f += 256) {
    const uint32_t x = base | pdep_dev(uint32_t(f), e.FREE);
    double g = w[e.wm + x];
    for (int i = 0; i < e.nin; ++i) g *= nu[e.in_msg[i] + pext_dev(x, e.in_mask[i])];
    acc += g;
  }
  const double s = block_sum256(acc, red);
  if (threadIdx.x == 0) mu[e.mu + xb] = s;
}

// nu_new[e][xbar_n] = sum_xbar_m W(xbar_m, xbar_n) mu[e][xbar_m], then normalised;
// chg[e] = max |nu_new - nu_old| over the message
__global__ void __launch_bounds__(256) lbp_nu_kernel(const LbpBond* __restrict__ bonds, const double* __restrict__ mu,
                                                     const double* __restrict__ nu_old, double* __restrict__ nu_new,
                                                     double* __restrict__ chg) {
  __shared__ double red[256];
  const LbpBond& e = bonds[blockIdx.x];
  double part = 0.0;
  for (int xn = threadIdx.x; xn < e.dn; xn += 256) {
    double v = 0.0;
    for (int xm = 0; xm < e.dm; ++xm) v = fma(e.W[int64_t(xm) * e.sp + int64_t(xn) * e.sq], mu[e.mu + xm], v);
    nu_new[e.msg + xn] = v;
    part += v;
  }
  const double s = block_sum256(part, red);
  double mx = 0.0;
  for (int xn = threadIdx.x; xn < e.dn; xn += 256) {
    const double v = s > 0.0 ? nu_new[e.msg + xn] / s : 1.0 / double(e.dn);
    nu_new[e.msg + xn] = v;
    mx = fmax(mx, fabs(v - nu_old[e.msg + xn]));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) chg[blockIdx.x] = red[0];
}

__global__ void lbp_fill_kernel(double* __restrict__ nu, const LbpBond* __restrict__ bonds, int nbond) {
  const int e = blockIdx.x;
  if (e >= nbond) return;
  for (int x = threadIdx.x; x < bonds[e].dn; x += blockDim.x) nu[bonds[e].msg + x] = 1.0 / double(bonds[e].dn);
}

// beliefs of cluster blockIdx.x, normalised
__global__ void __launch_bounds__(256) lbp_belief_kernel(const LbpCell* __restrict__ cells, const double* __restrict__ w,
                                                         const double* __restrict__ nu, double* __restrict__ p) {
  __shared__ double red[256];
  const LbpCell& c = cells[blockIdx.x];
  const int64_t d = int64_t(1) << c.k;
  double part = 0.0;
  for (int64_t x = threadIdx.x; x < d; x += 256) {
    double g = w[c.w + x];
    for (int i = 0; i < c.nin; ++i) g *= nu[c.in_msg[i] + pext_dev(uint32_t(x), c.in_mask[i])];
    p[c.w + x] = g;
    part += g;
  }
  const double s = block_sum256(part, red);
  for (int64_t x = threadIdx.x; x < d; x += 256) p[c.w + x] = s > 0.0 ? p[c.w + x] / s : 1.0 / double(d);
}

__global__ void max_reduce_kernel(const double* __restrict__ v, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// candidates (cluster, -belief, x) for the per-cluster ranking; padding sorts last
__global__ void lbp_cand_kernel(const double* __restrict__ p, const int32_t* __restrict__ cell_of_state,
                                const int64_t* __restrict__ off, int64_t total, Cand* __restrict__ a, int64_t np2) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= np2) return;
  if (i < total) {
    const int n = cell_of_state[i];
    a[i] = Cand{uint64_t(n), score_key(p[i]), 0u, uint32_t(i - off[n])};
  } else {
    a[i] = Cand{~0ull, ~0ull, ~0u, ~0u};
  }
}

// keep the first `keep` of each cluster in the sorted order: zero the others' weights
__global__ void lbp_apply_kernel(const Cand* __restrict__ a, const int64_t* __restrict__ off, int64_t total,
                                 int keep, double* __restrict__ w, float* __restrict__ w32) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const Cand c = a[i];
  const int n = int(c.gkey);
  const int64_t rank = i - off[n];
  if (rank >= keep) {
    w[off[n] + c.x] = 0.0;
    if (w32) w32[off[n] + c.x] = 0.0f;
  }
}

struct LbpPlan {
  std::vector<LbpBond> bonds;
  std::vector<LbpCell> cells;
  int64_t nmsg = 0, nmu = 0;
};

static LbpPlan lbp_plan(const tnb_clusters* cl) {
  const Lattice& L = cl->lat;
  LbpPlan pl;
  const int nc = L.cells();
  // message offsets of every directed bond m -> n
  std::vector<std::vector<int>> nbr(static_cast<size_t>(nc));
  std::map<int64_t, int64_t> msg_at;
  for (int n = 0; n < nc; ++n)
    for (int dr = -1; dr <= 1; ++dr)
      for (int dc = -1; dc <= 1; ++dc) {
        const int m = L.cell(n / L.C + dr, n % L.C + dc);
        if (m >= 0 && m != n && cl->B(n, m)) nbr[size_t(n)].push_back(m);
      }
  for (int m = 0; m < nc; ++m)
    for (int n : nbr[size_t(m)]) {
      msg_at[int64_t(m) * nc + n] = pl.nmsg;
      pl.nmsg += int64_t(1) << popcount32(cl->B(n, m));
    }
  for (int m = 0; m < nc; ++m)
    for (int n : nbr[size_t(m)]) {
      LbpBond e{};
      e.m = m;
      e.n = n;
      e.Bmn = cl->B(m, n);
      e.dm = 1 << popcount32(e.Bmn);
      e.dn = 1 << popcount32(cl->B(n, m));
      const int k = L.k[m];
      const uint32_t full = k ? ((k == 32) ? ~0u : ((1u << k) - 1u)) : 0u;
      e.FREE = full & ~e.Bmn;
      e.nf = 1 << popcount32(e.FREE);
      e.msg = msg_at[int64_t(m) * nc + n];
      e.mu = pl.nmu;
      pl.nmu += e.dm;
      if (!cl->weight_view(m, n, &e.W, &e.sp, &e.sq)) fail(TNB_EINVAL, "coupled clusters without a bond table");
      e.wm = cl->loc_off[size_t(m)];
      for (int mp : nbr[size_t(m)]) {
        if (mp == n) continue;
        e.in_msg[e.nin] = msg_at[int64_t(mp) * nc + m];
        e.in_mask[e.nin] = cl->B(m, mp);
        ++e.nin;
      }
      pl.bonds.push_back(e);
    }
  for (int n = 0; n < nc; ++n) {
    LbpCell c{};
    c.w = cl->loc_off[size_t(n)];
    c.k = L.k[n];
    for (int m : nbr[size_t(n)]) {
      c.in_msg[c.nin] = msg_at[int64_t(m) * nc + n];
      c.in_mask[c.nin] = cl->B(n, m);
      ++c.nin;
    }
    pl.cells.push_back(c);
  }
  return pl;
}

// Beliefs of every cluster into p (loc_off layout); returns the largest
// message change of the last iteration.
static double lbp_run(const tnb_clusters* cl, int iters, double* p, hipStream_t st) {
  const LbpPlan pl = lbp_plan(cl);
  const int nb = int(pl.bonds.size()), nc = int(pl.cells.size());
  DevBuf<LbpBond> db;
  DevBuf<LbpCell> dc;
  DevBuf<double> nu0, nu1, mu, chg, mx;
  if (nb) db.upload(pl.bonds, st);
  dc.upload(pl.cells, st);
  nu0.alloc(size_t(std::max<int64_t>(pl.nmsg, 1)));
  nu1.alloc(size_t(std::max<int64_t>(pl.nmsg, 1)));
  mu.alloc(size_t(std::max<int64_t>(pl.nmu, 1)));
  chg.alloc(size_t(std::max(nb, 1)));
  mx.alloc(1);
  HIPC(hipMemsetAsync(chg.p, 0, sizeof(double) * size_t(std::max(nb, 1)), st));
  KTimer _t("lbp", st, 0.0, 0.0);
  int maxdm = 1;
  for (const auto& e : pl.bonds) maxdm = std::max(maxdm, e.dm);
  if (nb) hipLaunchKernelGGL(lbp_fill_kernel, dim3(unsigned(nb)), dim3(256), 0, st, nu0.p, db.p, nb);
  double* cur = nu0.p;
  double* nxt = nu1.p;
  for (int it = 0; it < iters && nb; ++it) {
    hipLaunchKernelGGL(lbp_mu_kernel, dim3(unsigned(maxdm), unsigned(nb)), dim3(256), 0, st, db.p, cl->w_loc.p, cur,
                       mu.p);
    hipLaunchKernelGGL(lbp_nu_kernel, dim3(unsigned(nb)), dim3(256), 0, st, db.p, mu.p, cur, nxt, chg.p);
    std::swap(cur, nxt);
  }
  hipLaunchKernelGGL(lbp_belief_kernel, dim3(unsigned(nc)), dim3(256), 0, st, dc.p, cl->w_loc.p, cur, p);
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, st, chg.p, std::max(nb, 1), mx.p);
  HIPC(hipGetLastError());
  double out = 0.0;
  HIPC(hipMemcpyAsync(&out, mx.p, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  return iters > 0 ? out : 0.0;
}

}  // namespace tnb

using namespace tnb;

extern "C" tnb_status tnb_lbp_marginals(const tnb_clusters* cl, int32_t iters, double* d_p, int64_t p_len,
                                        double* max_change, tnb_stream stream) {
  return guarded([&] {
    if (!cl || cl->kind != KIND_CLUSTERS) fail(TNB_EINVAL, "not a clusters handle");
    if (iters < 0 || iters > 100000) fail(TNB_EINVAL, "iters must be in [0, 100000]");
    const int64_t total = cl->loc_off.back();
    if (!d_p || p_len < total) fail(TNB_EINVAL, "d_p too short");
    const double c = lbp_run(cl, iters, d_p, static_cast<hipStream_t>(stream));
    if (max_change) *max_change = c;
  });
}

extern "C" tnb_status tnb_reduce_clusters(tnb_clusters* cl, int32_t keep, int32_t iters, tnb_stream stream) {
  return guarded([&] {
    if (!cl || cl->kind != KIND_CLUSTERS) fail(TNB_EINVAL, "not a clusters handle");
    if (keep < 1) fail(TNB_EINVAL, "keep must be at least 1");
    if (iters < 0 || iters > 100000) fail(TNB_EINVAL, "iters must be in [0, 100000]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Lattice& L = cl->lat;
    const int64_t total = cl->loc_off.back();
    DevBuf<double> p(static_cast<size_t>(total));
    lbp_run(cl, iters, p.p, st);
    std::vector<int32_t> owner(static_cast<size_t>(total));
    for (int n = 0; n < L.cells(); ++n)
      for (int64_t i = cl->loc_off[size_t(n)]; i < cl->loc_off[size_t(n) + 1]; ++i) owner[size_t(i)] = n;
    DevBuf<int32_t> down;
    DevBuf<int64_t> doff;
    down.upload(owner, st);
    doff.upload(cl->loc_off, st);
    int64_t np2 = 1;
    while (np2 < total) np2 <<= 1;
    DevBuf<Cand> a(static_cast<size_t>(np2));
    hipLaunchKernelGGL(lbp_cand_kernel, dim3(nblk(np2)), dim3(256), 0, st, p.p, down.p, doff.p, total, a.p, np2);
    bitonic_sort(a.p, np2, st);
    hipLaunchKernelGGL(lbp_apply_kernel, dim3(nblk(total)), dim3(256), 0, st, a.p, doff.p, total, int(keep),
                       cl->w_loc.p, cl->w_loc32.n ? cl->w_loc32.p : nullptr);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(st));
  });
}
