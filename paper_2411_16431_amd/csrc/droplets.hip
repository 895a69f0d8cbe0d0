// Excitations above each branch from the boundary merge (Sec. III.A, Fig. 4).
//
// A group of the merge keeps its most probable member w; every other member m
// differs from w only in clusters that no longer couple to an unfixed one, so
// the difference F_m (a flip set: per cluster the XOR of the two
// configurations) is an excitation of w with dE = E(m) - E(w) of Eq. (1) over
// the fixed spins, and it keeps that energy as the branch grows.  w keeps its
// parent's excitations, gains F_m, and takes over m's parent's excitations
// F_d as F_m xor F_d with dE_m + dE_d (the two differences telescope).
//
// One workgroup per kept branch: it finds the group's best max_losers other
// members by score (a per-thread top list merged by argmax rounds), builds
// the candidate flip sets as sorted (cluster, mask) lists in LDS, filters them
// (size, energy, connectivity through couplings), sorts them by (dE, list) in
// a bitonic network and accepts them greedily at Hamming distance >=
// min_hamming.  Partial energies are table sums: the local table of the new
// cluster plus the compressed bond tables to its fixed neighbours (Eq. 3-5).
#include "beam.h"
#include "model.h"

namespace tnb {

constexpr int DMAX = 16, LMAX = 8, SMAX = 64;
constexpr int NCAND = DMAX + LMAX * (DMAX + 1);  // own, then per member its difference and its excitations
constexpr int NSORT = 256;                       // power of two >= NCAND

struct DropNbr {
  int m;
  int64_t off, sp, sq;
  uint32_t Bm, Bn;
};

struct DropStep {
  int dmax, lmax, hmin, smax, conn;
  double max_dE;
  int n, nb, C, ncell, merge, nnbr;
  int64_t d;
  uint32_t Un, FREE;
  int nf;
  const DropNbr* nbr;
  const double* E_loc;  // local table of cluster n
  const double* E_bond;
  const uint32_t* bonded;
};

// Partial energy of candidate (parent bp, value xp of cluster n).
__device__ inline double cand_energy(const DropStep& a, const int32_t* __restrict__ X, const double* __restrict__ Ep,
                                     int bp, uint32_t xp) {
  double e = a.E_loc[xp];
  for (int i = 0; i < a.nnbr; ++i) {
    const DropNbr& q = a.nbr[i];
    e += a.E_bond[q.off + int64_t(pext_dev(uint32_t(X[size_t(bp) * a.ncell + q.m]), q.Bm)) * q.sp +
                  int64_t(pext_dev(xp, q.Bn)) * q.sq];
  }
  return Ep[bp] + e;
}

// (s, b, x) ranks before (t, c, y): higher score, then lower parent, then lower value
__device__ inline bool ranks_before(double s, uint32_t b, uint32_t x, double t, uint32_t c, uint32_t y) {
  if (s != t) return s > t;
  if (b != c) return b < c;
  return x < y;
}

__global__ void __launch_bounds__(256) droplet_kernel(
    DropStep a, const Cand* __restrict__ sel, const double* __restrict__ score, const uint32_t* __restrict__ cls,
    const int32_t* __restrict__ X, const double* __restrict__ Ep, const int32_t* __restrict__ dcnt,
    const int32_t* __restrict__ dlen, const double* __restrict__ dEv, const int32_t* __restrict__ dcell,
    const uint32_t* __restrict__ dmask, double* __restrict__ Epn, int32_t* __restrict__ dcntn,
    int32_t* __restrict__ dlenn, double* __restrict__ dEvn, int32_t* __restrict__ dcelln,
    uint32_t* __restrict__ dmaskn) {
  extern __shared__ uint32_t lds[];
  int32_t* cc = reinterpret_cast<int32_t*>(lds);  // [NCAND][SMAX] clusters
  uint32_t* cm = lds + NCAND * SMAX;              // [NCAND][SMAX] masks
  __shared__ int clen[NCAND];                      // >= 0 length; -1 too long; -2 empty slot
  __shared__ double cdE[NCAND];
  __shared__ int valid[NCAND];
  __shared__ int order[NSORT];
  __shared__ double rs[256];
  __shared__ uint32_t rb[256], rx[256];
  __shared__ int rt[256];
  __shared__ uint32_t lb[LMAX], lx[LMAX];
  __shared__ int nl, acc[DMAX], nacc, reject, wcount[4], run;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.x;
  const Cand w = sel[j];
  const int b = int(w.b);
  const uint32_t x = w.x;
  const double ew = cand_energy(a, X, Ep, b, x);
  const int own = dcnt[b];
  for (int s = tid; s < NCAND; s += 256) clen[s] = -2;
  if (tid == 0) nl = 0;
  __syncthreads();

  // ---- the group's best other members (merge steps only)
  if (a.merge) {
    double ls[LMAX];
    uint32_t lbb[LMAX], lxx[LMAX];
    int cnt = 0;
    const uint32_t base = pdep_dev(pext_dev(x, a.Un), a.Un);
    const uint32_t cb = cls[b];
    for (int bp = 0; bp < a.nb; ++bp) {
      if (cls[bp] != cb) continue;  // uniform across the workgroup
      for (int f = tid; f < a.nf; f += 256) {
        const uint32_t xp = base | pdep_dev(uint32_t(f), a.FREE);
        if (bp == b && xp == x) continue;
        const double s = score[int64_t(bp) * a.d + xp];
        if (!(s > -INFINITY)) continue;
        if (cnt == a.lmax && !ranks_before(s, bp, xp, ls[cnt - 1], lbb[cnt - 1], lxx[cnt - 1])) continue;
        int p = cnt < a.lmax ? cnt++ : cnt - 1;
        while (p > 0 && ranks_before(s, bp, xp, ls[p - 1], lbb[p - 1], lxx[p - 1])) {
          ls[p] = ls[p - 1];
          lbb[p] = lbb[p - 1];
          lxx[p] = lxx[p - 1];
          --p;
        }
        ls[p] = s;
        lbb[p] = uint32_t(bp);
        lxx[p] = xp;
      }
    }
    // merge the per-thread lists: lmax rounds of a block argmax over heads
    int head = 0;
    for (int round = 0; round < a.lmax; ++round) {
      rs[tid] = head < cnt ? ls[head] : -INFINITY;
      rb[tid] = head < cnt ? lbb[head] : ~0u;
      rx[tid] = head < cnt ? lxx[head] : ~0u;
      rt[tid] = tid;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (tid < h && ranks_before(rs[tid + h], rb[tid + h], rx[tid + h], rs[tid], rb[tid], rx[tid])) {
          rs[tid] = rs[tid + h];
          rb[tid] = rb[tid + h];
          rx[tid] = rx[tid + h];
          rt[tid] = rt[tid + h];
        }
        __syncthreads();
      }
      const bool found = rs[0] > -INFINITY;
      if (found && rt[0] == tid) ++head;
      if (tid == 0 && found) {
        lb[nl] = rb[0];
        lx[nl] = rx[0];
        ++nl;
      }
      __syncthreads();
      if (!found) break;
    }
  }
  __syncthreads();
  const int nloser = nl;

  // ---- candidates: the parent's excitations
  for (int i = tid; i < own * SMAX; i += 256) {
    const int s = i / SMAX, e = i % SMAX;
    const int len = dlen[b * DMAX + s];
    if (e < len) {
      cc[s * SMAX + e] = dcell[(int64_t(b) * DMAX + s) * SMAX + e];
      cm[s * SMAX + e] = dmask[(int64_t(b) * DMAX + s) * SMAX + e];
    }
    if (e == 0) {
      clen[s] = len;
      cdE[s] = dEv[b * DMAX + s];
    }
  }
  // ---- each member's difference, by an ordered compaction over the clusters
  for (int l = 0; l < nloser; ++l) {
    const int slot = DMAX + l * (DMAX + 1);
    const int bp = int(lb[l]);
    const uint32_t xp = lx[l];
    if (tid == 0) run = 0;
    __syncthreads();
    for (int c0 = 0; c0 <= a.n; c0 += 256) {
      const int c = c0 + tid;
      uint32_t m = 0;
      if (c < a.n) m = uint32_t(X[size_t(bp) * a.ncell + c] ^ X[size_t(b) * a.ncell + c]);
      else if (c == a.n) m = xp ^ x;
      const unsigned long long bal = __ballot(m != 0);
      if (lane == 0) wcount[wv] = __popcll(bal);
      __syncthreads();
      int pos = run;
      for (int q = 0; q < wv; ++q) pos += wcount[q];
      pos += __popcll(bal & ((1ull << lane) - 1ull));
      if (m != 0 && pos < SMAX) {
        cc[slot * SMAX + pos] = c;
        cm[slot * SMAX + pos] = m;
      }
      __syncthreads();
      if (tid == 0) run += wcount[0] + wcount[1] + wcount[2] + wcount[3];
      __syncthreads();
    }
    if (tid == 0) {
      clen[slot] = run <= SMAX ? run : -1;
      cdE[slot] = cand_energy(a, X, Ep, bp, xp) - ew;
    }
    __syncthreads();
  }
  // ---- members' excitations composed with their difference
  for (int p = tid; p < nloser * DMAX; p += 256) {
    const int l = p / DMAX, dd = p % DMAX;
    const int bp = int(lb[l]);
    if (dd >= dcnt[bp]) continue;
    const int bs = DMAX + l * (DMAX + 1), slot = bs + 1 + dd;
    const int la = clen[bs];
    if (la < 0) {
      clen[slot] = -1;
      continue;
    }
    const int lbn = dlen[bp * DMAX + dd];
    const int32_t* gc = dcell + (int64_t(bp) * DMAX + dd) * SMAX;
    const uint32_t* gm = dmask + (int64_t(bp) * DMAX + dd) * SMAX;
    int i1 = 0, i2 = 0, o = 0;
    bool over = false;
    while (i1 < la || i2 < lbn) {
      int cell;
      uint32_t m;
      if (i2 >= lbn || (i1 < la && cc[bs * SMAX + i1] < gc[i2])) {
        cell = cc[bs * SMAX + i1];
        m = cm[bs * SMAX + i1];
        ++i1;
      } else if (i1 >= la || gc[i2] < cc[bs * SMAX + i1]) {
        cell = gc[i2];
        m = gm[i2];
        ++i2;
      } else {
        cell = gc[i2];
        m = cm[bs * SMAX + i1] ^ gm[i2];
        ++i1;
        ++i2;
      }
      if (m == 0) continue;
      if (o == SMAX) {
        over = true;
        break;
      }
      cc[slot * SMAX + o] = cell;
      cm[slot * SMAX + o] = m;
      ++o;
    }
    clen[slot] = over ? -1 : o;
    cdE[slot] = cdE[bs] + dEv[bp * DMAX + dd];
  }
  __syncthreads();
  // ---- filters: size, energy, one connected set of coupled clusters
  for (int s = tid; s < NCAND; s += 256) {
    const int len = clen[s];
    bool ok = len >= 1 && len <= a.smax && cdE[s] <= a.max_dE;
    if (ok && a.conn) {
      unsigned long long seen = 1ull, done = 0ull;
      while (seen != done) {
        const int i = __ffsll(static_cast<long long>(seen & ~done)) - 1;
        done |= 1ull << i;
        const int ci = cc[s * SMAX + i];
        const int ri = ci / a.C, ki = ci % a.C;
        const uint32_t nbm = a.bonded[ci];
        for (int q = 0; q < len; ++q) {
          if (seen >> q & 1ull) continue;
          const int cq = cc[s * SMAX + q];
          const int dr = cq / a.C - ri, dc = cq % a.C - ki;
          if (dr >= -1 && dr <= 1 && dc >= -1 && dc <= 1 && (nbm >> ((dr + 1) * 3 + (dc + 1)) & 1u)) seen |= 1ull << q;
        }
      }
      ok = __popcll(seen) == len;
    }
    valid[s] = ok ? 1 : 0;
  }
  for (int i = tid; i < NSORT; i += 256) order[i] = i < NCAND ? i : -1;
  __syncthreads();
  // ---- order: valid first, then dE, then the (cluster, mask) list, then slot
  auto before = [&](int p, int q) -> bool {
    const bool vp = p >= 0 && valid[p], vq = q >= 0 && valid[q];
    if (vp != vq) return vp;
    if (!vp) return p >= 0 && (q < 0 || p < q);
    if (cdE[p] != cdE[q]) return cdE[p] < cdE[q];
    const int lp = clen[p], lq = clen[q];
    for (int e = 0; e < lp && e < lq; ++e) {
      const int c1 = cc[p * SMAX + e], c2 = cc[q * SMAX + e];
      if (c1 != c2) return c1 < c2;
      const uint32_t m1 = cm[p * SMAX + e], m2 = cm[q * SMAX + e];
      if (m1 != m2) return m1 < m2;
    }
    if (lp != lq) return lp < lq;
    return p < q;
  };
  for (int k = 2; k <= NSORT; k <<= 1)
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      const int i = tid, l = i ^ jj;
      if (l > i) {
        const bool up = (i & k) == 0;
        const int oi = order[i], ol = order[l];
        if (up ? before(ol, oi) : before(oi, ol)) {
          order[i] = ol;
          order[l] = oi;
        }
      }
      __syncthreads();
    }
  // ---- greedy acceptance at Hamming distance >= min_hamming
  if (tid == 0) nacc = 0;
  __syncthreads();
  for (int p = 0; p < NCAND; ++p) {
    const int s = order[p];
    if (s < 0 || !valid[s] || nacc >= a.dmax) break;  // uniform
    if (tid == 0) reject = 0;
    __syncthreads();
    if (tid < nacc) {
      const int t = acc[tid];
      const int l1 = clen[s], l2 = clen[t];
      int i1 = 0, i2 = 0, hd = 0;
      while (i1 < l1 || i2 < l2) {
        if (i2 >= l2 || (i1 < l1 && cc[s * SMAX + i1] < cc[t * SMAX + i2])) {
          hd += __popc(cm[s * SMAX + i1]);
          ++i1;
        } else if (i1 >= l1 || cc[t * SMAX + i2] < cc[s * SMAX + i1]) {
          hd += __popc(cm[t * SMAX + i2]);
          ++i2;
        } else {
          hd += __popc(cm[s * SMAX + i1] ^ cm[t * SMAX + i2]);
          ++i1;
          ++i2;
        }
      }
      if (hd < a.hmin) atomicOr(&reject, 1);
    }
    __syncthreads();
    if (tid == 0 && !reject) acc[nacc++] = s;
    __syncthreads();
  }
  // ---- the branch's new excitations and partial energy
  const int na = nacc;
  for (int i = tid; i < na * SMAX; i += 256) {
    const int q = i / SMAX, e = i % SMAX;
    const int s = acc[q];
    const int64_t o = (int64_t(j) * DMAX + q) * SMAX + e;
    if (e < clen[s]) {
      dcelln[o] = cc[s * SMAX + e];
      dmaskn[o] = cm[s * SMAX + e];
    }
    if (e == 0) {
      dlenn[j * DMAX + q] = clen[s];
      dEvn[j * DMAX + q] = cdE[s];
    }
  }
  if (tid == 0) {
    dcntn[j] = na;
    Epn[j] = ew;
  }
}

// States of branch i with each of its first cnt excitations applied.
__global__ void droplet_export_kernel(const int32_t* __restrict__ X, int ncell, int nfixed, int i,
                                      const int32_t* __restrict__ cell_of, const int32_t* __restrict__ bit, int N,
                                      int cnt, const int32_t* __restrict__ dlen, const int32_t* __restrict__ dcell,
                                      const uint32_t* __restrict__ dmask, const double* __restrict__ dEv,
                                      int8_t* __restrict__ out, double* __restrict__ dE) {
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= int64_t(cnt) * N) return;
  const int q = int(idx / N), s = int(idx % N);
  const int n = cell_of[s];
  int8_t v = 0;
  if (n < nfixed) {
    uint32_t xv = uint32_t(X[size_t(i) * ncell + n]);
    const int len = dlen[i * DMAX + q];
    const int64_t o = (int64_t(i) * DMAX + q) * SMAX;
    for (int e = 0; e < len; ++e)
      if (dcell[o + e] == n) xv ^= dmask[o + e];
    v = (xv >> bit[s]) & 1u ? int8_t(1) : int8_t(-1);
  }
  out[idx] = v;
  if (s == 0) dE[q] = dEv[i * DMAX + q];
}

static void ensure_i(DevBuf<int32_t>& b, size_t n) {
  if (b.n < n) b.alloc(n);
}
static void ensure_u(DevBuf<uint32_t>& b, size_t n) {
  if (b.n < n) b.alloc(n);
}

void droplet_step(tnb_beam* bm, int n, uint32_t Un, bool merge, int nb, int nsel, hipStream_t st) {
  const tnb_clusters* cl = bm->env->cl;
  const Lattice& L = cl->lat;
  const int r = n / L.C, c = n % L.C;
  std::vector<DropNbr> nv;
  for (int dr = -1; dr <= 0; ++dr)
    for (int dc = -1; dc <= 1; ++dc) {
      const int m = L.cell(r + dr, c + dc);
      if (m < 0 || m >= n || !cl->B(m, n)) continue;
      auto it = cl->bond_of.find(int64_t(m) * L.cells() + n);
      if (it == cl->bond_of.end()) continue;
      const auto& bd = cl->bonds[it->second];
      nv.push_back(DropNbr{m, bd.off, bd.cols, 1, cl->B(m, n), cl->B(n, m)});
    }
  DevBuf<DropNbr> dn;
  if (!nv.empty()) dn.upload(nv, st);
  const int k = L.k[n];
  const uint32_t full = k ? ((k == 32) ? ~0u : ((1u << k) - 1u)) : 0u;
  DropStep a{};
  a.dmax = bm->dopt.max_droplets;
  a.lmax = bm->dopt.max_losers;
  a.hmin = bm->dopt.min_hamming;
  a.smax = bm->dopt.max_cells;
  a.conn = bm->dopt.connected_only ? 1 : 0;
  a.max_dE = bm->dopt.max_dE;
  a.n = n;
  a.nb = nb;
  a.C = L.C;
  a.ncell = bm->ncell;
  a.merge = merge ? 1 : 0;
  a.nnbr = int(nv.size());
  a.d = int64_t(1) << k;
  a.Un = Un;
  a.FREE = full & ~Un;
  a.nf = 1 << popcount32(a.FREE);
  a.nbr = nv.empty() ? nullptr : dn.p;
  a.E_loc = cl->E_loc.p + cl->loc_off[n];
  a.E_bond = cl->E_bond.p;
  a.bonded = bm->bonded.p;
  const size_t M = size_t(bm->M);
  ensure(bm->Epn, M);
  ensure_i(bm->dcntn, M);
  ensure_i(bm->dlenn, M * DMAX);
  ensure(bm->dEvn, M * DMAX);
  ensure_i(bm->dcelln, M * DMAX * SMAX);
  ensure_u(bm->dmaskn, M * DMAX * SMAX);
  const size_t shm = size_t(2) * NCAND * SMAX * sizeof(uint32_t);
  HIPC(hipFuncSetAttribute(reinterpret_cast<const void*>(droplet_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                           int(shm)));
  KTimer _t("droplets", st, 0.0, 0.0);
  hipLaunchKernelGGL(droplet_kernel, dim3(unsigned(nsel)), dim3(256), shm, st, a, bm->win.p, bm->score.p,
                     merge ? bm->cls.p : nullptr, bm->X.p, bm->Ep.p, bm->dcnt.p, bm->dlen.p, bm->dEv.p, bm->dcell.p,
                     bm->dmask.p, bm->Epn.p, bm->dcntn.p, bm->dlenn.p, bm->dEvn.p, bm->dcelln.p, bm->dmaskn.p);
  HIPC(hipGetLastError());
  HIPC(hipStreamSynchronize(st));  // dn is freed on return
}

}  // namespace tnb

using namespace tnb;

extern "C" tnb_status tnb_beam_droplets_enable(tnb_beam* bm, const tnb_droplet_opts* opts) {
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (bm->step != 0) fail(TNB_EINVAL, "droplets must be switched on before the first step");
    if (!opts || opts->max_droplets == 0) {
      bm->dopt = tnb_droplet_opts{};
      return;
    }
    const tnb_droplet_opts& o = *opts;
    if (o.max_droplets < 0 || o.max_droplets > DMAX) fail(TNB_EINVAL, "max_droplets must be in [0, 16]");
    if (o.max_losers < 1 || o.max_losers > LMAX) fail(TNB_EINVAL, "max_losers must be in [1, 8]");
    if (o.max_cells < 1 || o.max_cells > SMAX) fail(TNB_EINVAL, "max_cells must be in [1, 64]");
    if (o.min_hamming < 1) fail(TNB_EINVAL, "min_hamming must be at least 1");
    if (std::isnan(o.max_dE)) fail(TNB_EINVAL, "max_dE is NaN");
    const tnb_clusters* cl = bm->env->cl;
    const Lattice& L = cl->lat;
    const size_t M = size_t(bm->M);
    ensure(bm->Ep, M);
    ensure_i(bm->dcnt, M);
    ensure_i(bm->dlen, M * DMAX);
    ensure(bm->dEv, M * DMAX);
    ensure_i(bm->dcell, M * DMAX * SMAX);
    ensure_u(bm->dmask, M * DMAX * SMAX);
    HIPC(hipMemset(bm->Ep.p, 0, sizeof(double) * M));
    HIPC(hipMemset(bm->dcnt.p, 0, sizeof(int32_t) * M));
    std::vector<uint32_t> bonded(size_t(L.cells()), 0u);
    for (int m = 0; m < L.cells(); ++m)
      for (int dr = -1; dr <= 1; ++dr)
        for (int dc = -1; dc <= 1; ++dc) {
          const int q = L.cell(m / L.C + dr, m % L.C + dc);
          if (q >= 0 && q != m && cl->B(m, q)) bonded[size_t(m)] |= 1u << ((dr + 1) * 3 + (dc + 1));
        }
    bm->bonded.upload(bonded, nullptr);
    HIPC(hipDeviceSynchronize());
    bm->dopt = o;
  });
}

extern "C" tnb_status tnb_beam_droplets(const tnb_beam* bm, int32_t i, int32_t max_count, int8_t* d_states,
                                        double* d_dE, int32_t* count, tnb_stream stream) {
  return guarded([&] {
    if (!bm || bm->kind != KIND_BEAM) fail(TNB_EINVAL, "not a beam handle");
    if (bm->dopt.max_droplets == 0) fail(TNB_EINVAL, "droplet bookkeeping is off");
    if (i < 0 || i >= bm->npar) fail(TNB_EINVAL, "branch index out of range");
    if (max_count < 0 || (max_count > 0 && (!d_states || !d_dE))) fail(TNB_EINVAL, "bad output");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int32_t have = 0;
    HIPC(hipMemcpyAsync(&have, bm->dcnt.p + i, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    const int cnt = std::min(max_count, have);
    const Lattice& L = bm->env->cl->lat;
    if (cnt > 0)
      hipLaunchKernelGGL(droplet_export_kernel, dim3(nblk(int64_t(cnt) * L.N)), dim3(256), 0, st, bm->X.p,
                         bm->ncell, bm->step, i, bm->cell_of.p, bm->bit.p, L.N, cnt, bm->dlen.p, bm->dcell.p,
                         bm->dmask.p, bm->dEv.p, d_states, d_dE);
    HIPC(hipGetLastError());
    if (count) *count = cnt;
    HIPC(hipStreamSynchronize(st));
  });
}
