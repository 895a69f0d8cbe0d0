// Beam state shared by the branch-and-bound step and the row adjoint.
#pragma once
#include "env.h"

namespace tnb {

struct Cand {
  uint64_t gkey;
  uint64_t skey;  // ascending skey = descending score
  uint32_t b;
  uint32_t x;
};

inline unsigned nblk(int64_t n, int b = 256) { return unsigned((n + b - 1) / b); }

// Ascending sort of npow2 candidates (a power of two) by (gkey, skey, b, x).
void bitonic_sort(Cand* a, int64_t npow2, hipStream_t st);
__host__ __device__ inline uint64_t score_key(double v) {
  uint64_t u;
  memcpy(&u, &v, sizeof(u));
  uint64_t asc = (u >> 63) ? ~u : (u | (1ull << 63));  // ascending in v
  return ~asc;                                          // ascending in -v
}
__host__ __device__ inline double key_score(uint64_t k) {
  uint64_t asc = ~k;
  uint64_t u = (asc >> 63) ? (asc & ~(1ull << 63)) : ~asc;
  double v;
  memcpy(&v, &u, sizeof(v));
  return v;
}


// ---- per-column geometry of the beam's row ----------------------------------
struct UpNb {
  uint32_t Bup_in_up = 0;  // spins of the upper cell facing n
  uint32_t Bn = 0;         // spins of n facing the upper cell
  int cell = -1;
  const double* W = nullptr;
  int64_t sp = 0, sq = 0;
};
struct BCol {
  int n, k;
  uint32_t PRR = 0, Bvd = 0, Bbd = 0, Bxh = 0;
  int dpi = 1, dvd = 1, dbd = 1, dxh = 1, da2 = 1;  // da2: Psi site 2c-1 a' size
  uint32_t pos_h = 0, pos_a = 0;                     // within PRR_{c-1}
  uint32_t Bleft_h = 0;                              // spins of (r,c-1) facing n
  const double* Wh = nullptr;                        // W(left, n)
  int64_t Wh_sp = 0, Wh_sq = 0;
  const double* w = nullptr;
  uint32_t cmask = 0, cval = 0;                      // clamp (x & cmask) == cval
  UpNb up[3];
  int nup = 0;
};

__device__ inline double phi_of(const BCol& c, const int32_t* __restrict__ Xb, uint32_t x) {
  double f = 1.0;
  for (int i = 0; i < c.nup; ++i) {
    const UpNb& u = c.up[i];
    f *= u.W[pext_dev(uint32_t(Xb[u.cell]), u.Bup_in_up) * u.sp + pext_dev(x, u.Bn) * u.sq];
  }
  return f;
}

// Local weight of cluster value x with the optional clamp (x & cmask) == cval.
__device__ inline double wloc(const BCol& c, uint32_t x) {
  return (x & c.cmask) == c.cval ? c.w[x] : 0.0;
}

}  // namespace tnb

struct tnb_beam {
  uint32_t kind = tnb::KIND_BEAM;
  tnb_env* env = nullptr;
  int M = 0, step = 0, npar = 1, ncell = 0;
  tnb::DevBuf<int32_t> X, Xn, rid, ridn;
  tnb::DevBuf<double> logp, logpn, L, Ln;
  int Ld = 1;
  std::vector<tnb::DevBuf<double>> R;  // R[c]: [anc][Dr(2c)][dpi_c]
  int nanc = 0;
  double pd_log = -INFINITY;
  tnb::DevBuf<double> q, score, T, u, U, V;
  tnb::DevBuf<tnb::Cand> cand, win;
  tnb::DevBuf<int> flag, dead;
  tnb::DevBuf<int64_t> pos, total, tsum;
  tnb::DevBuf<uint32_t> words, cls, km;
  tnb::DevBuf<int> kc;
  tnb::DevBuf<int32_t> cell_of, bit;
  std::vector<tnb::BCol> geo;  // of the current row
  int geo_row = -1;
  // row-moment layout of the step `lay_step` (host copy kept for the upload)
  int lay_step = -1;
  std::vector<int32_t> lay_spins, lay_edges, lay_items;
  std::vector<int> lay_off;  // per column c..C-1: first item, then the end
  tnb::DevBuf<int32_t> items;
  tnb::DevBuf<double> lam, lh, vp, qa, zs, zl, rt0, rt1;
  tnb::DevBuf<int32_t> iota;
  // final selection: exported candidates, their energies, duplicate flags
  tnb::DevBuf<int8_t> sel_states;
  tnb::DevBuf<double> sel_E;
  tnb::DevBuf<int> sel_dup;
  // droplets: per branch its partial energy and up to DMAX excitations, each
  // a sorted list of (cluster, XOR mask) pairs (at most SMAX) and its dE
  tnb_droplet_opts dopt{};
  tnb::DevBuf<double> Ep, Epn;
  tnb::DevBuf<int32_t> dcnt, dcntn, dlen, dlenn, dcell, dcelln;
  tnb::DevBuf<uint32_t> dmask, dmaskn;
  tnb::DevBuf<double> dEv, dEvn;
  tnb::DevBuf<uint32_t> bonded;  // per cluster: coupled king neighbours, bit (dr+1)*3 + (dc+1)
};

namespace tnb {

void ensure(DevBuf<double>& b, size_t n);
std::vector<BCol> beam_geom(const tnb_clusters* cl, int r);
// Right environments R[c] of every current parent for row r (per ancestor).
void row_envs(tnb_beam* bm, int r, hipStream_t st);
// q[b][x] for the current step, and T[b][b'][m] (row environments built first).
void compute_q(tnb_beam* bm, hipStream_t st);
// One right-to-left pass of the row transfer over column c (c >= 1): from
// Rin (R^{(c)}) to Rout (R^{(c-1)}), with column geometry cc.
// Rows of Rout are rescaled by their largest magnitude; when logs is not
// null the log of that factor is added to logs[anc].
// Row b of Rin and Rout belongs to the state in row b of bm->X (nb rows).
void row_step(tnb_beam* bm, const BCol& cc, int c, int nb, const double* Rin, double* Rout, double* logs,
              hipStream_t st);
// Rescale each of the nb rows of R (per entries) by its largest magnitude;
// logs[b] += log(factor) when logs is not null.
void normalise_rows(double* R, int64_t per, int nb, double* logs, hipStream_t st);
// q of the current column for every parent against right environments Rc
// (parent b reads row rid[b] of Rc; column geometry cc; T must be in place).
void q_against(tnb_beam* bm, const BCol& cc, const double* Rc, const int32_t* rid, double* q, hipStream_t st);
// Droplet bookkeeping of the step that fixed cluster n (droplets.hip): the
// kept branches sel[0 .. nsel) of the merge, with the scores of every
// candidate and (merge) the parents' boundary classes; writes the *n buffers.
void droplet_step(tnb_beam* bm, int n, uint32_t Un, bool merge, int nb, int nsel, hipStream_t st);
// Eq. (1) for K states [K][N] of +-1 (clusters.hip): edges in order, then fields, no FMA.
__global__ void ising_energy_kernel(const int8_t* __restrict__ s, int64_t K, int N, int E,
                                    const int* __restrict__ ei, const int* __restrict__ ej,
                                    const double* __restrict__ J, const double* __restrict__ h,
                                    double* __restrict__ out);

}  // namespace tnb
