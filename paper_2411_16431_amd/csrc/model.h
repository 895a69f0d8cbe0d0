// Device-resident clustered model (Eq. 3-6) shared by the contraction and
// beam code.
#pragma once
#include <map>

#include "common.h"

struct tnb_clusters {
  uint32_t kind = tnb::KIND_CLUSTERS;
  tnb::Lattice lat;
  double beta = 0.0;
  // B(m, n): mask of the spins of m coupled to king neighbour n, indexed by
  // m*9 + (dr+1)*3 + (dc+1).
  std::vector<uint32_t> maskv;
  // local tables, concatenated over clusters
  std::vector<int64_t> loc_off;
  tnb::DevBuf<double> E_loc, w_loc;
  tnb::DevBuf<float> w_loc32;  // the weights rounded to FP32 (FP32 contractions)
  std::vector<double> E_min_loc;
  // bond tables of unordered neighbour pairs m < n, [p of m][q of n]
  struct Bond {
    int m, n;
    int64_t off;
    int rows, cols;
    double Emin;
  };
  std::vector<Bond> bonds;
  std::map<int64_t, int> bond_of;  // m*cells + n (m < n) -> index
  tnb::DevBuf<double> E_bond, W_bond;
  tnb::DevBuf<float> W_bond32;
  double shift = 0.0;  // sum over all tables of -beta * min energy
  // the instance on the device (energies of returned states, Eq. 1)
  tnb::DevBuf<int32_t> d_ei, d_ej;
  tnb::DevBuf<double> d_J, d_h;

  uint32_t B(int m, int n) const {
    if (m < 0 || n < 0) return 0;
    int C = lat.C;
    int dr = n / C - m / C, dc = n % C - m % C;
    if (dr < -1 || dr > 1 || dc < -1 || dc > 1 || (dr == 0 && dc == 0)) return 0;
    return maskv[size_t(m) * 9 + (dr + 1) * 3 + (dc + 1)];
  }
  int k(int n) const { return n < 0 ? 0 : lat.k[n]; }
  // Weight table W(p, q) = ptr[p*sp + q*sq] for the ordered pair (m, n),
  // p = P^{mn} x_m, q = P^{nm} x_n.  Returns false when m, n are uncoupled.
  bool weight_view(int m, int n, const double** ptr, int64_t* sp, int64_t* sq) const {
    if (m < 0 || n < 0) return false;
    int a = m < n ? m : n, b = m < n ? n : m;
    auto it = bond_of.find(int64_t(a) * lat.cells() + b);
    if (it == bond_of.end()) return false;
    const Bond& bd = bonds[it->second];
    *ptr = W_bond.p + bd.off;
    if (m < n) { *sp = bd.cols; *sq = 1; }
    else { *sp = 1; *sq = bd.cols; }
    return true;
  }
  // The FP32 copy of the same table, same strides.
  const float* weight32(int m, int n) const {
    if (m < 0 || n < 0) return nullptr;
    int a = m < n ? m : n, b = m < n ? n : m;
    auto it = bond_of.find(int64_t(a) * lat.cells() + b);
    if (it == bond_of.end()) return nullptr;
    return W_bond32.p + bonds[it->second].off;
  }
};
