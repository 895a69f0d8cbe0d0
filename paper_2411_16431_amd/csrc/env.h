// Boundary MPSs of the lower half-lattice (device resident).
#pragma once
#include "linalg.h"
#include "model.h"

namespace tnb {

// One MPS tensor, layout [sigma][alpha][beta] (physical index slowest, so a
// gather by sigma reads one contiguous Dl x Dr matrix).
struct Site {
  DevBuf<double> data;
  int dl = 1, d = 1, dr = 1;
  size_t size() const { return size_t(dl) * d * dr; }
};

struct Mps {
  std::vector<Site> sites;
  double logscale = 0.0;  // Psi = exp(logscale) * (stored tensors)
};

// Masks and dimensions of the row-r MPO and of the boundary MPSs around it.
struct RowGeom {
  struct Col {
    int n = -1, up = -1;
    int k = 0;
    uint32_t PL = 0, PR = 0, Bup = 0, Bdn = 0;
    int dL = 1, dR = 1, du = 1, dv = 1, dvd = 1;  // dv: Psi_r site 2c; dvd: Psi_{r+1} site 2c
    const double* w = nullptr;
    const float* w32 = nullptr;  // the same weights in FP32
    const double* Wv = nullptr;  // W(v, u) = Wv[v*Wv_sp + u*Wv_sq]
    int64_t Wv_sp = 0, Wv_sq = 0;
  };
  struct Med {
    int da = 1, db = 1, da2 = 1, db2 = 1;  // up (Psi_r) and down (Psi_{r+1}) splits
    int dR = 1, dL = 1, dld = 1, drd = 1;
    uint32_t pos_h_rho = 0, pos_h_ell = 0;   // positions (within rho / l) of the horizontal bits
    uint32_t pos_d_rho = 0, pos_d_ell = 0;   // ... of the bits facing the upper diagonal cells
    uint32_t pos_a2 = 0, pos_b2 = 0;         // ... of the bits facing the lower diagonal cells
    const double* Wh = nullptr;
    const float* Wh32 = nullptr;             // the same table in FP32
    int64_t Wh_sp = 0, Wh_sq = 0;
    const double* Wdr = nullptr;             // W(a, l_d)
    int64_t Wdr_sp = 0, Wdr_sq = 0;
    const double* Wdl = nullptr;             // W(b, rho_d)
    int64_t Wdl_sp = 0, Wdl_sq = 0;
  };
  int r = 0;
  std::vector<Col> col;
  std::vector<Med> med;
};

RowGeom row_geom(const tnb_clusters* cl, int r);
std::vector<int> phys_dims(const tnb_clusters* cl, int r);  // of Psi_r (2C-1 sites)

}  // namespace tnb

struct tnb_env {
  uint32_t kind = tnb::KIND_ENV;
  tnb_clusters* cl = nullptr;
  tnb_env_opts opts{};
  std::vector<tnb::Mps> psi;  // psi[r], r = 1..R (psi[0] unused)
  double logZ = 0.0;
  int zsign = 1;  // sign of the approximate Z (top-row contraction)
  tnb::la::Scratch ws;
};
