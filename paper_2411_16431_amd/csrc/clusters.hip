// Cluster tables (Eq. 3-5), Boltzmann weights (Eq. 6) and Ising energies
// (Eq. 1).  All tables are written by one thread per entry with coalesced
// stores; these kernels are bound by the HBM write of the tables.
#include <algorithm>
#include <memory>
#include <mutex>
#include <numeric>

#include "model.h"

namespace tnb {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }

Lattice validate_instance(const tnb_instance* inst) {
  if (!inst) fail(TNB_EINVAL, "instance is NULL");
  Lattice L;
  L.N = inst->n_spins;
  L.E = inst->n_edges;
  L.R = inst->rows;
  L.C = inst->cols;
  if (L.N < 1 || L.E < 0 || L.R < 1 || L.C < 1) fail(TNB_EINVAL, "empty or negative instance sizes");
  if (int64_t(L.R) * L.C > (1 << 20)) fail(TNB_EUNSUPPORTED, "lattice larger than 2^20 clusters");
  if ((L.E && (!inst->edge_i || !inst->edge_j || !inst->J)) || !inst->h || !inst->cell_of)
    fail(TNB_EINVAL, "instance array is NULL");
  L.ei.assign(inst->edge_i, inst->edge_i + L.E);
  L.ej.assign(inst->edge_j, inst->edge_j + L.E);
  L.J.assign(inst->J, inst->J + L.E);
  L.h.assign(inst->h, inst->h + L.N);
  L.cell_of.assign(inst->cell_of, inst->cell_of + L.N);
  for (int e = 0; e < L.E; ++e) {
    if (L.ei[e] < 0 || L.ej[e] >= L.N || L.ei[e] >= L.ej[e])
      fail(TNB_EINVAL, "edge " + std::to_string(e) + " is not 0 <= i < j < n_spins");
    if (e && (int64_t(L.ei[e - 1]) * L.N + L.ej[e - 1] >= int64_t(L.ei[e]) * L.N + L.ej[e]))
      fail(TNB_EINVAL, "edges are not sorted by (i, j) or contain duplicates");
    if (!std::isfinite(L.J[e])) fail(TNB_EINVAL, "non-finite coupling J");
  }
  for (int i = 0; i < L.N; ++i) {
    if (!std::isfinite(L.h[i])) fail(TNB_EINVAL, "non-finite field h");
    if (L.cell_of[i] < 0 || L.cell_of[i] >= L.R * L.C) fail(TNB_EINVAL, "cell_of out of range");
  }
  L.spins.assign(L.cells(), {});
  L.bit.assign(L.N, 0);
  for (int i = 0; i < L.N; ++i) {
    auto& s = L.spins[L.cell_of[i]];
    L.bit[i] = int(s.size());
    s.push_back(i);
  }
  L.k.resize(L.cells());
  for (int n = 0; n < L.cells(); ++n) {
    L.k[n] = int(L.spins[n].size());
    if (L.k[n] > 24) fail(TNB_EUNSUPPORTED, "cluster with more than 24 spins");
  }
  for (int e = 0; e < L.E; ++e) {
    int a = L.cell_of[L.ei[e]], b = L.cell_of[L.ej[e]];
    if (std::abs(a / L.C - b / L.C) > 1 || std::abs(a % L.C - b % L.C) > 1)
      fail(TNB_EINVAL, "edge " + std::to_string(e) + " joins clusters that are not king neighbours");
  }
  return L;
}

// ---------------------------------------------------------------- kernels
// E_n[x]: intra-cluster couplings in edge order, then fields in spin order,
// each term +-J (exact) added with round-to-nearest; no contraction.
__global__ void local_energy_kernel(const int64_t* __restrict__ off, const int* __restrict__ kk,
                                    const int* __restrict__ eoff, const int* __restrict__ ebi,
                                    const int* __restrict__ ebj, const double* __restrict__ eJ,
                                    const int* __restrict__ foff, const double* __restrict__ fh,
                                    double* __restrict__ E) {
  const int n = blockIdx.y;
  const int k = kk[n];
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 ? x != 0 : x >= (1u << k)) return;
  double acc = 0.0;
  for (int e = eoff[n]; e < eoff[n + 1]; ++e) {
    const double sign = (((x >> ebi[e]) ^ (x >> ebj[e])) & 1u) ? -1.0 : 1.0;
    acc = __dadd_rn(acc, __dmul_rn(eJ[e], sign));
  }
  for (int b = 0; b < foff[n + 1] - foff[n]; ++b) {
    const double s = ((x >> b) & 1u) ? 1.0 : -1.0;
    acc = __dadd_rn(acc, __dmul_rn(fh[foff[n] + b], s));
  }
  E[off[n] + x] = acc;
}

// Ebar^{mn}[p, q] over the edges between m and n in edge order.
__global__ void bond_energy_kernel(const int64_t* __restrict__ off, const int* __restrict__ rows,
                                   const int* __restrict__ cols, const int* __restrict__ eoff,
                                   const int* __restrict__ pp, const int* __restrict__ pq,
                                   const double* __restrict__ eJ, double* __restrict__ E) {
  const int t = blockIdx.y;
  const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t total = int64_t(rows[t]) * cols[t];
  if (idx >= total) return;
  const uint32_t p = uint32_t(idx / cols[t]), q = uint32_t(idx % cols[t]);
  double acc = 0.0;
  for (int e = eoff[t]; e < eoff[t + 1]; ++e) {
    const double sign = (((p >> pp[e]) ^ (q >> pq[e])) & 1u) ? -1.0 : 1.0;
    acc = __dadd_rn(acc, __dmul_rn(eJ[e], sign));
  }
  E[off[t] + idx] = acc;
}

// min over each table; one 256-thread block per table, fixed reduction tree.
__global__ void table_min_kernel(const double* __restrict__ E, const int64_t* __restrict__ off,
                                 const int64_t* __restrict__ len, double* __restrict__ out) {
  __shared__ double red[256];
  const int t = blockIdx.x;
  double m = INFINITY;
  for (int64_t i = threadIdx.x; i < len[t]; i += blockDim.x) m = fmin(m, E[off[t] + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[t] = red[0];
}

// w = exp(-beta (E - Emin)) for every table entry.
__global__ void boltzmann_kernel(const double* __restrict__ E, double* __restrict__ w,
                                 const int64_t* __restrict__ off, const int64_t* __restrict__ len,
                                 const double* __restrict__ Emin, double beta) {
  const int t = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= len[t]) return;
  const double d = __dsub_rn(E[off[t] + i], Emin[t]);
  w[off[t] + i] = exp(__dmul_rn(-beta, d));
}

__global__ void ising_energy_kernel(const int8_t* __restrict__ s, int64_t K, int N, int E,
                                    const int* __restrict__ ei, const int* __restrict__ ej,
                                    const double* __restrict__ J, const double* __restrict__ h,
                                    double* __restrict__ out) {
  const int64_t kx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (kx >= K) return;
  const int8_t* st = s + kx * N;
  double acc = 0.0;
  for (int e = 0; e < E; ++e) {
    const double ss = double(int(st[ei[e]]) * int(st[ej[e]]));
    acc = __dadd_rn(acc, __dmul_rn(J[e], ss));
  }
  for (int i = 0; i < N; ++i) acc = __dadd_rn(acc, __dmul_rn(h[i], double(st[i])));
  out[kx] = acc;
}

// ---- device memory: hipMalloc or the caller's allocator ---------------------
// Installed allocators are kept for the life of the process (blocks hold a
// pointer to the one that gave them), so replacing one never strands a block.
static std::mutex g_alloc_mu;
static std::vector<std::unique_ptr<Allocator>> g_allocators;
static const Allocator* g_current = nullptr;

const Allocator* current_allocator() {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  return g_current;
}

void* dev_alloc(size_t bytes, const Allocator** owner) {
  const Allocator* a = current_allocator();
  *owner = a;
  void* p = nullptr;
  if (!a) {
    HIPC(hipMalloc(&p, bytes));
    return p;
  }
  p = a->alloc(bytes, a->user);
  if (!p) fail(TNB_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
  return p;
}

void dev_free(void* p, const Allocator* owner) {
  if (!owner) (void)hipFree(p);
  else owner->release(p, owner->user);
}

static bool g_prof = false;
static std::vector<ProfRec> g_recs;
static std::mutex g_prof_mu;  // calls on several host threads record concurrently
// Free timing events per device (events belong to the device that was
// current when they were created).  Records return theirs when cleared.
constexpr int kPoolDevices = 64;
static std::vector<hipEvent_t> g_pool[kPoolDevices];
static std::vector<int> g_rec_dev;  // device of each record's events
bool prof_on() { return g_prof; }
void prof_push(const ProfRec& r) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(g_prof_mu);
  g_recs.push_back(r);
  g_rec_dev.push_back(dev);
}
hipEvent_t prof_event() {
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= kPoolDevices) fail(TNB_EDEVICE, "device index out of range");
  {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    if (!g_pool[dev].empty()) {
      hipEvent_t e = g_pool[dev].back();
      g_pool[dev].pop_back();
      return e;
    }
  }
  hipEvent_t e;
  HIPC(hipEventCreate(&e));
  return e;
}

// A weight of 1 in device memory (the site weight of a cluster's empty side):
// a constant of the code object, one copy per device.
__device__ double g_unit64 = 1.0;
__device__ float g_unit32 = 1.0f;

// Address of a device symbol on the current device, looked up once per device.
template <class T, class Get>
static const T* per_device_symbol(Get get) {
  static std::mutex mu;
  static const T* ptr[64] = {nullptr};
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(TNB_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    HIPC(get(&p));
    ptr[dev] = static_cast<const T*>(p);
  }
  return ptr[dev];
}

const double* unit_weight() {
  return per_device_symbol<double>([](void** p) { return hipGetSymbolAddress(p, HIP_SYMBOL(g_unit64)); });
}
const float* unit_weight32() {
  return per_device_symbol<float>([](void** p) { return hipGetSymbolAddress(p, HIP_SYMBOL(g_unit32)); });
}

__global__ void to_f32_kernel(const double* __restrict__ x, int64_t n, float* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = float(x[i]);
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace tnb

using namespace tnb;

extern "C" const char* tnb_last_error(void) { return tnb::last_error(); }

extern "C" tnb_status tnb_energies(const tnb_instance* inst, const int8_t* d_states, int64_t K,
                                   double* d_E, tnb_stream stream) {
  return guarded([&] {
    Lattice L = validate_instance(inst);
    if (K < 0) fail(TNB_EINVAL, "K < 0");
    if (K == 0) return;
    if (!d_states || !d_E) fail(TNB_EINVAL, "device pointer is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    DevBuf<int> ei, ej;
    DevBuf<double> J, h;
    ei.upload(L.ei, s);
    ej.upload(L.ej, s);
    J.upload(L.J, s);
    h.upload(L.h, s);
    hipLaunchKernelGGL(ising_energy_kernel, dim3(unsigned(cdiv(K, 128))), dim3(128), 0, s, d_states,
                       K, L.N, L.E, ei.p, ej.p, J.p, h.p, d_E);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));  // temporaries are freed on return
  });
}

// ---- Eq. (1) without device allocation -----------------------------------
// Staging area for the instance (J, h, edge lists) of tnb_energies_noalloc:
// a file-scope device array, one copy per GPU, held for the life of the
// process.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
namespace tnb {
namespace {
constexpr size_t kStageBytes = size_t(2) << 20;  // 2 MiB
__device__ __align__(256) double scratch[kStageBytes / sizeof(double)];

std::mutex g_stage_mu;
char* g_stage[64] = {nullptr};

char* stage_area() {
  int dev = 0;
  HIPC(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(TNB_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_stage_mu);
  if (!g_stage[dev]) {
    void* p = nullptr;
    HIPC(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_stage[dev] = static_cast<char*>(p);
  }
  return g_stage[dev];
}
}  // namespace
}  // namespace tnb

extern "C" tnb_status tnb_energies_noalloc(const tnb_instance* inst, const int8_t* d_states, int64_t K,
                                           double* d_E, tnb_stream stream) {
  return guarded([&] {
    Lattice L = validate_instance(inst);
    if (K < 0) fail(TNB_EINVAL, "K < 0");
    const size_t bytes = 16 * size_t(L.E) + 8 * size_t(L.N);
    if (bytes > kStageBytes)
      fail(TNB_EUNSUPPORTED, "instance exceeds the 2 MiB staging area (16 bytes per edge + 8 per spin)");
    if (K == 0) return;
    if (!d_states || !d_E) fail(TNB_EINVAL, "device pointer is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = stage_area();
    double* J = reinterpret_cast<double*>(base);
    double* h = J + L.E;
    int* ei = reinterpret_cast<int*>(h + L.N);
    int* ej = ei + L.E;
    if (L.E) {
      HIPC(hipMemcpyAsync(J, L.J.data(), size_t(L.E) * sizeof(double), hipMemcpyHostToDevice, s));
      HIPC(hipMemcpyAsync(ei, L.ei.data(), size_t(L.E) * sizeof(int), hipMemcpyHostToDevice, s));
      HIPC(hipMemcpyAsync(ej, L.ej.data(), size_t(L.E) * sizeof(int), hipMemcpyHostToDevice, s));
    }
    if (L.N) HIPC(hipMemcpyAsync(h, L.h.data(), size_t(L.N) * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(ising_energy_kernel, dim3(unsigned(cdiv(K, 128))), dim3(128), 0, s, d_states, K, L.N, L.E,
                       ei, ej, J, h, d_E);
    HIPC(hipGetLastError());
    HIPC(hipStreamSynchronize(s));  // the host copies of the instance end with this call
  });
}

extern "C" tnb_status tnb_build_clusters(const tnb_instance* inst, double beta, tnb_stream stream,
                                         tnb_clusters** out) {
  return guarded([&] {
    if (!out) fail(TNB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!(beta >= 0.0) || !std::isfinite(beta)) fail(TNB_EINVAL, "beta must be finite and >= 0");
    auto cl = std::make_unique<tnb_clusters>();
    cl->lat = validate_instance(inst);
    cl->beta = beta;
    const Lattice& L = cl->lat;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int ncell = L.cells();
    // projector masks B(m, n) (Eq. 5)
    cl->maskv.assign(size_t(ncell) * 9, 0u);
    auto dir = [&](int m, int n) { return (n / L.C - m / L.C + 1) * 3 + (n % L.C - m % L.C + 1); };
    std::vector<int> intra_cnt(ncell, 0);
    std::map<int64_t, std::vector<int>> inter;
    for (int e = 0; e < L.E; ++e) {
      int i = L.ei[e], j = L.ej[e];
      int a = L.cell_of[i], b = L.cell_of[j];
      if (a == b) continue;
      cl->maskv[size_t(a) * 9 + dir(a, b)] |= 1u << L.bit[i];
      cl->maskv[size_t(b) * 9 + dir(b, a)] |= 1u << L.bit[j];
      inter[int64_t(std::min(a, b)) * ncell + std::max(a, b)].push_back(e);
    }
    // local tables (a1)
    std::vector<int> kk(L.k.begin(), L.k.end()), eoff(ncell + 1, 0), foff(ncell + 1, 0), ebi, ebj;
    std::vector<double> eJ, fh;
    cl->loc_off.assign(ncell + 1, 0);
    std::vector<std::vector<int>> intra(ncell);
    for (int e = 0; e < L.E; ++e)
      if (L.cell_of[L.ei[e]] == L.cell_of[L.ej[e]]) intra[L.cell_of[L.ei[e]]].push_back(e);
    int maxk = 0;
    for (int n = 0; n < ncell; ++n) {
      for (int e : intra[n]) {
        ebi.push_back(L.bit[L.ei[e]]);
        ebj.push_back(L.bit[L.ej[e]]);
        eJ.push_back(L.J[e]);
      }
      eoff[n + 1] = int(ebi.size());
      for (int i : L.spins[n]) fh.push_back(L.h[i]);
      foff[n + 1] = int(fh.size());
      cl->loc_off[n + 1] = cl->loc_off[n] + (int64_t(1) << L.k[n]);
      maxk = std::max(maxk, L.k[n]);
    }
    DevBuf<int64_t> d_loff, d_boff;
    DevBuf<int> d_kk, d_eoff, d_ebi, d_ebj, d_foff;
    DevBuf<double> d_eJ, d_fh;
    d_loff.upload(cl->loc_off, s);
    d_kk.upload(kk, s);
    d_eoff.upload(eoff, s);
    d_ebi.upload(ebi.empty() ? std::vector<int>{0} : ebi, s);
    d_ebj.upload(ebj.empty() ? std::vector<int>{0} : ebj, s);
    d_eJ.upload(eJ.empty() ? std::vector<double>{0.0} : eJ, s);
    d_foff.upload(foff, s);
    d_fh.upload(fh, s);
    cl->E_loc.alloc(size_t(cl->loc_off[ncell]));
    cl->w_loc.alloc(size_t(cl->loc_off[ncell]));
    hipLaunchKernelGGL(local_energy_kernel, dim3(unsigned(cdiv(int64_t(1) << maxk, 256)), ncell),
                       dim3(256), 0, s, d_loff.p, d_kk.p, d_eoff.p, d_ebi.p, d_ebj.p, d_eJ.p,
                       d_foff.p, d_fh.p, cl->E_loc.p);
    HIPC(hipGetLastError());
    // bond tables (a2)
    std::vector<int> rows, cols, boff_e(1, 0), pp, pq;
    std::vector<double> bJ;
    std::vector<int64_t> boff(1, 0);
    int64_t maxent = 1;
    for (auto& kv : inter) {
      int m = int(kv.first / ncell), n = int(kv.first % ncell);
      uint32_t bm = cl->B(m, n), bn = cl->B(n, m);
      tnb_clusters::Bond bd{m, n, boff.back(), 1 << popcount32(bm), 1 << popcount32(bn), 0.0};
      if (int64_t(bd.rows) * bd.cols > (int64_t(1) << 26))
        fail(TNB_EUNSUPPORTED, "bond table larger than 2^26 entries");
      cl->bond_of[kv.first] = int(cl->bonds.size());
      cl->bonds.push_back(bd);
      rows.push_back(bd.rows);
      cols.push_back(bd.cols);
      for (int e : kv.second) {
        int i = L.ei[e], j = L.ej[e];
        if (L.cell_of[i] != m) std::swap(i, j);
        pp.push_back(popcount32(bm & ((1u << L.bit[i]) - 1u)));
        pq.push_back(popcount32(bn & ((1u << L.bit[j]) - 1u)));
        bJ.push_back(L.J[e]);
      }
      boff_e.push_back(int(pp.size()));
      boff.push_back(boff.back() + int64_t(bd.rows) * bd.cols);
      maxent = std::max(maxent, int64_t(bd.rows) * bd.cols);
    }
    const int nb = int(cl->bonds.size());
    cl->E_bond.alloc(size_t(std::max<int64_t>(boff.back(), 1)));
    cl->W_bond.alloc(size_t(std::max<int64_t>(boff.back(), 1)));
    DevBuf<int> d_rows, d_cols, d_beoff, d_pp, d_pq;
    DevBuf<double> d_bJ;
    if (nb) {
      d_boff.upload(boff, s);
      d_rows.upload(rows, s);
      d_cols.upload(cols, s);
      d_beoff.upload(boff_e, s);
      d_pp.upload(pp, s);
      d_pq.upload(pq, s);
      d_bJ.upload(bJ, s);
      hipLaunchKernelGGL(bond_energy_kernel, dim3(unsigned(cdiv(maxent, 256)), nb), dim3(256), 0, s,
                         d_boff.p, d_rows.p, d_cols.p, d_beoff.p, d_pp.p, d_pq.p, d_bJ.p,
                         cl->E_bond.p);
      HIPC(hipGetLastError());
    }
    // minima and Boltzmann weights (a3)
    std::vector<int64_t> lens(ncell), blens(nb);
    for (int n = 0; n < ncell; ++n) lens[n] = cl->loc_off[n + 1] - cl->loc_off[n];
    for (int t = 0; t < nb; ++t) blens[t] = boff[t + 1] - boff[t];
    DevBuf<int64_t> d_llen, d_blen;
    DevBuf<double> d_lmin(ncell), d_bmin(std::max(nb, 1));
    d_llen.upload(lens, s);
    hipLaunchKernelGGL(table_min_kernel, dim3(ncell), dim3(256), 0, s, cl->E_loc.p, d_loff.p,
                       d_llen.p, d_lmin.p);
    hipLaunchKernelGGL(boltzmann_kernel, dim3(unsigned(cdiv(int64_t(1) << maxk, 256)), ncell),
                       dim3(256), 0, s, cl->E_loc.p, cl->w_loc.p, d_loff.p, d_llen.p, d_lmin.p,
                       beta);
    if (nb) {
      d_blen.upload(blens, s);
      hipLaunchKernelGGL(table_min_kernel, dim3(nb), dim3(256), 0, s, cl->E_bond.p, d_boff.p,
                         d_blen.p, d_bmin.p);
      hipLaunchKernelGGL(boltzmann_kernel, dim3(unsigned(cdiv(maxent, 256)), nb), dim3(256), 0, s,
                         cl->E_bond.p, cl->W_bond.p, d_boff.p, d_blen.p, d_bmin.p, beta);
    }
    // FP32 copies of every weight table (exp(-beta (E - E_min)) lies in [0, 1])
    {
      const int64_t nl = cl->loc_off[ncell], nbw = int64_t(cl->W_bond.n);
      cl->w_loc32.alloc(size_t(std::max<int64_t>(nl, 1)));
      cl->W_bond32.alloc(size_t(std::max<int64_t>(nbw, 1)));
      if (nl) hipLaunchKernelGGL(to_f32_kernel, dim3(unsigned(cdiv(nl, 256))), dim3(256), 0, s, cl->w_loc.p, nl, cl->w_loc32.p);
      if (nb) hipLaunchKernelGGL(to_f32_kernel, dim3(unsigned(cdiv(nbw, 256))), dim3(256), 0, s, cl->W_bond.p, nbw, cl->W_bond32.p);
    }
    HIPC(hipGetLastError());
    cl->E_min_loc.resize(ncell);
    std::vector<double> bmin(nb);
    HIPC(hipMemcpyAsync(cl->E_min_loc.data(), d_lmin.p, ncell * sizeof(double),
                        hipMemcpyDeviceToHost, s));
    if (nb)
      HIPC(hipMemcpyAsync(bmin.data(), d_bmin.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    double shift = 0.0;
    for (int n = 0; n < ncell; ++n) shift += -beta * cl->E_min_loc[n];
    for (int t = 0; t < nb; ++t) {
      cl->bonds[t].Emin = bmin[t];
      shift += -beta * bmin[t];
    }
    cl->shift = shift;
    cl->d_ei.upload(L.ei, s);
    cl->d_ej.upload(L.ej, s);
    cl->d_J.upload(L.J, s);
    cl->d_h.upload(L.h, s);
    HIPC(hipStreamSynchronize(s));
    *out = cl.release();
  });
}

extern "C" tnb_status tnb_cluster_energies(const tnb_clusters* cl, int32_t cell, double* d_out,
                                           int64_t n_out, tnb_stream stream) {
  return guarded([&] {
    if (!cl || cl->kind != KIND_CLUSTERS) fail(TNB_EINVAL, "not a clusters handle");
    if (cell < 0 || cell >= cl->lat.cells()) fail(TNB_EINVAL, "cell out of range");
    int64_t len = cl->loc_off[cell + 1] - cl->loc_off[cell];
    if (n_out != len || !d_out) fail(TNB_EINVAL, "output length must be 2^k");
    HIPC(hipMemcpyAsync(d_out, cl->E_loc.p + cl->loc_off[cell], len * sizeof(double),
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  });
}

extern "C" tnb_status tnb_bond_energies(const tnb_clusters* cl, int32_t m, int32_t n,
                                        double* d_out, int64_t n_out, int32_t* rows,
                                        int32_t* cols_out, tnb_stream stream) {
  return guarded([&] {
    if (!cl || cl->kind != KIND_CLUSTERS) fail(TNB_EINVAL, "not a clusters handle");
    if (m < 0 || n < 0 || m >= cl->lat.cells() || n >= cl->lat.cells() || m >= n)
      fail(TNB_EINVAL, "need 0 <= m < n < cells");
    auto it = cl->bond_of.find(int64_t(m) * cl->lat.cells() + n);
    if (it == cl->bond_of.end()) fail(TNB_EINVAL, "clusters are not coupled");
    const auto& bd = cl->bonds[it->second];
    if (rows) *rows = bd.rows;
    if (cols_out) *cols_out = bd.cols;
    if (!d_out || n_out < int64_t(bd.rows) * bd.cols) fail(TNB_EINVAL, "output too small");
    HIPC(hipMemcpyAsync(d_out, cl->E_bond.p + bd.off, size_t(bd.rows) * bd.cols * sizeof(double),
                        hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
  });
}

extern "C" tnb_status tnb_profile_enable(int32_t on) {
  return guarded([&] {
    std::lock_guard<std::mutex> lock(tnb::g_prof_mu);
    if (on) {
      // the previous records' events go back to their device's pool, and the
      // current device's pool is topped up to 16384 events before timing
      for (size_t i = 0; i < tnb::g_recs.size(); ++i) {
        auto& pool = tnb::g_pool[tnb::g_rec_dev[i]];
        pool.push_back(tnb::g_recs[i].a);
        pool.push_back(tnb::g_recs[i].b);
      }
      tnb::g_recs.clear();
      tnb::g_rec_dev.clear();
      int dev = 0;
      HIPC(hipGetDevice(&dev));
      if (dev < 0 || dev >= tnb::kPoolDevices) fail(TNB_EDEVICE, "device index out of range");
      auto& pool = tnb::g_pool[dev];
      while (pool.size() < 16384) {
        hipEvent_t e;
        HIPC(hipEventCreate(&e));
        pool.push_back(e);
      }
    }
    tnb::g_prof = on != 0;
  });
}

extern "C" tnb_status tnb_profile_query(const char* name, double* total_ms, int64_t* launches,
                                        double* flops, double* bytes) {
  return guarded([&] {
    if (!name) fail(TNB_EINVAL, "name is NULL");
    std::lock_guard<std::mutex> lock(tnb::g_prof_mu);
    double ms = 0.0, fl = 0.0, by = 0.0;
    int64_t n = 0;
    for (auto& r : tnb::g_recs) {
      if (std::strcmp(r.name, name) != 0) continue;
      HIPC(hipEventSynchronize(r.b));
      float e = 0.f;
      HIPC(hipEventElapsedTime(&e, r.a, r.b));
      ms += e;
      fl += r.flops;
      by += r.bytes;
      ++n;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    if (flops) *flops = fl;
    if (bytes) *bytes = by;
  });
}

extern "C" tnb_status tnb_profile_names(char* buf, int64_t len) {
  return guarded([&] {
    if (!buf || len < 1) fail(TNB_EINVAL, "bad buffer");
    std::lock_guard<std::mutex> lock(tnb::g_prof_mu);
    std::string out;
    std::vector<std::string> seen;
    for (auto& r : tnb::g_recs) {
      bool dup = false;
      for (auto& x : seen) dup = dup || x == r.name;
      if (dup) continue;
      seen.push_back(r.name);
      if (!out.empty()) out += ",";
      out += r.name;
    }
    std::strncpy(buf, out.c_str(), size_t(len - 1));
    buf[len - 1] = '\0';
  });
}

extern "C" tnb_status tnb_set_allocator(const tnb_allocator* a) {
  return guarded([&] {
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    if (!a) {
      g_current = nullptr;
      return;
    }
    if (!a->alloc || !a->release) fail(TNB_EINVAL, "allocator needs both alloc and release");
    auto al = std::make_unique<Allocator>();
    al->alloc = a->alloc;
    al->release = a->release;
    al->user = a->user;
    g_current = al.get();
    g_allocators.push_back(std::move(al));
  });
}
