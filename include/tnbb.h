/*
 * tnbb.h -- C ABI of libtnbb: boundary-MPS conditional marginals and branch
 * and bound for Ising problems clustered into Potts variables on a king's
 * lattice, after "Limitations of tensor-network approaches for optimization
 * and sampling" (Dziubyna, Smierzchalski, Gardas, Rams, Mohseni).
 *
 * Conventions shared by every entry point
 *  - Spins s_i = +-1.  Cluster n = r*cols + c holds the spins with
 *    cell_of[i] == n in ascending index; bit b of the cluster variable x_n is
 *    its b-th spin, bit 1 meaning s = +1.
 *  - Host pointers are read during the call only and copied; device pointers
 *    (prefix d_) must stay valid until the work queued on `stream` has run.
 *  - All work is queued on the caller's HIP stream.  Calls that return values
 *    in host memory synchronise that stream.
 *  - Every call returns a tnb_status; on failure tnb_last_error() returns a
 *    message (thread-local, valid until the next call on the thread).  No C++
 *    exception crosses the ABI.  Handles are owned by the library and freed
 *    with tnb_destroy.
 *  - Every floating-point quantity is FP64.
 */
#ifndef TNBB_H
#define TNBB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TNB_OK = 0,
  TNB_EINVAL = -1,       /* invalid argument (checked before any GPU work)    */
  TNB_ENOMEM = -2,       /* device or host allocation failed                  */
  TNB_ENUMERIC = -3,     /* non-finite value, or every marginal of a parent
                            was non-positive                                  */
  TNB_EDEVICE = -4,      /* HIP runtime error                                  */
  TNB_EUNSUPPORTED = -5  /* size beyond what the library supports           */
} tnb_status;

typedef void* tnb_stream;  /* a hipStream_t; NULL is the null stream */

/* Arithmetic of the environment contractions (the benchmark spec's FP32 option,
 * Sec. VI compares the two).  TNB_F32: the site and mediating diagrams read
 * FP32 copies of their operands and of the Boltzmann weights (each table
 * already shifted by its minimum energy, so every weight lies in [0, 1]) and
 * accumulate in FP32 on the matrix cores; the bond-weight folds, the QR/SVD,
 * the truncation, the log-scales, the beam and every result stay FP64. */
typedef enum { TNB_F64 = 0, TNB_F32 = 1 } tnb_prec;

/* One Ising instance, H(s) = sum_e J_e s_i s_j + sum_i h_i s_i (Eq. 1), all
 * arrays in host memory.  Edges e have 0 <= edge_i[e] < edge_j[e] < n_spins,
 * sorted by (i, j), no duplicates.  Every edge must join clusters that are
 * king's-lattice neighbours (|dr| <= 1 and |dc| <= 1), a cluster holds at
 * most 24 spins (d <= 2^24, Sec. III), and J, h must be finite. */
typedef struct {
  int32_t n_spins;
  int32_t n_edges;
  const int32_t* edge_i;
  const int32_t* edge_j;
  const double* J;
  const double* h;
  int32_t rows;
  int32_t cols;
  const int32_t* cell_of;  /* [n_spins], r*cols + c */
} tnb_instance;

typedef struct tnb_clusters tnb_clusters;
typedef struct tnb_env tnb_env;
typedef struct tnb_beam tnb_beam;

/* Eq. (1) for K states.  d_states: device, int8 [K][n_spins] of +-1;
 * d_E: device, [K].  Couplings are added one after another in edge order,
 * then the fields in spin order, every operation rounded in FP64 (no fused
 * multiply-add), so the result is reproducible bit for bit.
 * Errors: TNB_EINVAL for a malformed instance or K < 0. */
tnb_status tnb_energies(const tnb_instance* inst, const int8_t* d_states, int64_t K,
                        double* d_E, tnb_stream stream);

/* tnb_energies for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same kernel and result, bit for bit, with the instance's couplings, fields
 * and edge lists staged in a static device array of the library (2 MiB per
 * GPU, held until the process ends) instead of allocated buffers.  The
 * instance must fit it: 16 * n_edges + 8 * n_spins <= 2 MiB, else
 * TNB_EUNSUPPORTED before any copy.  Every call on one GPU shares that
 * array, so calls that overlap on a GPU (other threads, other streams) race;
 * the call synchronises `stream` before it returns.  Other errors as
 * tnb_energies. */
tnb_status tnb_energies_noalloc(const tnb_instance* inst, const int8_t* d_states, int64_t K,
                                double* d_E, tnb_stream stream);

/* Clustered Hamiltonian, Eq. (3)-(5), and Boltzmann weights, Eq. (6).
 * Builds, on the device, for every cluster n the local energies
 * E_n[x], x in [0, 2^k_n) (intra-cluster couplings in edge order, then the
 * fields), the projector masks B_mn (spins of m coupled to neighbour n), the
 * compressed bond energies Ebar^{mn}[P^{mn} x_m, P^{nm} x_n] (Eq. 4-5), and
 * weights exp(-beta (E - min E)) for every table; the minima enter a total
 * log-scale.  beta >= 0.  *out receives a handle owned by the caller.
 * Errors: TNB_EINVAL (instance, beta), TNB_EUNSUPPORTED (a cluster with more
 * than 24 spins or a bond table with more than 2^26 entries), TNB_ENOMEM. */
tnb_status tnb_build_clusters(const tnb_instance* inst, double beta, tnb_stream stream,
                              tnb_clusters** out);

/* Copy the local-energy table E_n[x] of cluster `cell` (2^k entries) to
 * d_out (device, n_out doubles).  TNB_EINVAL if n_out != 2^k. */
tnb_status tnb_cluster_energies(const tnb_clusters* cl, int32_t cell, double* d_out,
                                int64_t n_out, tnb_stream stream);

/* Copy the bond-energy table Ebar^{mn} (row: P^{mn} x_m, column: P^{nm} x_n)
 * to d_out; *rows and *cols_out receive its shape.  TNB_EINVAL if m and n are
 * not coupled neighbours or n_out is too small. */
tnb_status tnb_bond_energies(const tnb_clusters* cl, int32_t m, int32_t n, double* d_out,
                             int64_t n_out, int32_t* rows, int32_t* cols_out,
                             tnb_stream stream);

/* Options of the boundary-MPS compression (Sec. III.B, "Variational zipper
 * algorithm for boundary MPS", Fig. 8). */
typedef struct {
  int32_t chi;           /* bond dimension of the boundary MPSs, >= 1        */
  int32_t sketch_extra;  /* oversampling: sketch width is 2*chi + extra      */
  int32_t power_iters;   /* subspace iterations of the randomized SVD        */
  double cut;            /* singular values below cut*sigma_max are dropped;
                            1e-7 <= cut < 1                                  */
  uint64_t seed;         /* Rademacher sketch seed (SplitMix64, counter-based)*/
  int32_t var_window;    /* 2: after each zipper step, one-site variational
                            updates of the new site and its right neighbour
                            (Fig. 8d); 0: none                               */
  int32_t var_sweeps;    /* full one-site variational sweeps of the 2*chi MPS
                            before the chi truncation, 0 .. 8                */
  int32_t prec;          /* tnb_prec of the diagram contractions             */
} tnb_env_opts;

/* Boundary MPSs Psi_R .. Psi_1 of the lower half-lattice (Fig. 6, 8) and
 * log Z (Eq. 10).  Psi_r (2*cols-1 sites: a vertical and a two-diagonal
 * site per column pair) is compress_chi(T_r Psi_{r+1}), the variational
 * zipper of Sec. III.B: a right-to-left zipper attaching one site or
 * mediating tensor at a time, each dashed box truncated to 2*chi by a
 * matrix-free randomized SVD and followed by a one-site variational update
 * of the two sites next to the zipper centre (var_window); then var_sweeps
 * full one-site variational sweeps at 2*chi that maximise the overlap with
 * T_r Psi_{r+1}; then a left-to-right SVD sweep to chi.  log_z (host, may
 * be NULL) receives log |Z|: a truncated environment need not stay positive,
 * and the sign of the approximate Z is reported by tnb_env_logz (the
 * conditional marginals, a ratio of two contractions of the same network,
 * take the sign of their sum and are unaffected).  The returned handle
 * keeps a reference to `cl`, which must outlive it.
 * Errors: TNB_EINVAL (options), TNB_ENUMERIC (zero or non-finite
 * contraction), TNB_ENOMEM. */
tnb_status tnb_contract_env(tnb_clusters* cl, const tnb_env_opts* opts, tnb_stream stream,
                            tnb_env** out, double* log_z);

/* Test and measurement entry points for one dashed box of the zipper
 * (Fig. 7 and Fig. 8c): the row-r MPO tensor at site k of Psi_r (k even:
 * the site tensor of column k/2, Fig. 7a-b; k odd: the mediating tensor
 * between columns (k-1)/2 and (k+1)/2, Fig. 7c-d) between site k of
 * Psi_{r+1} below and a connector on its right.  0 <= r < rows.
 * tnb_diagram_dims: *dm_in is the MPO bond on the box's left (its matrix has
 * rows [m][a], m < dm_in, a < Da), *dm_out the MPO bond on its right (the
 * connector's first index), *ds the physical dimension of Psi_r at k and
 * *ds_below that of Psi_{r+1} at k; any pointer may be NULL. */
tnb_status tnb_diagram_dims(const tnb_clusters* cl, int32_t r, int32_t k, int32_t* dm_in,
                            int32_t* dm_out, int32_t* ds, int32_t* ds_below);

/* Apply the box to caller tensors (device, FP64, row-major), queued on
 * `stream` and synchronised before return.  d_A: site k of Psi_{r+1},
 * [ds_below][Da][Db].
 *  mode 0, D X:  d_K connector [dm_out][Db][Dg]; d_X [ds][Dg][s] (rows
 *                (sigma, g)); d_out [dm_in][Da][s].
 *  mode 1, D^T Y: d_K as in mode 0; d_X [dm_in][Da][s]; d_out [ds][Dg][s].
 *  mode 2, left transfer (the environment of the overlap one site further
 *                right, Fig. 8d): d_K the left environment [dm_in][Da][Dg];
 *                d_X the new site [ds][Dg][s]; d_out [dm_out][Db][s].
 * 1 <= Da, Db, Dg <= 128, 1 <= s <= 256; out_len is d_out's capacity in
 * doubles.  prec (tnb_prec) selects the arithmetic of the diagram kernels;
 * the tensors are FP64 either way.  The product path of tnb_contract_env
 * runs the same kernels.
 * Errors: TNB_EINVAL (handle, indices, sizes, NULL tensors),
 * TNB_EUNSUPPORTED (tiles beyond the LDS), TNB_ENOMEM. */
tnb_status tnb_diagram_apply(const tnb_clusters* cl, int32_t r, int32_t k, int32_t mode, int32_t prec,
                             const double* d_A, int32_t Da, int32_t Db, const double* d_K,
                             int32_t Dg, const double* d_X, int32_t s, double* d_out,
                             int64_t out_len, tnb_stream stream);

/* log |Z| of an environment and the sign (+1 or -1) of the approximate Z
 * (the top-row contraction); either pointer may be NULL.
 * Errors: TNB_EINVAL (handle). */
tnb_status tnb_env_logz(const tnb_env* env, double* log_z, int32_t* sign);

/* Norm-free diagnostic: number of sites of Psi_r and the shape of site k. */
tnb_status tnb_env_site_shape(const tnb_env* env, int32_t r, int32_t k, int32_t* dl,
                              int32_t* d, int32_t* dr);

/* Beam of at most M partial configurations (Sec. III.A), starting with the
 * single empty configuration at step 0.  The handle references `env`. */
tnb_status tnb_beam_create(tnb_env* env, int32_t M, tnb_beam** out);

/* Current step n (cluster r*cols + c about to be fixed), number of parents
 * and the size d of the next cluster; any pointer may be NULL. */
tnb_status tnb_beam_info(const tnb_beam* beam, int32_t* step, int32_t* n_parents, int32_t* d);

/* Marginals of every parent b of the current step, in one of three forms:
 *  TNB_MARG_VECTOR: the conditional distribution p(x_{n+1} | boundary of b)
 *    of the next cluster (Eq. 7, 9; Fig. 6b), [n_parents][d], normalised per
 *    parent.  The marginal is a ratio of contractions of one network, so a
 *    common sign of the approximate environment cancels: entries are taken
 *    with the sign of their sum, and those left non-positive are clipped to 0.
 *  TNB_MARG_SPIN: <s_i>_b = sum_x p(x | b) s_i(x) for the k spins of the next
 *    cluster (bit order), [n_parents][k].
 *  TNB_MARG_ADJOINT: <s_i>_b of every spin of the unfixed clusters of the
 *    current row by the adjoint sweep, [n_parents][n_spins of tnb_row_layout]
 *    (the d_m1 output of tnb_row_moments).
 * out_len is d_out's capacity in doubles.  Synchronises `stream`.
 * Errors: TNB_EINVAL (mode, size), TNB_ENUMERIC (a parent with no positive
 * marginal, or a zero row contraction; reported, not dropped). */
typedef enum { TNB_MARG_VECTOR = 0, TNB_MARG_SPIN = 1, TNB_MARG_ADJOINT = 2 } tnb_marg_mode;
tnb_status tnb_marginals(tnb_beam* beam, int32_t mode, double* d_out, int64_t out_len, tnb_stream stream);

/* One branch-and-bound step (Fig. 3): branch every parent over all d values
 * of the next cluster, score with the chain rule (Eq. 7) in log space, keep
 * the most probable candidate of every boundary configuration (Eq. 8; ties
 * go to the smaller (parent, x)), then the M most probable.  When no fixed
 * cluster couples to an unfixed one (at the last cluster, or when only
 * uncoupled clusters remain) no merge is done.  p_disc_log (host, may be
 * NULL) receives the log
 * of the largest probability discarded so far (-inf if none).
 * TNB_EINVAL when every cluster is already fixed. */
tnb_status tnb_branch_step(tnb_beam* beam, double* p_disc_log, tnb_stream stream);

/* Export the current partial configurations, best first: d_states (device,
 * int8 [K][n_spins], unfixed spins 0), d_logp (device, [K], may be NULL);
 * *count (host) receives min(K, n_parents). */
tnb_status tnb_beam_export(const tnb_beam* beam, int32_t K, int8_t* d_states, double* d_logp,
                           int32_t* count, tnb_stream stream);

/* Final selection of a finished beam (every cluster fixed): the energies
 * of all candidates by Eq. (1) (as tnb_energies, bit for bit), and the K
 * lowest distinct configurations, ordered by energy and then by their spin
 * vectors lexicographically (spin 0 first, -1 < +1).  d_states (device,
 * int8 [K][n_spins] of +-1) and d_E (device, [K]) receive them; *count
 * (host, may be NULL) the number written, min(K, distinct candidates).
 * The last branching step does not merge, so the candidates are the M
 * most probable completions (Sec. III.A).  Synchronises `stream`.
 * Errors: TNB_EINVAL (handle, K < 0, NULL outputs, unfinished beam). */
tnb_status tnb_beam_lowest(tnb_beam* beam, int32_t K, int8_t* d_states, double* d_E, int32_t* count,
                           tnb_stream stream);

/* The same selection over caller arrays: the K lowest distinct of n
 * configurations d_states (device, int8 [n][n_spins] of +-1) with energies
 * d_E (device, [n]), ordered as in tnb_beam_lowest, into d_out ([K][n_spins])
 * and d_E_out ([K]); *count (host, may be NULL) = min(K, distinct).  Used to
 * pool the results of several runs, e.g. the eight lattice transformations
 * of Sec. V.A.  Synchronises `stream`.  Errors: TNB_EINVAL (sizes, NULL
 * pointers). */
tnb_status tnb_select_lowest(const int8_t* d_states, const double* d_E, int64_t n, int32_t n_spins,
                             int32_t K, int8_t* d_out, double* d_E_out, int32_t* count, tnb_stream stream);

/* Layout of the row moments at the current step n = (r, c): the spins of
 * the unfixed clusters (r, c) .. (r, cols-1), cluster by cluster in
 * ascending spin index, and the couplings with both ends in one of those
 * clusters, in edge order.  *n_spins and *n_edges (host, may be NULL)
 * receive the counts; spins and edges (host, may be NULL) receive up to cap
 * ids each (spin indices, edge indices into the instance).
 * TNB_EINVAL when every cluster is already fixed. */
tnb_status tnb_row_layout(const tnb_beam* beam, int32_t* n_spins, int32_t* n_edges, int32_t* spins,
                          int32_t* edges, int32_t cap);

/* Row moments by the adjoint of the row contraction (Eq. 9-10, Fig. 6b):
 * for every parent b of the current step, <s_i>_b = -1/beta dlogZ_b/dh_i for
 * every spin of tnb_row_layout and <s_i s_j>_b = -1/beta dlogZ_b/dJ_ij for
 * every listed coupling, where Z_b is the network of Fig. 6(b) conditioned
 * on b with the boundary MPS below row r held fixed.  One backward sweep
 * over the row, left to right, reusing the right environments of the
 * forward pass as checkpoints.  The values are signed ratios of the
 * approximate contraction (no clipping), so they are exact derivatives of
 * log|Z_b| and may leave [-1, 1] where the approximate environment has
 * negative terms.  d_m1 (device) receives [n_parents][n_spins], d_m2
 * (device, may be NULL) [n_parents][n_edges]; m1_len and m2_len are their
 * capacities in doubles.
 * Errors: TNB_EINVAL (sizes, finished beam), TNB_ENUMERIC (a zero or
 * non-finite Z_b). */
tnb_status tnb_row_moments(tnb_beam* beam, double* d_m1, int64_t m1_len, double* d_m2, int64_t m2_len,
                           tnb_stream stream);

/* The same <s_i>_b by the plain method, one contraction per branch: for
 * every listed spin, Z_b(s_i = +1) and Z_b(s_i = -1) from two clamped
 * contractions, each starting from the stored right environment of the
 * spin's column; <s_i>_b = (Z+ - Z-) / (Z+ + Z-).  Same layout, errors and
 * capacity rule as tnb_row_moments (no couplings). */
tnb_status tnb_row_moments_per_branch(tnb_beam* beam, double* d_m1, int64_t m1_len, tnb_stream stream);

/* Autotuner of kernel launch variants.  Some diagram stages have several
 * launch variants that compute the same sums and differ in how the work is
 * tiled over workgroups (sketch columns per workgroup of the binned mediating
 * kernel: bit-identical results), GEMM tile shapes (bit-identical) or in the
 * order of their additions (the
 * grouped mediating kernel, which sums the items of one weight group before
 * weighting them: equal up to rounding).  mode 1: the first launch of every
 * new shape times each candidate once with HIP events on the launch stream,
 * keeps the fastest and leaves its result; mode 0: use the stored choices and
 * the default variant for unseen shapes.  path (may be NULL: in memory only) names a JSON file of
 * {"shape": variant} that is read now and rewritten after every new choice.
 * Process-wide; calls that tune concurrently are serialised.
 * Errors: TNB_EINVAL (mode). */
tnb_status tnb_autotune(int32_t mode, const char* path);

/* Measurement support.  tnb_profile_enable(1) clears and starts recording a
 * pair of HIP events around every launch of the instrumented kernels, on the
 * stream the kernel runs on, together with its algorithmic flop and byte
 * counts; tnb_profile_enable(0) stops recording.  tnb_profile_query
 * synchronises the recorded events and returns, for the kernel `name`
 * (e.g. "site_apply", "medf_Y2", "renv_V", "beam_q"), the summed duration in
 * milliseconds, the number of launches and the summed algorithmic flops and
 * bytes; unknown names give zeros.  tnb_profile_names writes a
 * comma-separated list of recorded names into buf (NUL-terminated,
 * truncated to len). */
tnb_status tnb_profile_enable(int32_t on);
tnb_status tnb_profile_query(const char* name, double* total_ms, int64_t* launches, double* flops,
                             double* bytes);
tnb_status tnb_profile_names(char* buf, int64_t len);

/* Device memory of the library.  By default hipMalloc/hipFree; with an
 * allocator installed, every later allocation of a handle or of a call's
 * scratch goes through alloc(bytes, user) (which returns NULL on failure:
 * TNB_ENOMEM) and is returned through release(ptr, user) by the allocator
 * that gave it, even after another one is installed.  The allocator must
 * order the reuse of a released block after the work already queued on the
 * stream of the call that released it (a stream-ordered caching allocator
 * such as PyTorch's, used on the same stream, does).  NULL restores
 * hipMalloc/hipFree.  Process-wide; installed allocators stay registered
 * until the process ends.  Errors: TNB_EINVAL (a missing function). */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*release)(void* ptr, void* user);
  void* user;
} tnb_allocator;
tnb_status tnb_set_allocator(const tnb_allocator* a);

/* Loopy belief propagation over the cluster graph (Sec. IV, Fig. 9), with
 * messages on projected cluster states (Eq. 4): every directed bond m -> n
 * carries nu[m->n](P^{nm} x_n), uniform at the start; one iteration forms
 * mu[m->n](xbar_m) = sum over x_m with P^{mn} x_m = xbar_m of the local weight
 * times the messages into m from its other neighbours, then
 * nu[m->n](xbar_n) = sum_xbar_m W_mn(xbar_m, xbar_n) mu[m->n](xbar_m),
 * normalised to sum 1, for every bond at once.  After `iters` iterations the
 * beliefs p_n(x) ~ w_n(x) prod_m nu[m->n](P^{nm} x), normalised per cluster,
 * are written to d_p (device, FP64): cluster n's 2^{k_n} values at offset
 * sum_{n' < n} 2^{k_n'}; p_len is d_p's capacity.  *max_change (may be NULL)
 * receives the largest change of a message in the last iteration.
 * Errors: TNB_EINVAL (handle, iters outside [0, 100000], d_p too short). */
tnb_status tnb_lbp_marginals(const tnb_clusters* cl, int32_t iters, double* d_p, int64_t p_len,
                             double* max_change, tnb_stream stream);

/* Local dimensional reduction (Sec. IV): keep the `keep` states of largest
 * belief (after `iters` iterations; ties: the smaller x) in every cluster and
 * give the others weight 0, so that every later tnb_contract_env and search
 * on this handle works on the reduced state space.  Call before building
 * environments.  Errors: TNB_EINVAL (handle, keep < 1, iters). */
tnb_status tnb_reduce_clusters(tnb_clusters* cl, int32_t keep, int32_t iters, tnb_stream stream);

/* Excitations above each branch from the boundary merge (Sec. III.A, Fig. 4).
 * When tnb_branch_step groups candidates by their boundary, the group's most
 * probable member is kept and every other member differs from it only away
 * from the boundary: that difference (a flip set over clusters, with its
 * energy dE = E(branch with the set flipped) - E(branch) of Eq. 1) is an
 * excitation of the kept branch, which also takes over the other members'
 * excitations (composed with the difference; energies add exactly).
 * Kept per branch: among its own excitations and those from the first
 * max_losers members (by score, then parent, then cluster value), the ones
 * with at most max_cells flipped clusters, dE <= max_dE and (connected_only)
 * flipped clusters connected through couplings, visited by increasing dE
 * (ties: the flip set as a sequence of (cluster, mask) pairs) and accepted
 * while at Hamming distance >= min_hamming from every accepted one, at most
 * max_droplets.  Limits: max_droplets <= 16, max_losers <= 8, max_cells <= 64,
 * min_hamming >= 1. */
typedef struct {
  int32_t max_droplets;    /* 0 switches the bookkeeping off */
  int32_t max_losers;
  int32_t min_hamming;
  int32_t max_cells;
  double max_dE;
  int32_t connected_only;
} tnb_droplet_opts;

/* Switch the bookkeeping on (or off with NULL or max_droplets = 0) for a beam
 * that has taken no step yet.  Errors: TNB_EINVAL (handle, limits, steps
 * already taken), TNB_ENOMEM. */
tnb_status tnb_beam_droplets_enable(tnb_beam* beam, const tnb_droplet_opts* opts);

/* The excitations of branch i of the current beam (0 <= i < npar, the order
 * of tnb_beam_export): up to max_count states d_states [max_count][n_spins]
 * (int8 +-1, 0 for spins of unfixed clusters; the branch's state with the
 * flip set applied) and their dE (d_dE, FP64), by increasing dE; *count
 * receives the number written.  Queued on `stream` and synchronised.
 * Errors: TNB_EINVAL (handle, bookkeeping off, i, outputs). */
tnb_status tnb_beam_droplets(const tnb_beam* beam, int32_t i, int32_t max_count, int8_t* d_states,
                             double* d_dE, int32_t* count, tnb_stream stream);

/* Free a handle from tnb_build_clusters, tnb_contract_env or tnb_beam_create
 * (free dependants before what they reference).  NULL is ignored. */
void tnb_destroy(void* handle);

/* Message of the last failure on this thread ("" if none). */
const char* tnb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TNBB_H */
