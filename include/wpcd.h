/*
 * wpcd.h -- C ABI of the MI355X (gfx950) wave-packet continuum discretisation
 * (WPCD) library for two-body partial-wave scattering.
 *
 * For every (potential sample, partial-wave channel) item the library
 *   1. projects the potential onto N_WP momentum wave packets   (wpcd_project),
 *   2. diagonalises H = H0 + V in the free wave-packet basis    (wpcd_eigh),
 *   3. builds the on-shell T-matrix at every bin energy from the eigenpairs and
 *      the energy-averaged scattering-packet resolvent          (wpcd_tmatrix),
 *   4. turns S = 1 - i pi p t into phase shifts, Stapp mixing angles
 *      (wpcd_observables) and total cross sections            (wpcd_sigma_tot).
 * The method is that of Miller, Ekstroem and Forssen, "Wave-packet continuum
 * discretisation for nucleon-nucleon scattering predictions" (arXiv:2106.00454):
 * Sec. 3.1 (wave packets, diagonalisation, scattering-packet bins, coupled
 * channels), Sec. 3.2 (LS equation in the packet basis, energy averaging,
 * potential projection, five-step recipe), App. A (S-matrix, Stapp
 * parametrisation, total cross section) and App. B (resolvent in a packet basis).
 *
 * Units and conventions
 *   momenta k in fm^-1; reduced potential U = m_N V/(hbar c)^2 in fm; energies as
 *   k^2 in fm^-2; states <k'|k> = delta(k'-k)/(k'k), so the LS kernel carries no
 *   2/pi; T_lab in MeV (non-relativistic, equal masses: p = sqrt(m_N T_lab/2)/(hbar c),
 *   m_N = 938.918 MeV, hbar c = 197.327 MeV fm); phase shifts and mixing angles in
 *   degrees, principal values in (-90, 90]; cross sections in mb.
 *   Momentum wave packets (f = 1, N_i = dk_i); on-shell momentum of bin k is its
 *   midpoint kbar_k; H0 diagonal e_k = (k_{k-1}^2 + k_{k-1} k_k + k_k^2)/3.
 *   Coupled channels (n_ch = 2) stack two copies of the free basis channel-major:
 *   basis row r = a*N + i for orbital index a (0: l = J-1, 1: l = J+1) and bin i.
 *
 * Ownership and memory
 *   All array arguments of the compute calls are DEVICE pointers owned by the
 *   caller; the library never frees them.  Host pointers are marked "_host".
 *   The context owns the resident grids (bounds, H0, Gauss nodes) and every batch
 *   owns the device workspace of its eigensolver; both are freed by their destroy
 *   call.  Compute calls are asynchronous on the given HIP stream; results are
 *   valid once that stream has been synchronised.
 *
 * Errors
 *   Every call returns a status: WPCD_OK or a negative WPCD_ERR_*.  Argument
 *   checks happen before any launch and return WPCD_ERR_INVALID with nothing
 *   enqueued.  A failed HIP call returns WPCD_ERR_DEVICE (WPCD_ERR_NOMEM for a
 *   failed allocation).  WPCD_ERR_DEVICE from a compute call (wpcd_project*,
 *   wpcd_eigh*, wpcd_tmatrix, wpcd_observables, wpcd_sigma_tot) is sticky:
 *   every later compute call on the same context returns it too, with the
 *   first failure's message, until wpcd_destroy.  wpcd_last_error() returns a
 *   thread-local message describing the last failure of this thread.
 *   Per-item numerical failures are written to caller-provided int32 status
 *   arrays (one entry per item) instead of failing the whole call; the
 *   outputs of an item that wpcd_tmatrix flags are NaN (T, and from it the
 *   phase shifts, mixing angles and its sample's cross sections).
 *
 * Threading: one context per device; calls on one context must not run
 * concurrently from several host threads.
 *
 * Lifetimes: batches, matrix-inversion solvers, graphs and servers use their
 * context in every call, so the context must outlive those calls; their
 * destroy calls touch only their own resources and may come before or after
 * wpcd_destroy of the context (e.g. in whatever order a garbage collector
 * finalises the handles).
 */
#ifndef WPCD_H
#define WPCD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WPCD_OK = 0,
  WPCD_ERR_INVALID = -1,     /* bad argument, detected before any launch     */
  WPCD_ERR_NOMEM = -2,       /* device allocation failed                     */
  WPCD_ERR_DEVICE = -3,      /* a HIP runtime call failed; sticky for the
                                compute calls of the context (below)        */
  WPCD_ERR_NOCONV = -4,      /* per item: Jacobi sweep cap reached           */
  WPCD_ERR_AGAIN = -5,       /* wpcd_poll: the request is still pending      */
  WPCD_ERR_BUSY = -6,        /* wpcd_submit: the admission queue is full     */
  WPCD_ERR_NUMERIC = -7,     /* per item: NaN/Inf, zero eigenvalue, a
                                scattering family with < 2 members, unsorted
                                or zero-width scattering bins               */
  WPCD_ERR_UNSUPPORTED = -8  /* size or mode the library does not support    */
};

/* Arithmetic of the eigensolver and T contraction.
 * WPCD_MIXED: FP32 one-sided Jacobi (held in LDS for n <= 200, in the batch's
 *             device workspace above), then FP64 refinement of every
 *             eigenpair; FP32 T contraction over an FP64 resolvent table.
 * WPCD_F64:   FP64 one-sided Jacobi in device memory, FP64 T contraction.   */
enum { WPCD_MIXED = 0, WPCD_F64 = 1 };

/* Element type of the fine-mesh potential passed to wpcd_project. */
enum { WPCD_DTYPE_F32 = 0, WPCD_DTYPE_F64 = 1 };

typedef struct wpcd_context* wpcd_ctx;
typedef struct wpcd_batch_s* wpcd_batch;

typedef struct {
  int32_t max_sweeps;    /* Jacobi sweep cap (default 30)                       */
  int32_t refine_steps;  /* FP64 refinement steps in WPCD_MIXED (default 2, 0..4) */
  double jacobi_tol_f32; /* one-sided Jacobi: skip a pair once |w_p.w_q| <=
                            tol*|w_p||w_q|; a sweep whose largest rotated pair
                            was below 8*tol ends the iteration (FP32 path;
                            default 2e-7)                                      */
  double jacobi_tol_f64; /* same for the FP64 path (default 1e-15)              */
  int32_t jacobi_block;  /* variant of the LDS FP32 Jacobi: 0 (default) column
                            blocks of 2 held in registers, two blocks per lane
                            group and 4 rotations per block step, with tracked
                            column norms (one dot product per pair) and scaled
                            rotations (each column carries a scale factor, one
                            FMA per element and column), in a recursive
                            halving ordering in which each lane group keeps
                            one of its blocks in registers for a whole level
                            (one block per step through LDS); 7 the same in
                            the round-robin ordering; 1 one column pair per
                            lane group, three dot products per pair; 2 one pair
                            per group, tracked norms; 3 as 0 with plain
                            rotations; 4 blocks of 4 columns, tracked norms;
                            5 blocks of 4 columns, scaled rotations, one
                            16-lane row per block pair whose four quarters
                            compute the four angles of a stage at once; 6
                            the same with blocks of 2 columns (two halves);
                            7 see above; other values: WPCD_ERR_INVALID      */
  int32_t refine_close_log10; /* closeness constant of the first refinement
                            step, c = 10^k (pairs whose first-order update
                            would exceed 1/c are solved by Rayleigh-Ritz);
                            later steps use 100x more each; 0 = default 3   */
  double jacobi_stop_f32; /* FP32 Jacobi (LDS and device-memory): end the
                            iteration after a sweep whose largest rotated
                            pair had |w_p.w_q|/(|w_p||w_q|) below this; must
                            lie in (0, 1); 0 = default max(2e-4, 8 x
                            jacobi_tol_f32).  The FP64 path always uses
                            8 x jacobi_tol_f64                               */
  int32_t jacobi_start;  /* start of the LDS FP32 Jacobi in wpcd_eigh: 0
                            (default) warm: items of a batch that share grid,
                            channel count, J and basis form a group; the
                            first ones (up to one per compute unit and size
                            class, each group's first among them) start from
                            the columns of B in descending norm order, the
                            others from B Q0 with Q0 the eigenvectors of a
                            cold item of their group: in the LDS-resident
                            sizes the one whose V is nearest to theirs on a
                            strided sample of 1024 entries, in device memory
                            the group's first (fewer sweeps when the
                            potentials are alike); 1 cold: every item starts
                            from B.  Results agree within the refinement's
                            accuracy either way.                             */
  int32_t refine_gemm;   /* dense products of the FP64 refinement: 0
                            (default) whole-item products (one work-group of
                            12 wavefronts per item, persistent over the
                            items) when every item of the batch has 193..208
                            rows, else 64 x 64 tiles; 1 always tiles.  Same
                            results up to rounding order.                    */
  int32_t refine_rr_steps; /* refinement steps, counted from the last, that
                            solve clusters of close eigenvalues by Rayleigh-
                            Ritz; the earlier steps give a close pair the
                            symmetric update R_ij/2 (the cluster's subspace
                            is still corrected, its basis inside the cluster
                            is left to the later Rayleigh-Ritz).  0 (default)
                            = every step; 1..refine_steps                    */
} wpcd_config;

/* Create a context on HIP device `hip_device`; cfg may be NULL for defaults. */
int wpcd_create(wpcd_ctx* out, int hip_device, const wpcd_config* cfg);
void wpcd_destroy(wpcd_ctx ctx);
const char* wpcd_last_error(void);
/* Library version string (static storage). */
const char* wpcd_version(void);

/* ---------------------------------------------------------------- grids ----
 * Register a momentum bin grid (Sec. 3.2, step 1): k_bounds_host[0] = 0 <
 * k_1 < ... < k_N, N = n_wp >= 2, n_gauss in [1, 16] Gauss-Legendre nodes per
 * bin for the projection.  The library computes and keeps resident on the
 * device the bin widths, midpoints, boundary energies, H0 diagonal, nodes and
 * weights.  Returns a grid id >= 0 in *grid_id.                              */
int wpcd_grid_create(wpcd_ctx ctx, const double* k_bounds_host, int n_wp, int n_gauss, int* grid_id);

/* Kind of free wave packet of a grid (Sec. 3.1, definition of the free
 * packets and their normalisation).
 * WPCD_PACKET_MOMENTUM: f(k) = 1, N_i = dk_i; H0 diagonal
 *   (k_{i-1}^2 + k_{i-1} k_i + k_i^2)/3; on-shell momentum the bin midpoint
 *   (what wpcd_grid_create registers).
 * WPCD_PACKET_ENERGY: f(k) = sqrt(k/mu) = sqrt(2k) in these units, N_i =
 *   dE_i = k_i^2 - k_{i-1}^2; H0 diagonal the energy midpoint
 *   (k_{i-1}^2 + k_i^2)/2; on-shell momentum q_i = sqrt of that (Sec. 3.2,
 *   choice of the on-shell point).
 * The projection weights become w k f(k)/sqrt(N_i), the packet T-matrix maps
 * to t(q,q) = f(q)^2 T_ii/(N_i q^2), and wpcd_sigma_tot interpolates between
 * the on-shell momenta q_i; resolvent, scattering-packet bins and T are the
 * same for both kinds.                                                      */
enum { WPCD_PACKET_MOMENTUM = 0, WPCD_PACKET_ENERGY = 1 };
/* wpcd_grid_create with a packet kind (WPCD_ERR_INVALID for other values). */
int wpcd_grid_create_packets(wpcd_ctx ctx, const double* k_bounds_host, int n_wp, int n_gauss, int packet,
                             int* grid_id);
/* Copy the grid's Gauss nodes and weights (N*n_gauss each, bin-major) to host
 * memory, e.g. to evaluate a potential at exactly the nodes the library uses.  */
int wpcd_grid_nodes(wpcd_ctx ctx, int grid_id, double* nodes_host, double* weights_host);

/* ---------------------------------------------------------------- batches --
 * One item = one channel of one potential sample.  n_ch = 1 (uncoupled) or 2
 * (coupled, l = J-1 and J+1); J weights the item by 2J+1 in wpcd_sigma_tot;
 * items with equal sample_id (0 <= sample_id < n_samples) are summed into one
 * cross section.  Items are packed in the order given; per item with
 * N = n_wp of its grid, n = n_ch*N and M = n_ch*N*n_gauss the packed arrays hold
 *   u_fine  : M*M   (row-major, channel-major rows and columns, symmetric)
 *   v64     : n*n   (row-major, symmetric)
 *   eval    : n     (ascending)
 *   evec    : n*n   (row-major: evec[r*n + m] = <x_r|z_m>, eigenvector m is
 *                    column m)
 *   t       : 2*N*n_ch*n_ch doubles (complex interleaved re,im; index
 *                    ((k*n_ch + a)*n_ch + b))
 *   delta   : N*n_ch  (index k*n_ch + a)
 *   mix     : N       (Stapp eps_J for coupled items, 0 for uncoupled)
 *   s_dev   : N*n_ch  (1 - |S_aa|, a diagnostic of non-unitarity)
 * wpcd_batch_create validates the items, uploads their descriptors and
 * allocates the eigensolver workspace of the batch.                          */
typedef struct {
  int32_t grid_id;
  int32_t n_ch;
  int32_t J;
  int32_t sample_id;
  int32_t basis_id; /* -1: V from a fine-mesh potential (wpcd_project);
                       >= 0: V = sum_t c_t B_t from a registered basis
                       (wpcd_project_affine), which must match grid_id and
                       n_ch.  Such items take no space in u_fine and
                       n_terms entries in the packed coefficient array.   */
  int32_t S;        /* total spin 0 or 1, or -1 (not given; only
                       wpcd_saclay needs it)                               */
  int32_t l;        /* orbital momentum of the first channel: l = J for
                       uncoupled items (or 1 for 3P0, J = 0), J - 1 for
                       coupled ones (S = 1); ignored when S = -1          */
} wpcd_item;

typedef struct {
  int64_t u_elems, v_elems, eval_elems, t_doubles, delta_elems, mix_elems, coef_elems;
  int32_t n_items, n_samples, max_n, max_nbins;
} wpcd_batch_layout;

int wpcd_batch_create(wpcd_ctx ctx, const wpcd_item* items_host, int n_items, wpcd_batch* out);
void wpcd_batch_destroy(wpcd_batch b);
int wpcd_batch_layout_get(wpcd_batch b, wpcd_batch_layout* out);
/* Per-item element offsets into the packed arrays (host arrays of n_items;
 * any pointer may be NULL).                                                  */
int wpcd_batch_offsets(wpcd_batch b, int64_t* u_off_host, int64_t* v_off_host, int64_t* eval_off_host,
                       int64_t* t_off_host, int64_t* delta_off_host, int64_t* mix_off_host,
                       int64_t* coef_off_host);

/* ---------------------------------------------------------------- bases ----
 * wpcd_basis_register (Sec. 3.2: the packet potential matrix is linear in U):
 * for potentials of the affine form U = sum_t c_t U_t, projects the n_terms
 * fine-mesh terms U_t once and keeps B_t = proj(U_t) resident in the context
 * (FP64, n_terms*n*n doubles, n = n_ch*N).  u_terms is a DEVICE array of n_terms
 * consecutive M*M matrices (layout of u_fine above, M = n_ch*N*n_gauss) of
 * dtype u_dtype; it is read on `stream`, and the call returns after the
 * projection has finished (it synchronises that stream), so the caller may
 * free u_terms afterwards.  1 <= n_terms <= 16.  Returns a basis id >= 0.     */
int wpcd_basis_register(wpcd_ctx ctx, int grid_id, int n_ch, int n_terms, const void* u_terms, int u_dtype,
                        hipStream_t stream, int* basis_id);

/* ------------------------------------------------------------ compute calls --
 * wpcd_project (Sec. 3.2, the packet potential matrix as a double bin integral):
 *   V_(a,i),(b,j) = (dk_i dk_j)^(-1/2) sum_{alpha in i, beta in j}
 *                   w_alpha k_alpha w_beta k_beta U_(a,alpha),(b,beta)
 * from U at the grid's Gauss nodes, for every item with basis_id = -1.
 * u_dtype selects FP32 (accumulated in FP32) or FP64 (accumulated in FP64)
 * input; V is written as FP64.                                               */
int wpcd_project(wpcd_batch b, const void* u_fine, int u_dtype, double* v64, hipStream_t stream);
/* wpcd_project_affine (Sec. 3.2, projection of an affine potential): for every
 * item with basis_id >= 0, V = sum_t coef[c_off + t] * B_t in FP64 (items with
 * basis_id = -1 are left untouched, as wpcd_project leaves basis items).  coef
 * is a DEVICE array of layout.coef_elems doubles; item i's n_terms values
 * start at its coef offset (wpcd_batch_offsets).                            */
int wpcd_project_affine(wpcd_batch b, const double* coef, double* v64, hipStream_t stream);

/* wpcd_eigh (Sec. 3.1, H = C D C^T; Sec. 3.2, step 2): eigenpairs of
 * H = diag(e, .., e) + V, eigenvalues ascending.  status[i] >= 0 is the number
 * of Jacobi sweeps item i used; WPCD_ERR_NOCONV if the sweep cap was reached
 * (results still written), WPCD_ERR_NUMERIC on NaN/Inf.  In WPCD_MIXED mode the
 * FP32 eigenpairs are refined in FP64 (Newton-type update of all eigenpairs
 * with a Rayleigh-Ritz solve inside clusters of close eigenvalues).  The work
 * is enqueued on `stream`; for items in the device-memory Jacobi (every item
 * in WPCD_F64, those above n = 200 in WPCD_MIXED) the call enqueues the
 * sweeps a few at a time and waits on events until two sweeps after the
 * first one that left them all converged (see wpcd_batch_jacobi_launches),
 * except while the stream is being captured.                                */
int wpcd_eigh(wpcd_batch b, const double* v64, int mode, double* eval, double* evec, int32_t* status,
              hipStream_t stream);

/* wpcd_eigh_noalloc: wpcd_eigh for callers that cannot allocate device
 * memory while they run (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, kernels and results as
 * wpcd_eigh, but the eigensolver work-space (FP32 eigenvectors, the per-item
 * FP64 work-space of 7 n^2 + 40 doubles, cluster lists, Rayleigh quotients,
 * warm-start samples) is taken from a static device array of 128 MiB that the
 * library holds on every device it runs on until the process ends, instead of
 * the batch's own work-space.  The call allocates nothing and creates no
 * stream or event: every launch goes to `stream` (the reference choice and
 * the refinement's second stream of wpcd_eigh run in order on it) and the
 * stage timers do not record it.  A batch whose work-space exceeds 128 MiB
 * (e.g. more than 53 coupled N_WP = 100 items) returns WPCD_ERR_UNSUPPORTED
 * with nothing enqueued; WPCD_ERR_DEVICE if the array's device address is
 * unavailable.  All calls on one device share the array and it keeps the last
 * call's contents (every kernel writes the parts it reads first): calls that
 * may overlap on one device -- on different streams, or from several host
 * threads -- race and must not be issued.                                    */
int wpcd_eigh_noalloc(wpcd_batch b, const double* v64, int mode, double* eval, double* evec, int32_t* status,
                      hipStream_t stream);

/* wpcd_tmatrix (Sec. 3.1, scattering-packet bins; Sec. 3.2, steps 3-5 and the
 * energy average; App. B): for every bin k and channels a, b
 *   T_ab(k) = V_(a,k),(b,k) + sum_m VC_(a,k),m VC_(b,k),m gbar_km,
 *   VC_r,m = (eps_m - e_r) C_r,m   (exact for eigenpairs of H0 + V),
 * gbar_km = resolvent of packet m averaged over the free bin k.  Eigenvalues
 * below 0 (bound) or above k_N^2 (discrete states of the cut-off Hamiltonian)
 * contribute ln((E_k - eps)/(E_{k-1} - eps))/(E_k - E_{k-1}); the others are
 * dealt round-robin into n_ch families, each with bins B_1 = 0,
 * B_j = (eps_{j-1} + eps_j)/2, B_{n+1} = eps_n + (B_n - B_{n-1})/2.
 * status[i] = 0 or WPCD_ERR_NUMERIC.  mode as in wpcd_eigh (contraction
 * precision; the resolvent table is always FP64).                           */
int wpcd_tmatrix(wpcd_batch b, const double* v64, const double* eval, const double* evec, int mode,
                 double* t, int32_t* status, hipStream_t stream);

/* wpcd_observables (App. A, S = 1 - i pi p t, Stapp parametrisation; Sec. 3.1,
 * t(q,q) = T_kk/(dk_k q^2) at q = kbar_k): per item and bin, phase shifts
 * delta_a = arg(S_aa)/2, for coupled items eps_J = asin(Im(S12 exp(-i(d_- + d_+))))/2
 * with S12 = (S_12 + S_21)/2, and s_dev = 1 - |S_aa|.  s_dev may be NULL.   */
int wpcd_observables(wpcd_batch b, const double* t, double* delta_deg, double* mix_deg, double* s_dev,
                     hipStream_t stream);

/* wpcd_sigma_tot (App. A total cross section by the optical theorem in partial
 * waves; Sec. 5.1.1 mid-point linear interpolation):
 *   sigma(p) = 10 * pi/(2 p^2) sum_items (2J+1) sum_a (1 - Re S_aa(p)) [mb]
 * with S rebuilt from (delta, eps) linearly interpolated in q between bin
 * midpoints after unwrapping modulo 180 degrees (end segments extrapolated).
 * tlab_mev: device array of n_tlab energies, each with 0 < p <= k_N of every
 * item's grid (else NaN is written); sigma_mb: device array n_samples*n_tlab,
 * index s*n_tlab + j.                                                       */
int wpcd_sigma_tot(wpcd_batch b, const double* delta_deg, const double* mix_deg, const double* tlab_mev,
                   int n_tlab, double* sigma_mb, hipStream_t stream);

/* wpcd_sigma_band (Sec. 5.1.1, the spread of sigma_tot over the interpolation
 * point of the bins): for every fraction f of `fracs` (DEVICE array of n_frac
 * values in [0, 1], 1 <= n_frac <= 16) the phases of bin i are placed at
 * q_i = k_{i-1} + f (k_i - k_{i-1}) and sigma_tot is evaluated as in
 * wpcd_sigma_tot (unwrapping, linear interpolation in q, Stapp S, optical
 * theorem); sigma_lo_mb / sigma_hi_mb (DEVICE, n_samples*n_tlab each, index
 * s*n_tlab + j) receive the lowest and highest value over the fractions.
 * 1 <= n_tlab <= 256; energies with p outside (0, k_N] give NaN.  The paper's
 * band takes f = n/m with m = 10 and n = 0.1, 1, 2, ..., 9, 9.9.            */
int wpcd_sigma_band(wpcd_batch b, const double* delta_deg, const double* mix_deg, const double* tlab_mev,
                    int n_tlab, const double* fracs, int n_frac, double* sigma_lo_mb, double* sigma_hi_mb,
                    hipStream_t stream);

/* ------------------------------------------------------ matrix inversion ----
 * The paper's comparison method (Sec. 2.1, the wave-matrix form of the
 * discretised LS equation and its K-matrix variant; Sec. 4.1, one LU
 * factorisation per energy), batched over (item, energy) on the same device.
 * For on-shell momentum p, the K-matrix equation with N_Q Gauss-Legendre
 * nodes q_j, weights w_j on [0, L] (L = cutoff) and the pole subtracted,
 *   (1 - U diag(D)) K = U,  D_j = w_j q_j^2/(p^2 - q_j^2)  (j < N_Q),
 *   D_NQ = -p^2 sum_j w_j/(p^2 - q_j^2) + (p/2) ln((L + p)/(L - p)),
 * over the nodes with p appended, is solved by Gaussian elimination with
 * partial pivoting in FP64, one work-group per (item, energy).  The on-shell
 * K_ab(p) gives S = (1 - i pi p K/2)(1 + i pi p K/2)^-1 (unitary), phase
 * shifts and Stapp mixing angles (App. A), and the total cross section at p
 * from the optical theorem in partial waves (no interpolation: every energy is
 * solved exactly).  Energies come as T_lab values (p = sqrt(m_N T_lab/2)/hbar c,
 * 0 < p < cutoff).  Sizes: n_ch (N_Q + 1) unknowns must fit the LDS as an
 * augmented FP64 system: N_Q <= 140 uncoupled, <= 69 when any item is coupled
 * (else WPCD_ERR_UNSUPPORTED).
 * Per item (n_ch = K, P = N_Q + N_E points: the N_Q nodes, then the N_E
 * on-shell momenta, from wpcd_mi_points):
 *   u     : (K P)^2 doubles, U at the point set, row-major, channel-major rows
 *           and columns (row a*P + i), symmetric; DEVICE, caller-owned
 *   kmat  : N_E K^2 doubles, K_ab(p_e) at e*K*K + a*K + b
 *   delta : N_E K phase shifts (deg, index e*K + a), mix: N_E mixing angles
 *           (0 for uncoupled items)
 *   sigma : n_samples x N_E total cross sections in mb (index s*N_E + e)
 * status[i] = 0, or WPCD_ERR_NUMERIC (a zero or non-finite pivot; that item's
 * outputs are NaN).                                                         */
typedef struct wpcd_mi_s* wpcd_mi;
typedef struct {
  int32_t n_ch, J, sample_id, pad;
} wpcd_mi_item;
typedef struct {
  int64_t u_elems, kmat_elems, delta_elems, mix_elems;
  int32_t n_items, n_samples, n_q, n_e;
} wpcd_mi_layout;
int wpcd_mi_create(wpcd_ctx ctx, const wpcd_mi_item* items_host, int n_items, int n_q, double cutoff,
                   const double* tlab_host, int n_e, wpcd_mi* out);
void wpcd_mi_destroy(wpcd_mi m);
/* the N_Q + N_E points (fm^-1) and the N_Q quadrature weights; either may be NULL */
int wpcd_mi_points(wpcd_mi m, double* points_host, double* weights_host);
/* sizes and per-item element offsets (host arrays of n_items; any may be NULL) */
int wpcd_mi_layout_get(wpcd_mi m, wpcd_mi_layout* out, int64_t* u_off_host, int64_t* kmat_off_host,
                       int64_t* delta_off_host, int64_t* mix_off_host);
/* sigma_mb may be NULL (no cross sections) */
int wpcd_mi_solve(wpcd_mi m, const double* u, double* kmat, double* delta_deg, double* mix_deg, double* sigma_mb,
                  int32_t* status, hipStream_t stream);

/* wpcd_saclay (App. A, spin-scattering matrix in partial waves, Saclay
 * amplitudes, differential cross section): for every sample, T_lab energy e
 * and c.m. scattering angle theta_j, the phases of each of the sample's items
 * are interpolated at p as in wpcd_sigma_tot, S is rebuilt in the Stapp form,
 * and the partial-wave sum
 *   M^s_{ms,ms'} = (2 pi/(i p)) sum sqrt((2l+1)/(4 pi)) Y_{l'}^{ms-ms'}(theta, 0)
 *                  <l' ms-ms', s ms'|J ms> <l 0, s ms|J ms> (S_{l'l} - delta_{l'l})
 * (ms incoming, ms' outgoing spin projection; every (S, l, J) counted once,
 * as for neutron-proton scattering) gives the Saclay amplitudes
 *   a = (M11 + M00 - M1,-1)/2, b = (M11 + M^0_00 + M1,-1)/2,
 *   c = (M11 - M^0_00 + M1,-1)/2, d = -(M10 + M01)/(sqrt2 sin theta)
 *   (equivalently (M00 - a)/cos theta), e = i (M01 - M10)/sqrt2,
 * and dsigma/dOmega = (|a|^2 + |b|^2 + |c|^2 + |d|^2 + |e|^2)/2.  Every item
 * needs wpcd_item.S and .l.  tlab_mev (n_tlab) and theta_deg (n_theta) are
 * DEVICE arrays, n_tlab * n_theta <= 1024; dsdo_mb: n_samples*n_tlab*n_theta
 * (index (s*n_tlab + e)*n_theta + j) in mb/sr; amp (may be NULL): 10 doubles
 * per (s, e, j), a..e as (re, im) in fm.  (2 pi/p) Im(a + b) at theta = 0 is
 * the total cross section of wpcd_sigma_tot.                              */
int wpcd_saclay(wpcd_batch b, const double* delta_deg, const double* mix_deg, const double* tlab_mev, int n_tlab,
                const double* theta_deg, int n_theta, double* amp, double* dsdo_mb, hipStream_t stream);

/* ------------------------------------------------------------ whole path --
 * wpcd_run: the whole path of a batch on one stream, in the order of the
 * method (Sec. 3.2, steps 1-5; App. A): wpcd_project for fine-mesh items
 * (u_fine, u_dtype), wpcd_project_affine for basis items (coef), wpcd_eigh,
 * wpcd_tmatrix, wpcd_observables and, when n_tlab > 0, wpcd_sigma_tot.
 * Arguments and errors as for those calls (the first failing call's status
 * is returned; later steps are not enqueued).  u_fine may be NULL for a batch
 * without fine-mesh items, coef for one without basis items, s_dev always. */
typedef struct {
  const void* u_fine;
  int32_t u_dtype;
  int32_t n_tlab;
  const double* coef;
  double* v64;
  double* eval;
  double* evec;
  int32_t* eig_status;
  double* t;
  int32_t* t_status;
  double* delta_deg;
  double* mix_deg;
  double* s_dev;
  const double* tlab_mev;
  double* sigma_mb;
} wpcd_path_args;
int wpcd_run(wpcd_batch b, const wpcd_path_args* a, int mode, hipStream_t stream);

/* Autotuner of the batch path's schedules: runs wpcd_run(b, a, mode) once
 * per candidate schedule as a warm-up, then `reps` times between HIP events
 * on `stream` (after the work already enqueued there; the call waits for the
 * last run), and keeps the fastest in the context's configuration
 * (jacobi_block, refine_gemm; later calls on the context use it).  The
 * candidates (WPCD_MIXED) are the LDS Jacobi with two-column blocks
 * (jacobi_block 0) or four-column blocks and one angle per quarter row (5),
 * each with whole-item or tiled refinement products (refine_gemm 0 / 1);
 * WPCD_F64 has a single schedule.  All candidates give the same results up to
 * rounding order.  cache_path (may be NULL): a text file with one line per
 * tuned batch signature (mode and, per eigensolver size class, item count and
 * largest n); a matching line is applied without timing (from_cache = 1), a
 * new result is appended.  The outputs of `a` hold the last candidate's run.
 * The stage timers must be off.                                             */
typedef struct {
  int32_t jacobi_block, refine_gemm; /* the chosen schedule                    */
  int32_t from_cache, n_cand;        /* taken from the cache; candidates timed */
  double best_ms;                    /* its time per run                       */
  double cand_ms[4];                 /* per candidate: {0,0}, {5,0}, {0,1}, {5,1} */
} wpcd_tune_result;
int wpcd_autotune(wpcd_batch b, const wpcd_path_args* a, int mode, int reps, const char* cache_path,
                  wpcd_tune_result* out, hipStream_t stream);

/* HIP graph of a batch's whole path: wpcd_graph_create captures the launches
 * of wpcd_run(b, a, mode) (including the second stream of wpcd_eigh) into a
 * graph and instantiates it; wpcd_graph_launch replays it on `stream` (the
 * same kernels on the same buffers: change the inputs in place between
 * replays).  Capturing enqueues no work.  The capture holds no memset node
 * and allocates nothing.  The stage timers must be off (WPCD_ERR_INVALID
 * otherwise: they cannot time replays).  The batch and every buffer of `a`
 * must outlive the graph.  wpcd_graph_nodes returns the number of nodes
 * (kernel launches and stream joins) one replay runs.                      */
typedef struct wpcd_graph_s* wpcd_graph;
int wpcd_graph_create(wpcd_batch b, const wpcd_path_args* a, int mode, wpcd_graph* out);
int wpcd_graph_launch(wpcd_graph g, hipStream_t stream);
int wpcd_graph_nodes(wpcd_graph g, int64_t* nodes);
void wpcd_graph_destroy(wpcd_graph g);

/* ---------------------------------------------------------------- serving --
 * A request loop over one context (the paper's posterior-sweep use case, Sec. 1
 * and Sec. 5: many independent parameter-vector solves).  A request is one
 * parameter sample: a set of channels, each an affine potential over a
 * registered basis (wpcd_basis_register) with its own coefficients, and the
 * T_lab values of its total cross section.  Requests are queued by
 * wpcd_submit; a worker thread owned by the server admits queued requests in
 * arrival order while their device footprint fits the free part of a device
 * arena of hbm_budget_bytes and an in-flight slot is free, packs them into
 * one batch, and runs the whole path (affine projection, mixed-precision
 * eigensolver, T, phase shifts, cross sections) on that slot's stream, so
 * batches admitted while others run overlap on the device (continuous
 * batching).  An item's results depend on the other items of its batch only
 * through rounding: the kernels a batch takes follow its size mix (the
 * device-memory Jacobi's block width follows the largest n of its size class,
 * the refinement's product kernels the smallest and largest n of the batch),
 * and batches of the request loop always start cold.  Grids and bases stay
 * resident; register all of them before
 * wpcd_server_create (the server snapshots the context's tables).  The
 * context must not be used for other compute calls while a server runs.
 *
 * Thread safety: wpcd_submit and wpcd_poll may be called from any host
 * threads concurrently.                                                     */
typedef struct wpcd_server_s* wpcd_server;

typedef struct {
  int64_t hbm_budget_bytes; /* device arena for in-flight batches (default 4 GiB) */
  int32_t max_inflight;     /* concurrent batches, one stream each (1..8, default 4) */
  int32_t max_batch_items;  /* items per batch (default 4096)                  */
  int32_t max_queue;        /* queued requests before WPCD_ERR_BUSY (default 65536) */
  int32_t pad;
} wpcd_server_config;

typedef struct {
  int32_t basis_id;        /* registered basis: fixes grid and n_ch           */
  int32_t J;               /* total angular momentum (weight 2J+1 in sigma)   */
  const double* coef_host; /* the basis's n_terms coefficients (copied)       */
} wpcd_req_channel;

typedef struct {
  const wpcd_req_channel* channels_host; /* copied at submit                   */
  int32_t n_channels;                     /* 1..64                              */
  int32_t n_tlab;                         /* 0..1024                            */
  const double* tlab_host;                /* n_tlab T_lab values (copied)       */
  /* outputs, host memory owned by the caller, written by the worker thread
   * and valid once wpcd_poll has returned anything but WPCD_ERR_AGAIN:       */
  double* sigma_host;  /* n_tlab total cross sections (mb), may be NULL if n_tlab = 0 */
  double* delta_host;  /* optional: per channel N*n_ch phase shifts, channels concatenated */
  double* mix_host;    /* optional: per channel N mixing angles (0 if uncoupled), concatenated */
  int32_t* status_host; /* optional: per channel eigensolver status (sweeps or WPCD_ERR_*) */
} wpcd_request;

typedef struct {
  int64_t submitted, completed, batches, items, peak_arena_bytes;
  int32_t queued, inflight;
  int64_t jacobi_launches; /* kernel launches of the device-memory Jacobi (items above n = 200) */
  int64_t jacobi_sweeps;   /* sweeps it enqueued: all max_sweeps of them per launch sequence (the
                              worker does not wait on the device; converged items return at once) */
} wpcd_server_stats;

/* cfg may be NULL for defaults.  Allocates the arena and pinned staging and
 * starts the worker thread.                                                 */
int wpcd_server_create(wpcd_ctx ctx, const wpcd_server_config* cfg, wpcd_server* out);
/* Stops admitting, waits for in-flight batches, joins the worker and frees
 * everything; requests still queued are dropped (their poll would return
 * WPCD_ERR_INVALID afterwards, as the server no longer exists).             */
void wpcd_server_destroy(wpcd_server s);
/* Queues a request; *ticket identifies it for wpcd_poll.  Returns
 * WPCD_ERR_BUSY if max_queue requests are waiting, WPCD_ERR_INVALID for bad
 * arguments (unknown basis, too many channels or energies) and
 * WPCD_ERR_UNSUPPORTED if the request alone exceeds hbm_budget_bytes.       */
int wpcd_submit(wpcd_server s, const wpcd_request* req, uint64_t* ticket);
/* WPCD_ERR_AGAIN while pending; otherwise the request's outputs are written,
 * the ticket is retired and the return value is WPCD_OK, the first failing
 * item's code (WPCD_ERR_NOCONV / WPCD_ERR_NUMERIC), or WPCD_ERR_DEVICE if its
 * batch failed on the device.  Unknown or retired tickets: WPCD_ERR_INVALID. */
int wpcd_poll(wpcd_server s, uint64_t ticket);
int wpcd_server_stats_get(wpcd_server s, wpcd_server_stats* out);

/* ------------------------------------------------------------ stage timers --
 * When enabled, every compute call records a pair of HIP events on its stream
 * around each kernel group it launches (the eigensolver counts as three
 * stages: the Jacobi sweeps (one group per launch of the LDS kernel or per
 * device-memory launch sequence), the preparation of warm starts and the
 * refinement).  wpcd_stage_times waits for the
 * recorded events, adds their elapsed times to per-stage totals and returns
 * the totals in milliseconds and the number of launches per stage (arrays of
 * WPCD_N_STAGES, host memory, either may be NULL).  Enabling (again) resets
 * the totals.  Timing adds two event records per kernel group.              */
enum {
  WPCD_STAGE_PROJECT = 0,
  WPCD_STAGE_JACOBI_F32 = 1,
  WPCD_STAGE_JACOBI_F64 = 2,
  WPCD_STAGE_REFINE = 3,
  WPCD_STAGE_TMATRIX = 4,
  WPCD_STAGE_OBSERVABLES = 5,
  WPCD_STAGE_SIGMA = 6,
  WPCD_STAGE_WARM_PREP = 7,
  WPCD_N_STAGES = 8
};
int wpcd_profile_enable(wpcd_ctx ctx, int on);
int wpcd_stage_times(wpcd_ctx ctx, double* ms_host, int64_t* launches_host);
/* Work done by the LDS FP32 Jacobi (default variant) while the stage timers
 * were on, since they were last enabled: counts_host[0] = rotations applied,
 * [1] = column-pair visits (one dot product each), [2] = column-norm
 * evaluations (sum over items of sweeps * n^2 multiply-adds).  Synchronises
 * the device.  Used to state the kernel's algorithmic FLOP count.          */
int wpcd_jacobi_counts(wpcd_ctx ctx, int64_t* counts_host);
/* Launch counters of the batch's device-memory Jacobi (the FP64 path, and
 * the mixed path's items above n = 200): counts_host[0] = kernel launches,
 * [1] = sweeps enqueued, summed over its launch sequences since the batch
 * was created or the counters were last cleared (clear != 0 clears them after
 * reading).  Outside stream capture the sweeps are enqueued a few at a time
 * and stop two sweeps after the first one that left every item of the
 * sequence converged (the host waits on events for that); a captured
 * sequence enqueues max_sweeps sweeps, converged items returning at once.
 * Host counters: no device synchronisation.                                */
int wpcd_batch_jacobi_launches(wpcd_batch b, int clear, int64_t* counts_host);

#ifdef __cplusplus
}
#endif
#endif /* WPCD_H */
