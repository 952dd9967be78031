/*
 * tt.h -- C ABI of the MI355X adjoint-state traveltime library (libtt.so).
 *
 * Per-source hot path of adjoint-state traveltime tomography (Chen, Nagaso, Xu
 * & Tong, "TomoATT", arXiv 2412.00031): fast-sweeping solves of the factored
 * anisotropic Eikonal equation (Sec. 2.1 step 1, Eq. (4); Sec. 3.1), solves of
 * the discrete adjoint-state equation (Sec. 2.1 step 2, Eq. (5)), and the
 * sensitivity kernels summed over sources (Eqs. (6)-(9)).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer to caller-owned, contiguous
 *     memory; the library never frees or retains it.  Fields are FP64,
 *     shape [n0][n1][n2] with axis 2 fastest (N = n0*n1*n2 values).  Batched
 *     fields are [nsrc][N].
 *   - Axes: coord = 0 Cartesian (z depth, y, x; km), coord = 1 spherical
 *     (r km ascending with the first index, latitude rad, longitude rad).
 *     Node (i,j,k) sits at o + (i,j,k) * h.  Every n_a >= 4 and <= 8192, and
 *     n0 * (n1 + n2 - 1) * n1p < 2^31 with n1p = n1 + 7 rounded up to a
 *     multiple of 8 (the solver's per-node records use 32-bit indices).
 *   - Positions (sources, receivers) are [count][3] in the same axis units.
 *   - stream is a hipStream_t (NULL = default stream).  Every call enqueues
 *     its work on it and returns without waiting, and can be captured into a
 *     hipGraph (stream capture) -- except tt_forward / tt_adjoint with
 *     TT_FLAG_POLL or TT_FLAG_TIME_SWEEPS, which wait for completion.  Calls
 *     allocate no device memory.  tt_forward / tt_adjoint with more than one
 *     source group fork helper streams off `stream` and join them back with
 *     events; the first such call of a host thread creates those streams and
 *     events, so make it before capturing (or use groups = 1).
 *   - Workspace: ws/ws_bytes is caller-owned device memory of at least
 *     tt_workspace_size(...) bytes for the same arguments; its contents on
 *     entry do not matter and are scratch on exit.  Calls that overlap in
 *     time must not share a workspace.
 *   - Empty batches: a count of 0 (sources, receivers, events) is valid, and
 *     the pointers of arrays that then hold no element may be NULL.  The
 *     call returns TT_OK after writing what its outputs define for no input:
 *     chi = 0 in tt_misfit, zeros (or an unchanged sum with accumulate) in
 *     tt_kernel, zeros in tt_reloc_kernel without fields, nothing
 *     elsewhere.  tt_workspace_size refuses nsrc = 0 (it returns 0); such
 *     calls need no workspace.
 *   - Receivers and sources are expected inside the grid; positions outside
 *     are clamped to the nearest cell on the device (the host cannot read
 *     device data without a synchronisation).
 *   - Return value: TT_OK, TT_EINVAL (bad arguments, checked on the host before
 *     anything is enqueued: NULL pointers, sizes, n_a < 4, h <= 0, tol <= 0,
 *     kappa <= 0, max_iter < 1, too small a workspace), TT_EHIP (a HIP runtime
 *     error).  tt_last_error() describes the last failure of the calling
 *     thread.  Conditions that only the device can see (a source that does not
 *     converge within max_iter) are reported per source in status[].
 */
#ifndef TT_H
#define TT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_OK 0
#define TT_EINVAL (-1)
#define TT_EHIP (-2)
/* Not a return value: the per-source condition "max_iter reached without
 * convergence", reported in status[] as -iterations (a captured or
 * asynchronous call cannot return device facts). */
#define TT_ENOCONV (-3)

typedef struct tt_grid {
    int32_t n[3];   /* nodes per axis, each >= 4 */
    int32_t coord;  /* 0 Cartesian, 1 spherical */
    double o[3];    /* coordinate of node 0 per axis */
    double h[3];    /* spacing per axis, > 0 */
} tt_grid;

typedef struct tt_opts {
    double tol;        /* stop at the first iteration whose convergence measure is < tol */
    int32_t max_iter;  /* >= 1 */
    double kappa;      /* Lax-Friedrichs viscosity factor, >= max sqrt(1 + 2|xi|) */
    int32_t tile_k;    /* k-extent of one sweep tile, 1..62; 0 = library default
                          (tt_default_tile_k) */
    int32_t flags;     /* bit 0 (TT_FLAG_TIME_SWEEPS): time the sweep kernels with a HIP
                          event pair around the tile-plane launches of every
                          directional sweep on the call's stream (tt_sweep_timing) */
    double* eps_hist;  /* optional device buffer [nsrc][max_iter] that receives the
                          convergence measure of every iteration of every source
                          (entries past a source's last iteration are left as
                          they were), or NULL */
    int32_t groups;    /* the sources are split into this many contiguous groups,
                          each iterated on its own stream so that the groups'
                          tile-plane launches run concurrently (fewer idle units
                          at the narrow ends of every sweep and in the
                          convergence tail); 0 = automatic (nsrc / 32, at most
                          4); 1 when TT_FLAG_TIME_SWEEPS is set.  Results do not
                          depend on it. */
    const int32_t* budgets;  /* optional HOST array [nsrc] of per-source iteration
                          budgets, each in [1, max_iter] (e.g. the previous
                          solve's counts plus a margin), or NULL: every source
                          has max_iter.  An asynchronous solve gives each source
                          group the largest budget of its sources, so a group of
                          fast sources stops enqueuing early; a host-polled one
                          stops a group at that budget too.  A source converges
                          or reports -iterations as usual; results do not depend
                          on the budgets otherwise.  Read during the call only. */
} tt_opts;

#define TT_MAX_GROUPS 8

#define TT_FLAG_TIME_SWEEPS 1
/* bit 1: capture iterations (every sweep, boundary and convergence launch)
 * as a hipGraph once per call and replay it: one iteration per replay when
 * polling, four when asynchronous.  Ignored when TT_FLAG_TIME_SWEEPS is set
 * (per-launch events are recorded eagerly) and while the caller's stream is
 * itself being captured (the launches then become nodes of the caller's
 * graph). */
#define TT_FLAG_GRAPH 2
/* bit 2 (tt_adjoint only): solve the continuous adjoint equation (5) by upwind
 * finite volumes instead of the exact transpose of the discrete forward
 * system.  Each node owns its trapezoidal control volume; the flux P w,
 * w = -M grad T, leaves through six faces at the mean of the two nodal normal
 * velocities and carries the upwind node's P; P = 0 on the fixed cell and
 * outside the grid; the receivers inject sum_m R_m (trilinear weights).  The
 * same 8 directional Gauss-Seidel sweeps update the interior, each followed by
 * one Jacobi pass over the boundary nodes.  lam is returned as P s V (V the
 * trapezoidal node volume), the estimate of d chi / d s that Eqs. (6) and (9)
 * give, so tt_kernel and tt_kernel_density apply unchanged.  It agrees with
 * the exact discrete gradient to first order in the grid spacing. */
#define TT_FLAG_CONTINUOUS_ADJOINT 4
/* bit 3 (tt_forward, tt_adjoint): host-polled iterations.  Without it a solve
 * is asynchronous: exactly max_iter iterations are enqueued (max_iter is the
 * iteration budget), a source that converges is marked inactive on the device
 * and its workgroups exit at once in every later launch, and status[] is
 * written on the device (read it after synchronising).  With it the host
 * reads the count of active sources after each iteration (one iteration
 * behind, so the device never idles on the poll), stops enqueuing as soon as
 * every source has converged, and returns after completion.  Results are
 * bit-identical either way. */
#define TT_FLAG_POLL 8
/* bit 4 (tt_adjoint; also pass it to tt_workspace_size): keep one copy of the
 * adjoint's per-node coefficient records, in node order (48 bytes per node
 * and source), instead of four row-coalesced copies laid out so that every
 * sweep direction reads whole cache lines (4 x 48 bytes x n0 (n1 + n2 - 1)
 * n1p per source, about 9x the compact size at 101^3).  For batches whose
 * workspace would not fit otherwise; the sweeps are slower (about 30 % at
 * 101^3 x 128 sources).  Results are bit-identical. */
#define TT_FLAG_COMPACT_ADJOINT 16
/* bit 5 (tt_adjoint only): lam holds the initial field of the iteration on
 * entry (every source's [N] block; nodes of the fixed cell are reset to 0)
 * instead of lambda = 0, e.g. the previous inversion step's lambda of the same
 * sources.  The solve converges to the same tolerance as from 0; the start
 * changes the iteration count and the result only within that tolerance. */
#define TT_FLAG_ADJOINT_INIT 32

/* Bytes of device workspace needed by tt_forward (which = 0), tt_adjoint
 * (which = 1), tt_sample (which = 2) or tt_kernel (which = 3) for this grid,
 * source count and options (tile_k matters; opts may be NULL for defaults).
 * Returns 0 for invalid arguments. */
size_t tt_workspace_size(const tt_grid* grid, int32_t nsrc, const tt_opts* opts, int32_t which);

/* Source constants s0, xi0, eta0 of the factorisation T = T0 * tau: the model
 * interpolated trilinearly at each source (factor of Sec. 3.1).
 * src_par out: [nsrc][3].  Sources must lie inside the grid (device-side
 * clamping to the domain; the host cannot check device positions). */
int tt_source_params(const tt_grid* grid, const double* s, const double* xi, const double* eta,
                     int32_t nsrc, const double* src_pos, double* src_par, void* stream);

/* Forward solve of Eq. (4) for nsrc sources (Sec. 2.1 step 1, Sec. 3.1):
 * factored first-order Lax-Friedrichs fast sweeping, 8 directions per
 * iteration, each directional sweep parallel over 3-D tiles on tile
 * hyperplanes, every sweep followed by a boundary extrapolation pass.
 *   s, xi, eta [N]      model (slowness s/km, azimuthal anisotropy xi, eta)
 *   src_pos [nsrc][3]   source positions; src_par [nsrc][3] = s0, xi0, eta0
 *   tau_init [nsrc][N]  initial tau (warm start) or NULL for tau = 1
 *   tau [nsrc][N]       out: tau, with traveltime T = T0 * tau
 *   status [nsrc]       out (device): iterations done if converged;
 *                       -iterations if max_iter was reached without
 *                       convergence (the TT_ENOCONV condition: outputs are
 *                       still written)
 * tau may alias tau_init.  Asynchronous on stream (see TT_FLAG_POLL). */
int tt_forward(const tt_grid* grid, const double* s, const double* xi, const double* eta,
               int32_t nsrc, const double* src_pos, const double* src_par, const double* tau_init,
               const tt_opts* opts, double* tau, int32_t* status, void* ws, size_t ws_bytes,
               void* stream);

/* tt_forward for callers that cannot allocate (code under hipGraph capture,
 * tight serving loops, harnesses that forbid allocation): the same solve with
 * the same arguments and results, but no caller workspace -- the workspace is
 * a fixed device array inside the library, tt_forward_noalloc_limit() bytes
 * (64 MiB) per device, held from the library's first use on that device until
 * the process ends.  The call allocates nothing (no device, pinned or graph
 * memory, no streams or events): one source group on `stream`, asynchronous.
 * Limits and errors: TT_EINVAL if the workspace this grid, batch and tile
 * depth need (tt_workspace_size with groups = 1) exceeds the array, or if
 * opts asks for TT_FLAG_POLL, TT_FLAG_TIME_SWEEPS or TT_FLAG_GRAPH (each
 * needs an allocation); otherwise as tt_forward.  Every call on one device
 * shares that device's array, whose contents are whatever the last call left
 * (the solve initialises everything it reads): calls that overlap in time on
 * one device -- on different streams or host threads -- race and give wrong
 * results; serialise them. */
int tt_forward_noalloc(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
                       const double* src_pos, const double* src_par, const double* tau_init, const tt_opts* opts,
                       double* tau, int32_t* status, void* stream);
size_t tt_forward_noalloc_limit(void);

/* Traveltimes at receivers, T(x_r) = sum_c w_c T0(c) tau(c) over the trilinear
 * corners c of the receiver's cell (receiver term of Eqs. (2), (3)).
 *   tau [nsrc][N], rec_pos [nrec][3], T_rec out [nsrc][nrec]. */
int tt_sample(const tt_grid* grid, int32_t nsrc, const double* src_pos, const double* src_par,
              const double* tau, int32_t nrec, const double* rec_pos, double* T_rec, void* ws,
              size_t ws_bytes, void* stream);

/* Relocation (Eq. (10), App. B).  By reciprocity the time from earthquake n
 * to receiver m is Gamma_m(x_n) + t_n, Gamma_m the traveltime field with
 * receiver m taken as the source (tt_forward with the receivers as sources,
 * nfield of them), t_n the earthquake's origin-time shift.  The misfits of
 * Eqs. (B1)-(B3) are then tt_misfit / tt_misfit_cr of T[n][m], whose adjoint
 * sources R = d chi / d T are d chi / d Gamma_m(x_n).
 *   field_pos [nfield][3], field_par [nfield][3] (tt_source_params of the
 *   receivers), tau [nfield][N] their converged fields; ev_pos [nev][3].
 *   Workspace: tt_workspace_size(grid, nfield, NULL, 2) bytes.
 * tt_reloc_times: T [nev][nfield] = Gamma_m(x_n) + t_n, Gamma_m sampled by its
 *   trilinear interpolant; ev_t0 [nev] or NULL (= 0).
 * tt_reloc_kernel: K [nev][4] = (sum_m R[n][m] dGamma_m/dx_a(x_n), a = 0, 1, 2,
 *   sum_m R[n][m]) = (the location kernel of Eq. (10) in grid coordinates --
 *   r km, latitude rad, longitude rad, or z, y, x km -- and K_tau), with
 *   R [nev][nfield].  The gradient is that of the trilinear interpolant inside
 *   the cell that samples x_n, so K is the exact derivative of the sampled
 *   misfit.  Deterministic.  Both asynchronous on stream. */
int tt_reloc_times(const tt_grid* grid, int32_t nfield, const double* field_pos, const double* field_par,
                   const double* tau, int32_t nev, const double* ev_pos, const double* ev_t0, double* T, void* ws,
                   size_t ws_bytes, void* stream);
int tt_reloc_kernel(const tt_grid* grid, int32_t nfield, const double* field_pos, const double* field_par,
                    const double* tau, int32_t nev, const double* ev_pos, const double* R, double* K, void* ws,
                    size_t ws_bytes, void* stream);

/* Misfit chi = alpha*chi_t + beta*chi_cs (Eqs. (1)-(3)) and adjoint sources
 * R = d chi / d T(x_r) (Eqs. (A1)-(A3)).
 *   T_rec, T_obs [nsrc][nrec]; w [nsrc][nrec] or NULL (= 1);
 *   pairs [npair][2] receiver index pairs shared by every source, each
 *   unordered pair listed once (npair may be 0, pairs NULL); wpair
 *   [nsrc][npair] or NULL (= 1).
 *   R out [nsrc][nrec]; chi out [1] (device scalar).
 * A pair index outside [0, nrec) is skipped and makes chi NaN.  Does not wait. */
int tt_misfit(int32_t nsrc, int32_t nrec, const double* T_rec, const double* T_obs, const double* w,
              int32_t npair, const int32_t* pairs, const double* wpair, double alpha, double beta,
              double* R, double* chi, void* stream);

/* Common-receiver differential misfit gamma*chi_cr (Eq. (4), third misfit)
 * and its adjoint sources (Eq. (A4)), ADDED to R and chi: call it after
 * tt_misfit on the same stream for chi = alpha*chi_t + beta*chi_cs +
 * gamma*chi_cr (Eq. (1)).  The source pairs are grouped by receiver:
 *   cr_off [nrec + 1] (device int32): the pairs recorded at receiver m are
 *       numbers cr_off[m] .. cr_off[m+1]-1; cr_off[0] = 0 and non-decreasing;
 *   cr_pair [cr_off[nrec]][2] (device int32) source indices (n, j), each
 *       unordered pair at one receiver listed once (NULL if cr_off[nrec] = 0);
 *   wcr [cr_off[nrec]] weights w_{n,j|m}, or NULL (= 1).
 *   T_rec, T_obs [nsrc][nrec]; R in/out [nsrc][nrec]; chi in/out (device
 *   scalar).  A negative or decreasing offset, pairs with cr_pair NULL, or a
 *   source index outside [0, nsrc) is skipped and makes chi NaN.  Pairs of one receiver are applied in list
 *   order (deterministic).  Does not wait. */
int tt_misfit_cr(int32_t nsrc, int32_t nrec, const double* T_rec, const double* T_obs, const int32_t* cr_off,
                 const int32_t* cr_pair, const double* wcr, double gamma, double* R, double* chi, void* stream);

/* Adjoint solve (Sec. 2.1 step 2, Eq. (5)) as the exact transpose of the
 * discrete forward system at the converged tau: J^T lambda = d chi / d tau with
 * d chi / d tau(c) = sum_m R_m w_c(m) T0(c).  Gauss-Seidel sweeps in the same 8
 * directions and tiles, each followed by the transposed boundary pass.
 *   tau [nsrc][N] converged forward fields; rec_pos [nrec][3];
 *   R [nsrc][nrec] adjoint sources (e.g. from tt_misfit);
 *   lam [nsrc][N] out: adjoint field (0 on boundary rows of fixed nodes);
 *       in/out with TT_FLAG_ADJOINT_INIT (its initial field);
 *   status [nsrc] out: as for tt_forward; the convergence measure is
 *   sum|d lambda| / sum|lambda| over one iteration.
 * Asynchronous on stream (see TT_FLAG_POLL). */
int tt_adjoint(const tt_grid* grid, const double* s, const double* xi, const double* eta,
               int32_t nsrc, const double* src_pos, const double* src_par, const double* tau,
               int32_t nrec, const double* rec_pos, const double* R, const tt_opts* opts,
               double* lam, int32_t* status, void* ws, size_t ws_bytes, void* stream);

/* Sensitivity kernels (Eqs. (6)-(8)) as discrete gradients summed over sources
 * in ascending source order (Eq. (9) relates them to K_s, K_xi, K_eta):
 *   grad[0] = d chi/d s   = sum_n lambda_n,
 *   grad[1] = d chi/d xi  = sum_n lambda_n (P_theta^2 - P_phi^2) / H,
 *   grad[2] = d chi/d eta = sum_n -2 lambda_n P_theta P_phi / H,
 * zero on boundary and fixed nodes.  grad [3][N]; accumulate != 0 adds to it. */
int tt_kernel(const tt_grid* grid, const double* s, const double* xi, const double* eta, int32_t nsrc,
              const double* src_pos, const double* src_par, const double* tau, const double* lam,
              double* grad, int32_t accumulate, void* ws, size_t ws_bytes, void* stream);

/* Kernel-density normalisation (Eqs. (18)-(19)).  The density of the event
 * kernels is the adjoint field of Eq. (5) with every adjoint source R = 1,
 * summed over sources: run tt_adjoint with R = 1 and tt_kernel on its fields,
 * and pass the s-gradient row of the result as dens [N].  With V the
 * trapezoidal node volume (r^2 cos(theta) dr dtheta dphi in spherical
 * coordinates, halved once per boundary axis), and since
 * K_s = s (d chi / d s) / V (Eq. (9)) and K_s = P s^2, per node:
 *   Kd   = dens / (s V)                                  (Eq. (19))
 *   K[0] = s grad[0] / V / (Kd + eps)^zeta   (K_s)        (Eq. (18))
 *   K[1] = grad[1] / V / (Kd + eps)^zeta     (K_xi),  K[2] likewise (K_eta).
 * grad [3][N] are the summed discrete gradients of the misfit (tt_kernel);
 * K [3][N] out; Kd [N] out (may be NULL).  eps >= 0, zeta finite (eps > 0 when
 * zeta is not an integer and Kd can be 0).  Asynchronous on stream. */
int tt_kernel_density(const tt_grid* grid, const double* s, const double* dens, const double* grad, double eps,
                      double zeta, double* K, double* Kd, void* stream);

/* Multiple-grid parameterisation (Eqs. (11)-(17)).  H (1..TT_MG_MAX_GRIDS)
 * inversion grids; grid q
 * has m[3q + a] (>= 1) strictly ascending node coordinates on axis a (r km,
 * latitude, longitude rad; or z, y, x km), concatenated in coords (device,
 * grid after grid, axes in turn).  Basis B = u v w / H with the tents of
 * Eqs. (12)-(14), which vanish outside each grid's coordinate range.
 * Coefficients and projections are stored per grid as [3][m0][m1][m2] (k
 * fastest; the paper's index l = i + m0 j + m0 m1 k names the same entries),
 * grids in turn; the three rows are the s, xi, eta parameters.  m is a host
 * array; every other pointer is device memory.
 *
 * tt_mg_project: out = d chi / d C (Eq. (17)) from the kernels K [3][N] (e.g.
 *   tt_kernel_density), by node quadrature: out = sum_x K(x) B(x) V(x).  With
 *   ds / s = sum C B (s row) and dxi = sum C B, d eta likewise (Eq. (15)), this
 *   is the gradient of Eq. (16).  B and V factor over the axes, so the sum is
 *   taken one axis at a time (K read once, partial sums in ws); grids whose
 *   staging does not fit in LDS take one wave per inversion node instead (no
 *   workspace).  Deterministic.  ws: device memory of at least
 *   tt_mg_workspace_size(grid, H, m) bytes (may be NULL when that is 0).
 * tt_mg_expand: field [3][N] = sum over grids and nodes of C B (Eq. (15)),
 *   overwritten.  Asynchronous on stream. */
#define TT_MG_MAX_GRIDS 16
size_t tt_mg_workspace_size(const tt_grid* grid, int32_t H, const int32_t* m);
int tt_mg_project(const tt_grid* grid, int32_t H, const int32_t* m, const double* coords, const double* K,
                  double* out, void* ws, size_t ws_bytes, void* stream);
int tt_mg_expand(const tt_grid* grid, int32_t H, const int32_t* m, const double* coords, const double* C,
                 double* field, void* stream);

/* Sweep-kernel timing gathered by tt_forward (which = 0) and tt_adjoint
 * (which = 1) calls of the calling thread that had TT_FLAG_TIME_SWEEPS set:
 * the summed device time of the timed sweeps (ms, HIP event pairs around the
 * back-to-back tile-plane launches of each directional sweep) and the number
 * of sweep-kernel launches they contain.  reset != 0 clears the totals after
 * reading.  Pointers may be NULL. */
int tt_sweep_timing(int32_t which, double* total_ms, int64_t* launches, int32_t reset);

/* The tile depth (tt_opts.tile_k) that tile_k = 0 selects: which = 0
 * tt_forward, 1 tt_adjoint; 0 for any other value. */
int32_t tt_default_tile_k(int32_t which);

/* Message for the last nonzero return of the calling thread ("" if none). */
const char* tt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TT_H */
