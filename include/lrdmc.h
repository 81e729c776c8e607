/*
 * lrdmc.h -- C ABI of the double-grid lattice-regularized diffusion Monte
 * Carlo (LRDMC) projection library for AMD Instinct MI355X (gfx950).
 *
 * Method: Nakano, Maezono & Sorella, "Speeding up the ab initio diffusion
 * Monte Carlo by a smart lattice regularization", arXiv:1909.01589.
 *   - main text Eq. (1): the kinetic Laplacian is split into a small-spacing
 *     part (a, weighted by p) and a large-spacing part (a', weighted by 1-p);
 *   - main text Eq. (3): p(r) = exp(-|r - R_c|^2 / 2 r_c^2), R_c the nearest
 *     nucleus; for molecules only the heaviest nuclei count ("Application
 *     to large systems");
 *   - main text Eq. (6)-(7) and supplement Eq. (S-13): the choice of r_c and
 *     a'/a (lrdmc_spacing).
 * The projection itself (finite-difference stencil, regularized potential,
 * fixed-node rule, continuous-time moves, fixed-population reconfiguration)
 * is the lattice-regularized DMC the paper builds on (its refs. Casula,
 * Filippi & Sorella 2005; Becca & Sorella 2017).
 *
 * Conventions
 *   - All floating point is FP64.  Arrays are row-major and C-contiguous.
 *   - Host pointers: the system and parameter descriptions of lrdmc_create
 *     (deep-copied; the caller may free them on return) and the outputs of
 *     lrdmc_spacing.  Every other array argument is a DEVICE pointer on the
 *     current HIP device (for instance the data pointer of a torch tensor);
 *     the caller owns it.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Entry points
 *     that take a stream enqueue their work on it and return after
 *     synchronizing it, so that errors found by the kernels are reported by
 *     the call that caused them.
 *   - Return value 0 on success, else a negative LRDMC_E* code; the message
 *     of the last failure of a context (with the walker index for per-walker
 *     failures) is returned by lrdmc_last_error.  After a non-zero return no
 *     output is promised to be complete.
 *   - Electron order: the n_up spin-up electrons first, then n_dn spin-down.
 *     A walker is pos[N][3], N = n_up + n_dn; W walkers are pos[W][N][3].
 *   - Moves: electron i has M/N = 12 lattice moves, index m = 12 i + 6 g + d,
 *     g = 0 for spacing a (weight p/a^2), g = 1 for a' (weight (1-p)/a'^2),
 *     d = 2 axis + (0 for +, 1 for -).  p is evaluated at the midpoint of the
 *     move.  With rotate != 0 the three axes are the columns of a uniform
 *     random rotation drawn for every move.
 *   - Random numbers: Philox4x64-10 with key (seed, 0) and counter
 *     (slot, generation, iteration, purpose); purpose 0 gives (u1, u2) of a
 *     move, 1 the rotation, 2 a Metropolis step (lrdmc_vmc), 3 the
 *     resampling offset at slot 2^64-1.
 *
 * Thread safety: a context may be used by one host thread at a time.
 */
#ifndef LRDMC_H
#define LRDMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRDMC_OK          0
#define LRDMC_EINVAL     -1  /* bad sizes or parameters                        */
#define LRDMC_ESINGULAR  -2  /* a Slater matrix is singular or non-finite      */
#define LRDMC_ENONFINITE -3  /* NaN/Inf in an energy, a weight or a position   */
#define LRDMC_ENOMEM     -4  /* host or device allocation failed               */
#define LRDMC_EDEVICE    -5  /* HIP runtime error                              */
#define LRDMC_ECOLLAPSE  -6  /* population collapse (lrdmc_set_collapse_threshold) */
#define LRDMC_EITERCAP   -7  /* a walker reached the move cap of a generation   */

/* Number of per-walker diagnostics written by lrdmc_eval_moves. */
#define LRDMC_NDIAG 9

typedef struct lrdmc_ctx lrdmc_ctx;

/* Trial function Psi = det A_up det A_dn exp(J).
 * Basis: shell q is an uncontracted, unnormalized Gaussian
 * P_l(d) exp(-alpha_q |d|^2), d = r - R[shell_nuc[q]], l = shell_l[q] in
 * {0,1,2} giving 1, 3 or 5 functions (p: x, y, z; d: xy, yz, zx, x^2-y^2,
 * 2z^2-x^2-y^2); K = sum of (2l+1).  Orbitals phi_j = sum_mu mo[mu][j] g_mu,
 * mo is [K][n_orb] and shared by both spins; the spin-sigma determinant uses
 * orbitals 0..n_sigma-1.  Jastrow (Pade):
 * J = sum_{i<j} c_ij r_ij/(1 + b_ee r_ij) - sum_{i,I} Z_I r_iI/(1 + b_en r_iI),
 * c_ij = 1/2 for opposite spins and 1/4 for equal spins (exact cusps). */
typedef struct {
    int32_t n_nuc;
    const double *Z;            /* [n_nuc] nuclear charges                   */
    const double *R;            /* [n_nuc][3] positions (bohr)               */
    int32_t n_up, n_dn;
    int32_t n_shell;
    const int32_t *shell_nuc;   /* [n_shell]                                 */
    const int32_t *shell_l;     /* [n_shell]                                 */
    const double *shell_alpha;  /* [n_shell]                                 */
    int32_t n_orb;
    const double *mo;           /* [K][n_orb]                                */
    double b_ee, b_en;
} lrdmc_system;

/* Lattice and projection parameters.
 * a: small (core) spacing; a_prime: large spacing, a_prime >= a;
 * r_c: parameter of the switch p (main text Eq. (3): width of the Gaussian;
 * Eq. (2): inverse length of the Pade form); nuclei with Z >= z_heavy
 * define R_c; tau: projection time per generation (1/Ha); seed: Philox key;
 * rotate: random lattice orientation per move (0 = fixed x, y, z axes);
 * refresh: generations between recomputations of a walker's inverse Slater
 * matrices and derivative tables from its positions.  0 or 1 recomputes at
 * every generation start; R > 1 keeps the Sherman-Morrison-updated state in
 * device memory and recomputes it at generations that are multiples of R
 * (and after lrdmc_set_walkers).  The results agree up to rounding. */
typedef struct {
    double a, a_prime, r_c, z_heavy, tau;
    uint64_t seed;
    int32_t rotate;
    int32_t refresh;
    int32_t switch_form;        /* 0: Gaussian p of Eq. (3) (this paper's     */
                                /* scheme); 1: Pade p of Eq. (2) (the earlier */
                                /* scheme, with lrdmc_spacing_pade)           */
    int32_t grids;              /* 2 (or 0): double grid, 12N moves; 1: single */
                                /* grid of spacing a, p = 1, 6N moves          */
} lrdmc_params;

/* Host-side parameter choice of the paper for heaviest charge Z and small
 * spacing a: r_c(a,Z) = beta (kappa alpha^-2 + 1)/(alpha^-2 + 1) Z^(-5/7),
 * alpha = 1/(a Z) (supplement Eq. (S-13)); N_core(r_c) from a Slater-rule
 * atomic density (main text Eq. (7)); a' = a sqrt((Z - N_core)/N_core)
 * (main text Eq. (6)).  The paper uses beta = 0.75, kappa = 2.5.
 * Outputs are host pointers; n_core may be NULL.
 * Errors: LRDMC_EINVAL for Z < 1, Z > 86, a <= 0, beta <= 0 or kappa <= 0. */
int lrdmc_spacing(double Z, double a, double beta, double kappa,
                  double *r_c, double *a_prime, double *n_core);

/* The earlier parametrization the paper compares against, for use with the
 * Pade switch (switch_form = 1): r_c = Z/2 in Eq. (2) and
 * a'/a = sqrt(Z^2/4 + 1) (main text Eq. (4)).  Host pointers.
 * Errors: LRDMC_EINVAL for Z <= 0 or a <= 0. */
int lrdmc_spacing_pade(double Z, double a, double *r_c, double *a_prime);

/* Create a context for n_walkers walkers on the current HIP device.
 * Deep-copies sys and prm to the device and allocates the walker state.
 * Errors: LRDMC_EINVAL (n_walkers < 1; n_up < 1; n_dn < 0; max(n_up, n_dn)
 * > 32; N > 64; n_orb < max(n_up, n_dn); K > 512; n_nuc < 1 or > 64; l
 * outside 0..2; alpha < 0; a <= 0; a_prime < a; r_c <= 0; tau <= 0; no
 * nucleus with Z >= z_heavy; refresh < 0), LRDMC_ENOMEM, LRDMC_EDEVICE. */
int lrdmc_create(const lrdmc_system *sys, const lrdmc_params *prm,
                 int32_t n_walkers, lrdmc_ctx **out);

/* Load walker positions pos[W][N][3] (device) and set the generation counter
 * that keys the random numbers of the next projection.  Clears any pending
 * reconfiguration.  Errors: LRDMC_EINVAL (NULL pointers). */
int lrdmc_set_walkers(lrdmc_ctx *ctx, const double *pos, uint64_t generation, void *stream);

/* One generation of projection (no reconfiguration): every walker slot s
 * starts with log w = 0 and projection time tau and, in continuous time,
 * waits tau_d = -ln(u1)/Delta(x), multiplies its weight by exp(-tau_d e_L(x))
 * and moves along lattice move m with probability T_m/Delta(x), until the
 * time is used up.  Delta(x) = sum_m T_m, T_m = k_m max(rho_m, 0)/2,
 * rho_m = Psi(x'_m)/Psi(x) (fixed node: moves with rho_m <= 0 are dropped).
 * If a reconfiguration is pending, slot s starts from the copy it selected.
 * Errors: LRDMC_ESINGULAR, LRDMC_ENONFINITE (with the slot index),
 * LRDMC_EITERCAP (a walker reached the move cap of lrdmc_set_move_cap in
 * one generation; with the slot index),
 * LRDMC_EDEVICE. */
int lrdmc_project(lrdmc_ctx *ctx, void *stream);

/* Fixed-population reconfiguration after a projection (systematic
 * resampling with one offset xi drawn from the counter stream):
 * w_j = exp(log w_j - max), t_s = (s + xi) sum(w)/W, idx_s = first j with
 * cumulative weight > t_s.  Writes the generation record at the device
 * pointers (each may be NULL): log_wbar = log(mean w) (including the max),
 * ebar = sum w_j e_L,j / sum w_j, n_moves = total moves of the generation,
 * ess = effective sample size (sum w)^2 / sum w^2 of the weights (W for
 * equal weights, 1 when one walker carries all the weight); idx (device,
 * [W] int32, may be NULL).  Advances the generation counter.
 * Errors: LRDMC_EINVAL (no projection since the last reconfiguration),
 * LRDMC_ENONFINITE, LRDMC_ECOLLAPSE (the weights' effective sample size
 * (sum w)^2 / sum w^2 fell below the collapse threshold times W; the
 * reconfiguration and the record are still written), LRDMC_EDEVICE. */
int lrdmc_branch(lrdmc_ctx *ctx, void *stream, double *log_wbar, double *ebar,
                 int64_t *n_moves, int32_t *idx, double *ess);

/* n_gen x (lrdmc_project + lrdmc_branch) without host synchronization in
 * between.  Device outputs (each may be NULL): log_wbar[n_gen], ebar[n_gen],
 * n_moves[n_gen], idx[n_gen][W], ess[n_gen].  Errors as for lrdmc_project and
 * lrdmc_branch; the first error of the run is reported (a population
 * collapse names its generation) and the remaining generations still run. */
int lrdmc_run(lrdmc_ctx *ctx, int32_t n_gen, void *stream, double *log_wbar,
              double *ebar, int64_t *n_moves, int32_t *idx, double *ess);

/* Copy the walker state to device buffers (each may be NULL): pos[W][N][3],
 * log_w[W], e_loc[W] (analytic local energy), n_moves[W] (moves of the last
 * projection).  After a reconfiguration, slot s holds the copy it selected,
 * with log_w = 0 and n_moves = 0. */
int lrdmc_get_walkers(lrdmc_ctx *ctx, double *pos, double *log_w, double *e_loc,
                      int32_t *n_moves, void *stream);

/* Check of the Sherman-Morrison-carried state (a diagnostic): for every
 * walker slot, res[s] (device [W]) = max |(A Ainv - I)_ik| over both spins,
 * with A recomputed from the walker's current positions and Ainv the inverse
 * stored in its state, carried by rank-one updates since the last refresh
 * (a residual far above rounding means the updates have drifted).  After a
 * reconfiguration slot s reports the walker it selected.  Synchronizes the
 * stream.  Errors: LRDMC_EINVAL (NULL; refresh <= 1 or no projection since the
 * walkers were set, so no state is stored), LRDMC_EDEVICE. */
int lrdmc_inverse_residual(lrdmc_ctx *ctx, double *res, void *stream);

/* Evaluate the move table at frozen positions pos[W][N][3] without moving:
 * rho[W][M] = Psi(x'_m)/Psi(x), k[W][M] = hopping coefficient of move m,
 * M = 12 N, and diag[W][LRDMC_NDIAG] =
 *   {E_L analytic, e_L lattice-assembled, L^a = sum_m k_m (rho_m - 1),
 *    sum_i lap_i Psi/Psi, V^a, V_sf, Delta, V, sum_m k_m},
 * with V^a = V + (L^a - lap Psi/Psi)/2, V_sf = -1/2 sum_{rho<0} k rho and
 * e_L = sum k/2 + V^a + V_sf - Delta.  The axes are those of iteration 0 of
 * the current generation (identity if rotate == 0).  Any output may be NULL.
 * Errors: LRDMC_ESINGULAR, LRDMC_ENONFINITE, LRDMC_EDEVICE. */
int lrdmc_eval_moves(lrdmc_ctx *ctx, const double *pos, double *rho, double *k,
                     double *diag, void *stream);

/* Stateless reconfiguration of W walkers with given offset xi in (0,1):
 * log_w[W], e_loc[W] (device) -> idx[W] (device int32) and stats[2] (device:
 * log_wbar, ebar; may be NULL).  Allocates a W-double scratch buffer on the
 * stream.  Errors: LRDMC_EINVAL (W < 1, xi outside (0,1)), LRDMC_ENONFINITE,
 * LRDMC_ENOMEM, LRDMC_EDEVICE. */
int lrdmc_reconfigure(const double *log_w, const double *e_loc, int32_t W, double xi,
                      int32_t *idx, double *stats, void *stream);

/* lrdmc_reconfigure for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and results, with the cumulative-weight
 * scratch in a fixed device array of LRDMC_NOALLOC_MAX_WALKERS doubles per
 * GPU (8 MiB, held until the process ends) instead of a stream allocation.
 * The call allocates nothing; it synchronizes the stream.  All calls on one
 * GPU share that array, so calls that overlap on one GPU (other streams or
 * host threads) race; sequential calls are independent.
 * Errors: LRDMC_EINVAL (W < 1, W > LRDMC_NOALLOC_MAX_WALKERS, xi outside
 * (0,1)), LRDMC_ENONFINITE, LRDMC_EDEVICE. */
#define LRDMC_NOALLOC_MAX_WALKERS (1 << 20)
int lrdmc_reconfigure_noalloc(const double *log_w, const double *e_loc, int32_t W, double xi,
                              int32_t *idx, double *stats, void *stream);

/* Kernel timing with HIP events recorded on the launch stream around every
 * projection and reconfiguration kernel of lrdmc_project, lrdmc_branch and
 * lrdmc_run.  enable != 0 clears the totals and starts accumulating, 0 stops.
 * lrdmc_timing writes (host) out[4] = {projection kernel ms, projection
 * launches, reconfiguration kernel ms, reconfiguration launches}.
 * Errors: LRDMC_EINVAL (NULL), LRDMC_EDEVICE. */
int lrdmc_set_timing(lrdmc_ctx *ctx, int32_t enable);
int lrdmc_timing(const lrdmc_ctx *ctx, double *out);

/* Derivatives of the trial function's Jastrow exponent J (Pade e-e and e-n
 * terms, cusp coefficients fixed) and of the local energy with respect to the
 * two Pade parameters theta = (b_ee, b_en), at the W walker configurations
 * pos (device [W][N][3], walker-major): the gradients that optimize the trial
 * function by variance minimisation before the projection.
 * out (device [W][6]): {E_L, J, dJ/db_ee, dJ/db_en, dE_L/db_ee, dE_L/db_en}.
 * Synchronizes the stream.  Errors: LRDMC_EINVAL (NULL), LRDMC_ESINGULAR,
 * LRDMC_ENONFINITE (walker slot in lrdmc_last_error), LRDMC_EDEVICE. */
int lrdmc_jastrow_grad(lrdmc_ctx *ctx, const double *pos, double *out, void *stream);

/* Replace the Pade parameters of ctx's Jastrow factor (finite, >= 0).  Later
 * projections, evaluations and gradients use them; walker states stored from
 * earlier projections are recomputed.  Errors: LRDMC_EINVAL. */
int lrdmc_set_jastrow(lrdmc_ctx *ctx, double b_ee, double b_en);

/* Variational Monte Carlo sampling of |Psi|^2 (the variational stage the
 * supplement's computational details run before the projection; Metropolis
 * algorithm): every walker takes n_steps single-electron moves.  Step t of
 * generation g of walker slot s draws (u0, u1, u2, u3) from the random
 * stream at counter (s, g, t, purpose 2): electron i = floor(u0 N) moves by
 * step * e, e on the unit sphere with cos(theta) = 2 u1 - 1, phi = 2 pi u2
 * (a symmetric proposal), accepted when u3 < (Psi(x')/Psi(x))^2.  Starts from
 * the current walkers (after a pending reconfiguration), replaces them,
 * advances the generation counter by one and sets log w = 0; lrdmc_get_walkers
 * then returns E_L at the final positions and the accepted count in n_moves.
 * The trial function includes the learned correction when one is set.
 * Synchronizes the stream.  Errors: LRDMC_EINVAL (no walkers, n_steps < 0,
 * step not finite and > 0), LRDMC_ESINGULAR, LRDMC_ENONFINITE, LRDMC_EDEVICE. */
int lrdmc_vmc(lrdmc_ctx *ctx, int32_t n_steps, double step, void *stream);

/* Learned correction of the Jastrow factor.  The supplement's computational
 * details use Jastrow-Slater trial functions whose Jastrow parameters are all
 * optimized; this adds a radial function learned by variance minimisation to
 * each pair term: J += sum_{i<j} F_ee(r_ij) + sum_{i,I} Z_I F_en(r_iI), with
 * F = 0 from r_cut on.  F is given by its node table
 * tab[2][n_nodes][3] = {F, F', F''} at r_k = k r_cut / (n_nodes - 1)
 * (type 0: electron pairs, 1: electron-nucleus) and is, between nodes, the
 * quintic that matches value, first and second derivative at both ends
 * (twice continuously differentiable).  The Pade cusps stay exact when
 * F'(0) = 0.  tab is a host array (on_device = 0, copied) or a device
 * array (on_device = 1, read on `stream`); the call synchronizes the stream.
 * tab = NULL or n_nodes = 0 removes the correction.  Later projections,
 * evaluations and gradients use the table; stored walker states are
 * recomputed.  Errors: LRDMC_EINVAL (2 <= n_nodes <= LRDMC_MAX_TABLE_NODES,
 * finite r_cut > 0, every entry finite; after a non-finite entry the
 * correction is removed), LRDMC_ENOMEM, LRDMC_EDEVICE. */
#define LRDMC_MAX_TABLE_NODES 4096
int lrdmc_set_jastrow_table(lrdmc_ctx *ctx, const double *tab, int32_t n_nodes, double r_cut,
                            int32_t on_device, void *stream);

/* Gradient with respect to the node table of the learned correction:
 * gtab (device [2][n_nodes][3], overwritten) = d/dtab sum_w (c_j[w] J_w +
 * c_e[w] E_L,w) over the W walker configurations pos (device [W][N][3]);
 * c_j, c_e are device [W] (either may be NULL for zero).  J and E_L are the
 * values lrdmc_jastrow_grad returns; the backward pass of a loss on them.
 * Accumulated with hardware floating-point atomics: the summation order
 * varies from call to call (differences at rounding level), and gtab must be
 * ordinary device memory (hipMalloc or a device tensor), not host-mapped or
 * fine-grained memory.  Synchronizes the stream.
 * Errors: LRDMC_EINVAL (NULL, no table set), LRDMC_ESINGULAR,
 * LRDMC_ENONFINITE, LRDMC_EDEVICE. */
int lrdmc_jastrow_table_grad(lrdmc_ctx *ctx, const double *pos, const double *c_j, const double *c_e,
                             double *gtab, void *stream);

/* The network that produces the correction's node table (the trial
 * function's learned Jastrow part; parameters optimized by the caller, as the
 * supplement's computational details optimize every Jastrow parameter).  Per
 * pair type (0: electron pairs, 1: electron-nucleus) a network 1 -> H -> H
 * -> 1 with SiLU activations silu(z) = z / (1 + exp(-z)):
 * g(x) = w3 . silu(W2 silu(W1 x + b1) + b2) + b3 at x = r / r_cut, and
 * f(r) = r^2 (1 - r/r_cut)^3 g(r/r_cut), so that f(0) = f'(0) = 0 (cusps of
 * the Pade part stay exact) and f, f', f'' vanish at r_cut.
 * params (device [2][P], P = lrdmc_net_param_count(H) = H^2 + 4H + 1), per
 * network in this order: W1[H], b1[H], W2[H][H] (row-major, row = output
 * unit), b2[H], w3[H], b3.
 * lrdmc_net_tabulate writes tab (device [2][n_nodes][3]) = {f, f', f''} at
 * r_k = k r_cut / (n_nodes - 1): the input of lrdmc_set_jastrow_table.
 * lrdmc_net_tabulate_backward writes gparams (device [2][P], overwritten) =
 * sum over the table of gtab * d tab / d params, given gtab (device
 * [2][n_nodes][3]); work is device scratch of lrdmc_net_workspace_size(H,
 * n_nodes) doubles.  Both are asynchronous on `stream` (no host
 * synchronization); the reduction order is fixed (deterministic).
 * lrdmc_net_param_count and lrdmc_net_workspace_size return 0 for sizes out
 * of range.  Errors: LRDMC_EINVAL (NULL, 1 <= H <= 256,
 * 2 <= n_nodes <= LRDMC_MAX_TABLE_NODES, finite r_cut > 0), LRDMC_EDEVICE
 * (launch failure); message in lrdmc_last_error(NULL). */
int32_t lrdmc_net_param_count(int32_t hidden);
int64_t lrdmc_net_workspace_size(int32_t hidden, int32_t n_nodes);
int lrdmc_net_tabulate(const double *params, int32_t hidden, int32_t n_nodes, double r_cut, double *tab,
                       void *stream);
int lrdmc_net_tabulate_backward(const double *params, int32_t hidden, int32_t n_nodes, double r_cut,
                                const double *gtab, double *gparams, double *work, void *stream);

/* Kernel selection.  The library carries, besides the projection kernel for
 * any system, kernels built for fixed system sizes (electrons per spin, basis
 * functions, nuclei; see LRDMC_FIXED_SHAPES in the kernel source).
 * lrdmc_create picks such a kernel when the system's sizes and LDS layout
 * match one; both compute the same method and agree to rounding.  For large
 * systems (a walker state above 40 KB) the general kernels keep the
 * orbital-projected inverse in the walker's device-memory state instead of
 * LDS, so that more walkers share a compute unit; results are the same.
 * lrdmc_use_generic(ctx, mode) for later launches (comparison and testing):
 * 0 = automatic, 1 = the general kernel, 2 = the general kernel with the
 * inverse in device memory at any size.  Errors: LRDMC_EINVAL (NULL, mode
 * outside 0..2).
 * lrdmc_is_specialized returns 1 when the next projection runs a fixed-size
 * kernel, else 0 (also for NULL). */
int lrdmc_use_generic(lrdmc_ctx *ctx, int32_t enable);
int32_t lrdmc_is_specialized(const lrdmc_ctx *ctx);

/* Arithmetic of the move table for later projections and evaluations.
 * mode 0 (default): FP64 throughout.  mode 1 (mixed precision): in the
 * ratios Psi(x')/Psi(x) of the table, the Jastrow pair
 * terms take 1/r and 1/(1/r + b) from the FP32 hardware estimates (relative
 * error about 2^-22 each) while distances, sums and everything else stay
 * FP64; the local energy, the weights, the Sherman-Morrison updates and the
 * reconfiguration are unchanged.  The ratios then differ from FP64 by about
 * 1e-7 relative and at most by the factor exp(dJ),
 * dJ = 2^-20 (sum_j c_ij / b_ee + sum_I Z_I / b_en) (eta = 2.3e-5 for the 18-electron
 * atom), so move indices agree with the FP64 path only until such a
 * difference decides one.  Energy: the weights keep the FP64 local energy and
 * only the rates T_m change, by factors 1 + d_m with |d_m| <= eta =
 * exp(dJ) - 1; the perturbation of the importance-sampled Hamiltonian has
 * zero column sums, so to first order the fixed-node energy moves by
 * dE = -< sum_m d_m T_m (f(x'_m)/f(x) - 1) > over phi^2 (phi the lattice
 * fixed-node ground state, f = phi/Psi): zero for an exact trial function
 * and at most eta <Delta> max |f'/f - 1|, where the +/- moves cancel the
 * part of f'/f - 1 that is first order in the spacing.  Errors:
 * LRDMC_EINVAL (NULL, mode outside 0..1). */
int lrdmc_set_precision(lrdmc_ctx *ctx, int32_t mode);

/* Population-collapse check of lrdmc_branch and lrdmc_run: a generation
 * whose weights have an effective sample size (sum w)^2 / sum w^2 below
 * min_fraction * W returns LRDMC_ECOLLAPSE (a population of W walkers then
 * carries the statistics of fewer than min_fraction W; the projection time
 * per generation is too long for the trial function, or the trial function
 * is poor).  Default 0 (off); 0.01 is the usual criterion.
 * Errors: LRDMC_EINVAL (NULL, min_fraction outside [0, 1]). */
int lrdmc_set_collapse_threshold(lrdmc_ctx *ctx, double min_fraction);

/* Move cap of lrdmc_project and lrdmc_run: a walker that makes max_moves
 * moves in one generation stops there and the call returns LRDMC_EITERCAP
 * with its slot (so that every wave ends even when Delta(x) tau is
 * pathologically large).  Default and maximum 2^22.
 * Errors: LRDMC_EINVAL (NULL, max_moves outside 1..2^22). */
int lrdmc_set_move_cap(lrdmc_ctx *ctx, int32_t max_moves);

/* Generation counter of the next projection. */
uint64_t lrdmc_generation(const lrdmc_ctx *ctx);

/* Message of the last failure of ctx (or of the last failing call without a
 * context when ctx is NULL).  Valid until the next call on ctx. */
const char *lrdmc_last_error(const lrdmc_ctx *ctx);

/* Free the context and its device memory.  NULL is allowed. */
void lrdmc_destroy(lrdmc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LRDMC_H */
