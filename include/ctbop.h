/*
 * ctbop.h -- C ABI of the MI355X (gfx950) library for the charge-transfer
 * bond-order potential of Si-C (Takamoto et al., arXiv:1802.07871).
 *
 * One call evaluates, for a configuration of atoms, the total energy E, the
 * forces F = -dE/dx and the equilibrated charges q:
 *
 *   E(x) = min over q with sum q = Q of
 *          sum_i [E0_i + chi_i q_i + J_i q_i^2 / 2]
 *        + 1/2 sum_i sum_(j,n)!=(i,0) q_i q_j C_ij(|x_j + n.h - x_i|)
 *        + 1/2 sum_i sum_(j,n) fc(r) [fR(r) - b_ij fA(r)]
 *
 * with the paper's vectorised bond order b_ij (Methods, Eqs. 3-5, expanded as
 * Eq. 7 with two channels and p = 2, normalised so b = 1 without neighbours),
 * environment sums zeta_l,ij over third atoms k (Eq. 2), and the charges
 * minimising the energy at every call (Methods: charges are minimised by
 * conjugate gradients at every step, a constant term E0 sits in the self
 * energy).  The pair terms, angular functions and the shielded, tapered
 * Coulomb kernel C_ij are the stand-in forms documented with the parameter
 * layout below.
 *
 * Conventions
 *   units      Angstrom, eV, e, fs, amu; Coulomb constant is parameter "ke".
 *   types      int32, 0 = Si, 1 = C.
 *   box        host double[9], three cell vectors as rows (x = frac . box),
 *              right-handed; pbc host int[3], nonzero = periodic along that
 *              vector.  Along a non-periodic vector the box should enclose the
 *              atoms (atoms outside are still handled, only more slowly).
 *              Every periodic vector's perpendicular width must be at least
 *              (rc_coul + skin) / 3.
 *   arrays     "_dev" pointers are device memory (HIP), "_host" host memory.
 *              Positions, forces and velocities are SoA: x[0..n), y[0..n),
 *              z[0..n) contiguous (3n doubles).
 *   ownership  every device byte is the caller's: inputs, outputs and the
 *              per-system buffer `sys` (lists, charges for the warm start,
 *              scratch).  The library never allocates device memory.  A
 *              context holds host-side parameters and options, a pinned
 *              host word pair for the solver's flag and, from its first
 *              evaluation on, one stream of its own (default priority) with
 *              two events.
 *   streams    every call enqueues work on the caller's stream (hipStream_t
 *              passed as void*, NULL = default stream).  An evaluation forks
 *              its covalent kernels onto the context's stream after the
 *              neighbour lists and joins them back (an event wait on the
 *              caller's stream) before the Coulomb forces, so the caller's
 *              stream orders every result as usual.  The charge solve
 *              stops on a device-side test, so the host waits on that stream
 *              between batches of solver iterations (cg_check) to read the
 *              flag; with info != NULL it also waits at the end to report.
 *   errors     every function returns a status; 0 = CTBOP_OK.  Errors found on
 *              the device (close contacts, list overflow, charge solve not
 *              converged or not positive definite) land in a status word in
 *              `sys`; they are returned when info != NULL, else read later
 *              with ctbop_status().  On error, outputs are unspecified.
 *              ctbop_last_error() gives a message for the calling thread.
 *
 * Parameter vector (CTBOP_N_PARAMS = 56 doubles), species base = 26 * t:
 *   base+0 A  +1 B  +2 lam1  +3 lam2  +4 R  +5 S  +6 sigma
 *   base+7..13  channel 1: gamma c d h n g alpha
 *   base+14..20 channel 2: gamma c d h n g alpha
 *   base+21 chi  +22 J  +23 gamma_coul  +24 E0  +25 mass
 *   52 B_mix_SiC  53 ke  54 rc_coul  55 p
 * Pair terms fR = A_ij exp(-lam1_ij r), fA = B_ij exp(-lam2_ij r) with A, B, R,
 * S geometric and lam arithmetic means (B_ij times B_mix_SiC for Si-C);
 * fc = 1 below R_ij, 0 above S_ij, half-cosine in between.  Channel l of the
 * centre atom's species: zeta_l,ij = sum_k fc(r_ik) w_l(cos theta_ijk)
 * exp[(alpha_l (r_ij - r_ik))^3], w_l = gamma_l [1 + c_l^2 x^2 / (d_l^2 (d_l^2
 * + x^2))], x = h_l - cos theta.  b_ij = G (sum_l (g_l + zeta_l^n_l)^-p)^(1/(2
 * sigma p)).  Coulomb C_ij(r) = ke T(r/rc) (r^3 + (gamma_i gamma_j)^-3/2)^-1/3
 * with T(x) = (1-x)^4 (1 + 4x + 10x^2 + 20x^3) below the cutoff.
 */
#ifndef CTBOP_H
#define CTBOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CTBOP_N_PARAMS 56

/* status codes */
#define CTBOP_OK               0
#define CTBOP_E_INVAL          1   /* bad argument or geometry                 */
#define CTBOP_E_NOMEM          2   /* sys buffer too small for this system     */
#define CTBOP_E_TOO_CLOSE      3   /* two atoms closer than 0.5 Angstrom        */
#define CTBOP_E_QEQ_NOCONV     4   /* charge solve hit cg_maxit                 */
#define CTBOP_E_QEQ_NOT_PD     5   /* p^T H p <= 0 met in the charge solve      */
#define CTBOP_E_NEIGH_OVERFLOW 6   /* more neighbours than the list capacity    */
#define CTBOP_E_HIP            7   /* a HIP runtime call failed                 */
#define CTBOP_E_BUSY           8   /* serving: request not admitted right now   */

/* flags of ctbop_compute_energy_forces_charges */
#define CTBOP_FLAG_WARM_START    1  /* start the charge solve from the last call's charges */
#define CTBOP_FLAG_FORCE_REBUILD 2  /* rebuild cell bins and lists regardless of motion   */
#define CTBOP_FLAG_EXTRAPOLATE   4  /* with WARM_START: start from the polynomial extrapolation
                                       of the last four (three, two) solutions, cubic
                                       (quadratic, linear), for consecutive MD steps;
                                       ctbop_md_run always does this                        */

typedef struct ctbop_ctx ctbop_ctx;

typedef struct {
    double cg_tol;     /* stop when RMS of the projected charge residual < cg_tol (eV/e); default 1e-9 */
    int    cg_maxit;   /* default 500                                                            */
    double skin;       /* Verlet skin (Angstrom): lists are rebuilt once an atom moved skin/2; 0.6 */
    int    long_cap;   /* Coulomb-list entries per atom (0: 512)                                  */
    int    short_cap;  /* covalent-list entries per atom (0: 64)                                  */
    int    fp64;       /* 1: every pair/triplet term in FP64 (default 0: FP32 terms, FP64 sums)   */
    int    cg_check;   /* charge-solve iterations launched between convergence checks (0: 4);
                          the first batch of a solve on a system buffer is at least as long
                          as that buffer's previous solve (iterations past convergence
                          return at once on the device flag)                                */
    double fq_kappa;   /* charge-dependent covalent coupling (e^-2, >= 0; default 0 = off): the
                          paper's covalent-ionic mixed bond function f_q (Methods, first
                          paragraph) has its form in the authors' earlier paper; the stand-in
                          scales the attraction of every bond (i,j) by exp(-fq_kappa (q_i -
                          q_j)^2), so the bond energy is 1/2 fc (fR - b_ij fA f_q).  The energy
                          is then not quadratic in q; the charges minimise it by projected,
                          preconditioned nonlinear conjugate gradients (Polak-Ribiere, Newton
                          line search) to the same cg_tol on the projected gradient.  Forces
                          are taken at the minimising charges.  Single-system evaluation, MD,
                          NVT, relaxation and the allocation-free call support it; the server,
                          the removal energies and the parameter adjoint return E_INVAL.      */
} ctbop_opts;

typedef struct {
    double energy;      /* total energy (eV)                                   */
    double cg_residual; /* final RMS projected residual of the charge solve    */
    double mu;          /* chemical potential (eV/e) at the solution           */
    int    cg_iters;
    int    rebuilt;     /* 1 if this call rebuilt bins and lists               */
    int    status;      /* device status word (CTBOP_* code)                   */
    int    max_long;    /* largest Coulomb-list row at the last rebuild        */
    int    max_short;   /* largest covalent-list row at the last rebuild       */
    unsigned long long nnz_long;   /* Coulomb-list entries at the last rebuild  */
    unsigned long long nnz_short;  /* covalent-list entries at the last rebuild */
    int    n_rebuild;   /* list rebuilds since this system buffer was set up   */
    unsigned long long cg_iters_total;  /* charge-solve iterations since set-up */
    double cg_res0;     /* starting RMS projected residual of the last solve   */
    unsigned long long nnz_coul;  /* Coulomb entries inside rc at the last assembly */
    unsigned long long nnz_coul_wide; /* of which stored with full (32-bit) indices in the
                                         solver's sliced copy (the rest: 16-bit halo
                                         positions or offsets)                         */
    unsigned long long nnz_coul_slots; /* entry slots the solver's product reads: per
                                          slice of 64 rows, 64 x its longest row */
    unsigned long long n_bonds;        /* covalent bonds (ordered pairs inside S_ij) at the
                                          last evaluation                              */
    unsigned long long n_triplets;     /* ordered bond pairs (i; j, k), j != k, sharing
                                          the centre i: the zeta_l terms (Eq. 2)        */
    unsigned long long nnz_coul_halo;  /* Coulomb entries whose tile stages the charge
                                          direction of its neighbours in on-chip memory
                                          (16-bit halo positions) at the last assembly  */
} ctbop_info;

/* Fill *o with the defaults above. */
void ctbop_default_opts(ctbop_opts *o);

/* Create a context from the flat parameter vector (host, n_params doubles,
 * copied) and options (may be NULL for defaults).  E_INVAL on a malformed
 * vector (n_params != CTBOP_N_PARAMS, non-positive sigma/n/g/p/J). */
int ctbop_create(const double *params_host, int n_params, const ctbop_opts *opts, ctbop_ctx **ctx);
int ctbop_destroy(ctbop_ctx *ctx);

/* Replace the context's parameters (host, copied; the same checks as
 * ctbop_create).  The list radii may change with them, so every system
 * buffer used with this context starts over at its next call (lists rebuilt,
 * cold charge start).  E_BUSY while a server runs on this context. */
int ctbop_set_params(ctbop_ctx *ctx, const double *params_host, int n_params);

/* Bytes of the per-system device buffer for n atoms in this cell.  The buffer
 * is reused across calls for the same system (it keeps the lists, the sort
 * order and the charges for the warm start); its content is opaque. */
int ctbop_system_bytes(ctbop_ctx *ctx, int n, const double *box_host, const int *pbc_host, size_t *bytes);

/* Forget what this context knows of the buffer at `sys`: its next use is
 * set up from scratch (state cleared, lists rebuilt, cold charge start), as
 * for a buffer never seen.  A context recognises a system buffer by its
 * address and geometry; call this whenever the memory at `sys` may have held
 * anything else since this context last used it (for instance a freed
 * buffer whose address the allocator handed out again).  Host-side only,
 * no device work. */
int ctbop_system_reset(ctbop_ctx *ctx, void *sys_dev);

/* Energy, forces and charges (the hot path).
 *   pos_dev   double[3n] SoA positions (any periodic image)
 *   types_dev int32[n]
 *   E_dev     double[1] out; F_dev double[3n] SoA out; q_dev double[n] out
 *   sys_dev   caller buffer of at least ctbop_system_bytes() bytes; pass the
 *             same buffer for successive calls on one system (positions and
 *             species may change between calls: lists are rebuilt once an
 *             atom moved skin/2 or changed species)
 *   info      host pointer or NULL (NULL: no final wait or report)       */
int ctbop_compute_energy_forces_charges(ctbop_ctx *ctx, int n, const double *pos_dev,
                                        const int32_t *types_dev, const double *box_host,
                                        const int *pbc_host, double total_charge, int flags,
                                        void *sys_dev, size_t sys_bytes, double *E_dev,
                                        double *F_dev, double *q_dev, ctbop_info *info,
                                        void *stream);

/* Allocation-free form of the call above, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc): the per-system buffer is a library-owned device
 * array of CTBOP_STATIC_SCRATCH_BYTES per device, held from the first call on
 * that device until the process ends.  The caller passes inputs and outputs
 * as above (device memory, on the current device).  The call itself
 * allocates nothing: no hipMalloc, hipFree, pinned host memory, stream or
 * event, and no timing events even with ctbop_profile on; its covalent
 * kernels run on the caller's stream.  Every call starts over (state
 * cleared, lists rebuilt, charges from zero: no warm start), so results are
 * those of ctbop_compute_energy_forces_charges with flags = 0 on a new
 * buffer.  All calls on one device share the one array: calls that overlap
 * on a device (other streams, other threads, other contexts) race and give
 * undefined results.  E_NOMEM, before any device work, when the system needs
 * more than CTBOP_STATIC_SCRATCH_BYTES (ctbop_system_bytes() gives the need;
 * about 12.5 KB per atom at the default capacities, so up to ~20,000 atoms). */
#define CTBOP_STATIC_SCRATCH_BYTES (256ull << 20)
int ctbop_compute_energy_forces_charges_static(ctbop_ctx *ctx, int n, const double *pos_dev,
                                               const int32_t *types_dev, const double *box_host,
                                               const int *pbc_host, double total_charge, double *E_dev,
                                               double *F_dev, double *q_dev, ctbop_info *info, void *stream);

/* Velocity-Verlet NVE for nsteps of dt_fs, re-evaluating energy, forces and
 * charges (warm-started) every step, lists rebuilt when an atom moved skin/2.
 * x_dev, v_dev (SoA, Angstrom and Angstrom/fs) are updated in place; F_dev
 * (SoA) and q_dev hold the final step's forces and charges; fixed_dev
 * (uint8[n] or NULL): nonzero atoms neither move nor change velocity but
 * still interact (the paper fixes its slab's bottom).  thermo_host (or NULL)
 * receives, for s = 0, every, 2*every, ..., nsteps, the pair (E_pot, E_kin)
 * in eV: 2 * (nsteps / every + 1) doubles.  Waits for the stream at the end. */
int ctbop_md_run(ctbop_ctx *ctx, int n, double *x_dev, double *v_dev, const int32_t *types_dev,
                 const uint8_t *fixed_dev, const double *box_host, const int *pbc_host,
                 double total_charge, double dt_fs, int nsteps, int thermo_every,
                 void *sys_dev, size_t sys_bytes, double *F_dev, double *q_dev,
                 double *thermo_host, ctbop_info *info, void *stream);

/* Gradient of a loss L(E, F, q) with respect to the 56 parameters, at the
 * configuration and equilibrated charges of the last evaluation on `sys_dev`
 * (which must have used the current parameters; E_INVAL otherwise), for
 * force/energy/charge fits (Methods: the parameters are fitted to energies,
 * forces and charges).  The caller gives the seeds
 *   dL_dE       dL/dE (host scalar)
 *   dL_dF_dev   double[3n] SoA dL/dF (device)
 *   dL_dq_dev   double[n] dL/dq (device) or NULL for zero
 * and receives grad_host[56] = dL/dtheta (host).  With the charges defined
 * by  H q + chi = mu 1, sum q = Q,  the result is
 *   w dE/dtheta + d(v.F)/dtheta  at fixed q   (w = dL/dE, v = dL/dF)
 *   - lambda . (dH/dtheta q + dchi/dtheta),   P H P lambda = P a, sum lambda = 0,
 *   a = dL/dq + d(v.F)/dq,
 * where P projects onto sum = 0: one adjoint charge solve (the forward's
 * projected PCG, stopped at a projected residual of cg_tol times its start)
 * and forward-mode (dual-number) passes of the covalent and Coulomb kernels
 * per parameter.  Masses get 0.  adj_ws_dev: caller device scratch of at least
 * ctbop_param_grad_bytes() bytes.  The system buffer's forward state
 * (charges, lists, warm start) is left as it was.  cg_iters (host, may be
 * NULL) gets the adjoint solve's iterations.  Waits for the stream. */
int ctbop_param_grad_bytes(ctbop_ctx *ctx, int n, const double *box_host, const int *pbc_host, size_t *bytes);
int ctbop_param_grad(ctbop_ctx *ctx, int n, const double *box_host, const int *pbc_host, void *sys_dev,
                     size_t sys_bytes, void *adj_ws_dev, size_t adj_bytes, double dL_dE,
                     const double *dL_dF_dev, const double *dL_dq_dev, double *grad_host, int *cg_iters,
                     void *stream);

/* NVT molecular dynamics: the paper runs its growth MD in the NVT ensemble
 * at 2500 K with the bottom of the slab fixed (growth-simulation section);
 * the thermostat is not named, so this is a Nose-Hoover chain of chain_len
 * (1..8) thermostats of period tau_fs on the mobile atoms at T_K kelvin,
 * integrated by a thermostat half step, velocity Verlet and a thermostat
 * half step (time reversible).  Arguments as for ctbop_md_run, plus:
 *   chain_dev    double[2 * chain_len] device, in/out: the thermostat
 *                positions xi_k then velocities vxi_k (zeros for a fresh start;
 *                pass the returned state to continue a run)
 *   thermo_host  NULL or 3 * (nsteps / every + 1) doubles: (E_pot, K, H) for
 *                s = 0, every, ...; K is the kinetic energy of the mobile
 *                atoms and H = E_pot + K + sum_k Q_k vxi_k^2 / 2 + Nf kT xi_1
 *                + kT sum_{k>1} xi_k, the conserved quantity.
 * Nf = 3 N_mobile, less 3 when no atom is fixed; Q_1 = Nf kT tau^2 and
 * Q_k = kT tau^2.  E_INVAL for chain_len outside 1..8, T, tau or dt <= 0, or
 * fewer than two mobile atoms.  Waits for the stream at the end. */
int ctbop_md_run_nvt(ctbop_ctx *ctx, int n, double *x_dev, double *v_dev, const int32_t *types_dev,
                     const uint8_t *fixed_dev, const double *box_host, const int *pbc_host, double total_charge,
                     double dt_fs, int nsteps, int thermo_every, double T_K, double tau_fs, int chain_len,
                     double *chain_dev, void *sys_dev, size_t sys_bytes, double *F_dev, double *q_dev,
                     double *thermo_host, ctbop_info *info, void *stream);

/* Structure relaxation at fixed cell: the paper relaxes its graphene-on-SiC
 * structures and annealed samples (graphene and anneal sections) without
 * naming the minimiser; this is FIRE (Bitzek et al., Phys. Rev. Lett. 97,
 * 170201, 2006) with its published constants (n_min 5, f_inc 1.1, f_dec 0.5,
 * alpha_start 0.1, f_alpha 0.99).  From rest with step dt0_fs, each iteration
 * is one velocity-Verlet step with the atoms' masses; then, unless the
 * largest force on a mobile atom is below fmax (eV/Angstrom), with P = F.v:
 * v <- (1 - alpha) v + alpha |v| F/|F|; if P > 0, after more than n_min
 * such steps in a row dt <- min(f_inc dt, dtmax_fs) and alpha <- f_alpha
 * alpha; if P <= 0, dt <- f_dec dt, v <- 0, alpha <- alpha_start.  Fixed
 * atoms (fixed_dev != 0) neither move nor count.  Charges are re-equilibrated
 * at every step (warm start from the extrapolation of the last solutions).
 *   x_dev        double[3n] SoA positions (device, in/out)
 *   v_dev        double[3n] device velocity workspace (zeroed on entry)
 *   E_trace_host NULL or max_steps + 1 doubles: the energy after step s
 *   steps_out    iterations taken; fmax_out the final largest force;
 *   converged    1 if it fell below fmax, 0 if max_steps ran out
 * F_dev, q_dev receive the final forces and charges.  E_INVAL for fmax <= 0,
 * dt0 <= 0 or dtmax < dt0; the solver codes of the evaluation otherwise.
 * Reads four reductions back after every step (waits for the stream). */
int ctbop_relax_fire(ctbop_ctx *ctx, int n, double *x_dev, double *v_dev, const int32_t *types_dev,
                     const uint8_t *fixed_dev, const double *box_host, const int *pbc_host, double total_charge,
                     double fmax, int max_steps, double dt0_fs, double dtmax_fs, void *sys_dev, size_t sys_bytes,
                     double *F_dev, double *q_dev, double *E_trace_host, int *steps_out, double *fmax_out,
                     int *converged, ctbop_info *info, void *stream);

/* Ring statistics of the carbon bond graph: the paper draws its growth and
 * anneal structures as C rings by size (3-8 members), C chains, and the
 * in-plane orientation of every 6-membered ring, a hue that repeats every 60
 * degrees and is zero when two opposite vertices point along the substrate's
 * [11-20] direction (growth-simulation and annealing sections).  Neither bonds
 * nor rings are defined there; here a bond joins two C atoms (type 1) with an
 * image of one within r_bond of the other, and a ring is a shortest-path
 * ring (Franzblau, Phys. Rev. B 44, 4925, 1991): a simple cycle of at most
 * max_size (3..8) bonds such that for every two of its atoms the shorter way
 * round is a shortest path of the whole bond graph.  A chain bond is a bond
 * on no such ring.  The orientation of a 6-ring: each of its three
 * vertex-to-opposite-vertex vectors, projected on the plane with normal
 * normal_host, makes an angle theta_k with ref_host (projected on that
 * plane); the orientation is arg(sum_k exp(6 i theta_k)) / 6 in [0, 60)
 * degrees, and the ring enters the histogram (nbins bins over [0, 60)) if its
 * own normal is within max_tilt_deg of normal_host (all rings at >= 90).
 *   x_dev, types_dev   positions (SoA) and types on the device; the lists of
 *                      sys_dev are brought up to date for them (as an
 *                      evaluation would), nothing else in it changes
 *   r_bond             in (0, S_CC]: the covalent list holds pairs up to S_CC
 *   ws_dev             device workspace of ctbop_rings_bytes() bytes
 *   counts_host[9]     rings by size (index = size; 0..2 stay 0)
 *   bonds_host[2]      C-C bonds, chain bonds
 *   hist_host          NULL or nbins counts
 *   ring_list_dev      NULL or ring_cap * 9 int32 on the device: size, then the
 *                      user indices in ring order from the smallest, towards
 *                      its smaller neighbour, -1 padded; ring_orient_dev
 *                      (NULL or ring_cap doubles) the orientation (-1: not a
 *                      6-ring).  The order of the rings in the list is not
 *                      fixed.  n_rings_host gets the number of rings found,
 *                      which may exceed ring_cap (then only ring_cap are listed).
 * E_INVAL for max_size outside 3..8, r_bond outside (0, S_CC], a periodic
 * width below max_size * r_bond (a ring could wind around the cell), a zero
 * normal or a reference along it; E_NEIGH_OVERFLOW when a C atom has more
 * than 12 C neighbours.  Waits for the stream. */
int ctbop_rings_bytes(ctbop_ctx *ctx, int n, const double *box_host, const int *pbc_host, int nbins, size_t *bytes);
int ctbop_rings(ctbop_ctx *ctx, int n, const double *x_dev, const int32_t *types_dev, const double *box_host,
                const int *pbc_host, void *sys_dev, size_t sys_bytes, double r_bond, int max_size,
                const double *normal_host, const double *ref_host, double max_tilt_deg, int nbins, void *ws_dev,
                size_t ws_bytes, int64_t *counts_host, int64_t *bonds_host, int64_t *hist_host,
                int32_t *ring_list_dev, double *ring_orient_dev, int64_t ring_cap, int64_t *n_rings_host,
                void *stream);

/* Device status word of `sys` (waits for the stream). */
int ctbop_status(ctbop_ctx *ctx, void *sys_dev, size_t sys_bytes, void *stream, int *code);

/* Per-kernel timing with HIP events recorded on the caller's stream around
 * each launch (for measurement; off by default).  Waits for `stream`, folds
 * finished timings in, copies accumulated milliseconds and launch counts of
 * the first nk kernel classes to ms_out / count_out (host, may be NULL),
 * clears them if reset != 0, then turns timing on (enable != 0) or off.
 * Classes: 0 charge-solve matrix-vector product, 1 Coulomb force/energy
 * gather, 2 Coulomb matrix assembly, 3 covalent bond pass, 4 covalent force
 * gather, 5 charge-solve update, 6 charge-solve direction, 7 list build,
 * 8 sliced copy of the Coulomb rows, 9 carbon adjacency, 10 ring search,
 * 11 chain bonds. */
int ctbop_profile(ctbop_ctx *ctx, int enable, int reset, void *stream, double *ms_out, long *count_out, int nk);

/* Kernel classes that ctbop_profile times while it is on: bit k for class k
 * (default: all). Events cost the work they bracket a little, so a
 * measurement of one kernel can time that class alone. */
int ctbop_profile_classes(ctbop_ctx *ctx, unsigned mask);

/* Message of the last error on the calling thread ("" if none). */
const char *ctbop_last_error(void);

/* Copy the lists of the last build to host memory, in user atom order, for
 * tests: for every atom i its long-list (Coulomb, r < rc + skin) and
 * short-list (covalent, r < S_ij + skin) neighbours as the user index j and
 * the displacement vector x_j + n.h - x_i (at the positions of the last call).
 * counts_*: int[n]; j_*: int[n*cap]; d_*: double[3*n*cap] (row i at i*cap). */
int ctbop_debug_lists(ctbop_ctx *ctx, int n, void *sys_dev, size_t sys_bytes, int long_cap,
                      int short_cap, int *counts_long, int *j_long, double *d_long,
                      int *counts_short, int *j_short, double *d_short, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of independent evaluation requests            */
/* ------------------------------------------------------------------------ */
/* A server runs a scheduler thread on one stream over a caller-owned device
 * arena.  Every admitted request becomes a segment (its own region of the
 * arena with its inputs, outputs, lists and charges); each tick launches the
 * set-up kernels for new segments and a few charge-solve iterations plus the
 * gated force kernels for all active segments, each kernel once over all of
 * them.  Requests are admitted in arrival order at tick boundaries while
 * slots and arena bytes allow (HBM-budget admission); a request that does
 * not fit waits.  A request with system_id >= 0 leaves its region (lists and
 * charges) on the device after it finishes; the next request with that id
 * and the same geometry reuses it (lists rebuilt only if atoms moved more
 * than skin/2, charges warm-started); retained regions are evicted least
 * recently used first when space runs out.  Each result is bitwise the one
 * the request gets when it runs alone. */
typedef struct ctbop_server ctbop_server;

typedef struct {
    int            n;             /* atoms                                              */
    const double  *pos_host;      /* 3n doubles, SoA; copied at submit                 */
    const int32_t *types_host;    /* n; copied at submit                                */
    double         box[9];        /* as for compute                                     */
    int            pbc[3];
    double         total_charge;
    long           system_id;     /* >= 0: keep lists and charges for the next request */
    double        *E_host;        /* outputs (host, may be NULL): must stay valid until */
    double        *F_host;        /* the result is polled; F is 3n SoA, q is n          */
    double        *q_host;
    const double  *q0_host;       /* NULL, or n starting charges for the charge solve   */
                                  /* (copied at submit; projected onto total_charge)    */
} ctbop_request;

typedef struct {
    long   ticket;
    int    status;                /* CTBOP_* code of this request                       */
    int    cg_iters;
    int    n_atoms;
    double t_submit, t_admit, t_done;   /* steady-clock seconds                         */
} ctbop_result;

/* Bytes of the server's own tables at the head of the arena. */
size_t ctbop_server_table_bytes(int max_slots, int max_tiles);
/* Arena bytes one request of n atoms in this cell occupies while it runs. */
int ctbop_server_request_bytes(ctbop_ctx *ctx, int n, const double *box_host, const int *pbc_host, size_t *bytes);
/* Start a server: arena_dev/arena_bytes caller-owned device memory, at most
 * max_slots requests in flight, cg_per_tick solver iterations per tick (0: 8;
 * a tick that starts with no request waiting for admission iterates until its
 * systems converge, checking between chunks, and ends early once a request
 * arrives and cg_per_tick iterations have run),
 * all work on `stream` (its device is the current device). */
int ctbop_server_create(ctbop_ctx *ctx, void *arena_dev, size_t arena_bytes, int max_slots, int cg_per_tick,
                        void *stream, ctbop_server **srv);
/* Queue a request (inputs copied); E_BUSY if the queue is full, E_NOMEM if it
 * can never fit the arena. */
int ctbop_server_submit(ctbop_server *srv, const ctbop_request *req, long *ticket);
/* Take up to max finished results (waiting up to wait_s seconds for one). */
int ctbop_server_poll(ctbop_server *srv, ctbop_result *out, int max, double wait_s, int *n_done);
/* ticks, admitted, completed, pending, active, retained, arena bytes in use,
 * peak bytes, busy seconds (first nout of these). */
int ctbop_server_stats(ctbop_server *srv, double *out, int nout);
/* Stop the scheduler (pending requests are dropped) and release host state. */
int ctbop_server_destroy(ctbop_server *srv);

/* ------------------------------------------------------------------------ */
/* Removal energies (the paper's Si-desorption test)                          */
/* ------------------------------------------------------------------------ */
/* The stability of an atom is the change of the total energy when that atom
 * is removed (growth-simulation section: Si atoms whose removal costs less
 * than 6.5 eV are removed, the test repeated every 1 ps).  For every
 * candidate i this returns dE_i = E(X without atom i) - E(X), both energies
 * at their own equilibrated charges with the same total charge Q:
 *   pos_host      3n doubles SoA, types_host n int32 (host, read during the call)
 *   cand_host     m atom indices (0 <= i < n; repeats allowed)
 *   E_host        out: E(X);  dE_host: out, m doubles;  iters_host: NULL or m ints,
 *                 the charge-solve iterations of each leave-one-out system
 *   arena_dev     caller-owned device memory of at least ctbop_removal_bytes(m) bytes
 *                 (more lets more leave-one-out systems run at once)
 * The full system is evaluated once at the head of the arena; the m systems
 * of n-1 atoms then run as a continuous batch through a server on the rest,
 * each starting its charge solve from the full system's charges (re-projected
 * onto Q), which leaves only the local relaxation to solve.  Waits for the
 * stream; E_INVAL on a bad index, E_NOMEM if the arena is too small. */
int ctbop_removal_bytes(ctbop_ctx *ctx, int n, const double *box_host, const int *pbc_host, int m, size_t *bytes);
int ctbop_removal_energies(ctbop_ctx *ctx, int n, const double *pos_host, const int32_t *types_host,
                           const double *box_host, const int *pbc_host, double total_charge, const int *cand_host,
                           int m, void *arena_dev, size_t arena_bytes, double *E_host, double *dE_host,
                           int *iters_host, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CTBOP_H */
