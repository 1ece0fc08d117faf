/*
 * nbhip.h -- C ABI of the MI355X (gfx950) short-range nonbonded library.
 *
 * The library evaluates, for one or more periodic systems packed back to back,
 * the short-range nonbonded interaction of the ACEMD paper (section 3): every
 * atom pair closer than the cutoff R, not excluded as a bonded pair, interacts
 * through a Lennard-Jones 12-6 term and the real-space part of the Ewald (PME)
 * electrostatics, under minimum-image periodic boundaries:
 *
 *   u_ij = 4 eps_ij [(sigma_ij/r)^12 - (sigma_ij/r)^6] + k_e q_i q_j erfc(beta r)/r,
 *   sigma_ij = (sigma_ti + sigma_tj)/2,  eps_ij = sqrt(eps_ti eps_tj),
 *
 * with the cutoff test r < R strict, and optionally a switch of the Lennard-Jones term
 * and scaled 1-4 pairs (nb_params.lj_switch_on, nb_system.pair14_*).  The kernel variant
 * NB_KERNEL_ATOM supports neither option.  Atoms are first
 * binned into a cell list (section 3: one thread per atom computes its cell;
 * cells a fraction of R wide), then a pair kernel visits the neighbouring cells.
 *
 * Conventions for every entry point:
 *   - Pointers marked [device] are HIP device pointers; [host] are host pointers.
 *   - The caller owns every buffer.  The library allocates no device memory for
 *     its kernels: all of their scratch lives in the caller's workspace (size from
 *     nb_workspace_bytes or nb_pme_workspace_bytes).  The one device state kept
 *     between calls is the FFT library's plans of the reciprocal part (their
 *     read-only tables, made by nb_pme_workspace_bytes or nb_pme_reciprocal on first
 *     use of a grid shape and batch size on a device, at most 32 per process, kept
 *     until the process ends).
 *   - Every call only enqueues work on `stream` and returns; the only call that
 *     synchronises is nb_read_status.
 *   - Problems visible on the host are reported by the return code before any
 *     work is enqueued; the message is available from nb_last_error().
 *     Problems only visible on the device set bits in a status word inside the
 *     workspace (NB_STATUS_*), read with nb_read_status.
 *   - No C++ exception, abort or exit crosses this interface.
 *   - Units: Angstrom, elementary charge, kJ/mol.
 */
#ifndef NBHIP_H
#define NBHIP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NB_OK = 0,
  NB_ERR_ARG = 1,        /* null pointer, negative or inconsistent size, bad option */
  NB_ERR_BOX = 2,        /* a box length <= 0 or not finite, or R >= min(L)/2 */
  NB_ERR_WORKSPACE = 3,  /* workspace NULL, misaligned or smaller than nb_workspace_bytes */
  NB_ERR_HIP = 4,        /* a HIP runtime call failed; see nb_last_error */
  NB_ERR_CAPACITY = 5,   /* a size exceeds what the 32-bit indexing of the library supports */
  NB_ERR_HOST = 6        /* a host-side failure (out of host memory, or an unexpected internal error):
                            nothing was enqueued; see nb_last_error */
} nb_status;

/* Bits of the device status word (nb_read_status).  They accumulate from
 * nb_build_cells onwards; nb_build_cells clears them. */
#define NB_STATUS_NONFINITE_POS 0x1u  /* a position was NaN or infinite (atom binned to cell 0) */
#define NB_STATUS_BAD_TYPE 0x2u       /* a type index outside [0, n_types) (treated as type 0) */
#define NB_STATUS_BAD_EXCLUSION 0x4u  /* an exclusion row not monotone or an index outside the system */
#define NB_STATUS_FAR_EXCLUSION 0x8u  /* informational: some exclusion is more than 64 atoms apart in index */
#define NB_STATUS_NOT_BUILT 0x10u     /* the workspace was not built by nb_build_cells for this system size,
                                         kernel variant, cluster size and split: the pair kernels wrote
                                         nothing */
#define NB_STATUS_FAR_PAIR14 0x20u    /* a 1-4 pair more than 64 atoms apart in index: left unscaled */
#define NB_STATUS_BAD_TOPOLOGY 0x40u  /* MD calls: a water or a bonded term names atoms outside the batch or
                                         in two systems (the term is skipped; such a water's atoms move
                                         as free atoms) */

typedef enum {
  NB_FP64 = 0,  /* double-precision pair arithmetic from double positions */
  NB_MIXED = 1  /* single-precision pair arithmetic, double accumulation and reductions */
} nb_precision;

/*
 * A batch of B >= 1 independent systems packed back to back: system b owns atoms
 * [atom_offset[b], atom_offset[b+1]) of every per-atom array.  A single box is the
 * batch B = 1.
 */
typedef struct {
  int32_t n_systems;          /* B >= 1 */
  const int64_t *atom_offset; /* [host] B+1 entries, atom_offset[0] = 0, non-decreasing; N = atom_offset[B] */
  const double *box;          /* [host] 3*B orthorhombic box lengths (Lx, Ly, Lz) per system */
  const void *pos;            /* [device] N*3 coordinates x,y,z per atom; float or double per pos_is_f64.
                                 Any real value is accepted: coordinates are wrapped into the box. */
  int32_t pos_is_f64;         /* 0: pos and charge are float; 1: double */
  const void *charge;         /* [device] N charges (e), same type as pos */
  const int32_t *type;        /* [device] N Lennard-Jones type indices in [0, n_types) */
  const double *lj_sigma;     /* [device] n_types sigma_t (A); shared by the whole batch */
  const double *lj_eps;       /* [device] n_types eps_t (kJ/mol), >= 0 */
  int32_t n_types;            /* 1 <= n_types <= NB_MAX_TYPES */
  const int32_t *excl_offset; /* [device] N+1 CSR row offsets into excl_index (global over the batch) */
  const int32_t *excl_index;  /* [device] excluded partners of each atom, as indices local to its system.
                                 A pair listed in either atom's row is excluded both ways (section 3
                                 stores bonded exclusions as per-atom bitmaps over index distance
                                 |i-j| <= 64; larger distances take a slower path). */
  const int32_t *pair14_offset; /* [device] N+1 CSR row offsets of the scaled 1-4 pairs, or NULL for none */
  const int32_t *pair14_index;  /* [device] 1-4 partners of each atom, local indices.  A pair listed in
                                 either row (and not excluded) has its Lennard-Jones term scaled by
                                 nb_params.scale14_lj and its real-space Coulomb term by scale14_coul
                                 (section 3: CHARMM/AMBER 1-4 pairs, stored in bitmaps beside the
                                 exclusions).  Only |i-j| <= 64 is supported, as in the paper's
                                 bitmaps: a farther 1-4 pair sets NB_STATUS_FAR_PAIR14 and
                                 interacts unscaled. */
} nb_system;

#define NB_MAX_TYPES 64

/* Kernel variants for nb_params.kernel. */
#define NB_KERNEL_AUTO 0    /* library default: NB_KERNEL_CLUSTER_HALF (both precisions) */
#define NB_KERNEL_ATOM 1    /* one lane per i atom, full neighbour shell, j read through the cache */
#define NB_KERNEL_CLUSTER 2 /* 4- or 8-atom clusters x box-filtered j atoms staged in LDS, 64 pairs per step */
#define NB_KERNEL_CLUSTER_HALF 3 /* as NB_KERNEL_CLUSTER, each pair once (half of the column stencil),
                                    the other atom's share added by atomics into per-atom accumulators:
                                    about half the pair work.  The accumulators are 64-bit fixed point
                                    (2^-32 units; the FP64 path adds a second limb of 2^-64 units), so
                                    results are bitwise reproducible.  Forces and energies agree with the
                                    other kernels to rounding.  The adjoint and the force VJP use
                                    NB_KERNEL_CLUSTER's form. */

#define NB_SCHED_AUTO 0
#define NB_SCHED_STATIC 1  /* one work item per wave, a grid covering every item */
#define NB_SCHED_DYNAMIC 2 /* persistent waves taking items from per-XCD atomic counters */

typedef struct {
  double cutoff;      /* R (A): 0 < R < min(L)/2 for every system */
  double ewald_beta;  /* beta (1/A) >= 0; beta = 0 gives the bare truncated Coulomb term */
  double coulomb_k;   /* k_e (kJ mol^-1 A e^-2), 1389.35457644382 for CODATA 2018 */
  int32_t precision;  /* nb_precision */
  int32_t cell_div_xy;/* cells per cutoff along x and y, 1..3 (0 = 2, the paper's R/2 bins) */
  int32_t cell_div_z; /* cells per cutoff along z, 1..16 (0 = the kernel's default) */
  int32_t kernel;     /* NB_KERNEL_* */
  int32_t split;      /* cluster kernel: work items per cluster, each taking an equal share of
                         its candidate j atoms, 1..8 (0 = 1) */
  int32_t cluster_size; /* cluster kernel: atoms per i-cluster, 4 or 8 (0 = 8; 4 for the FP64 full shell) */
  int32_t schedule;   /* cluster kernel: NB_SCHED_* (0 = static) */
  int32_t wg_per_cu;  /* dynamic schedule: resident one-wave workgroups per compute unit, 1..32 (0 = 16) */
  double lj_switch_on;/* r_on (A), 0 <= r_on < R; 0 = no switch.  Otherwise the Lennard-Jones term is
                         multiplied by S = (1-x)^2 (1+2x), x = (r^2 - r_on^2)/(R^2 - r_on^2) in [0, 1]
                         (the CHARMM energy switch; section 5's benchmark switches at 7.5 A for
                         R = 9 A), and the force is -d(S u_LJ)/dr; the Coulomb term is not switched */
  double scale14_lj;  /* factor of the Lennard-Jones term of 1-4 pairs (AMBER: 0.5) */
  double scale14_coul;/* factor of the real-space Coulomb term of 1-4 pairs (AMBER: 1/1.2);
                         nb_ewald_corrections adds -(1 - scale14_coul) k_e q_i q_j erf(beta r)/r
                         for them, so that with the reciprocal part the whole Coulomb interaction
                         of a 1-4 pair is scale14_coul k_e q_i q_j / r */
  int32_t table;      /* mixed path, forces and energies: 0 = direct evaluation; 1 = the paper's
                         tabulated variant (section 3, texture tables): r^-12, r^-6, erfc(beta r)/r
                         and the Coulomb force factor linearly interpolated from tables uniform in r
                         over [0, R], built by nb_build_cells; 2 = the same with cubic Hermite
                         interpolation.  Not combined with the switch or 1-4 pairs; the adjoint
                         always evaluates directly; the FP64 path ignores it */
  int32_t table_size; /* intervals of the tables, 16..65536 (0 = 4096 linear, the paper's n;
                         1024 cubic) */
} nb_params;

/* Bytes of device workspace needed for this batch and these parameters.
 * Host only; no HIP call.  The same (system, params) must be passed to every
 * later call that uses the workspace. */
nb_status nb_workspace_bytes(const nb_system *sys, const nb_params *params, size_t *bytes /*[host]*/);

/* Cell list (section 3): wraps each atom into its box, converts it to 32-bit
 * box-fraction fixed point, bins it into cells at least R/cell_div wide, and
 * stores the atoms sorted by (system, cell, original index) -- a deterministic
 * counting sort -- together with their charges, types and exclusion windows.
 * The workspace then holds everything the pair kernels read: positions,
 * charges, types and exclusions are captured at this call, so call it again
 * after any of them changes.  `workspace` must be 256-byte aligned. */
nb_status nb_build_cells(const nb_system *sys, const nb_params *params, void *workspace /*[device]*/,
                         size_t workspace_bytes, hipStream_t stream);

/* Forces F_i = -dE/dx_i [device, N*3 doubles, caller's atom order], and optionally
 * the energy E_b [device, B doubles] and virial W_b = sum_{i<j} d_ij (x) F_ij
 * [device, 9*B doubles, row-major] of every system.  Requires nb_build_cells on
 * this workspace.  force must not be NULL; energy and virial may be NULL. */
nb_status nb_nonbonded_forces(const nb_system *sys, const nb_params *params, void *workspace,
                              size_t workspace_bytes, double *force, double *energy, double *virial,
                              hipStream_t stream);

/* Energy of every system [device, B doubles] and optionally the per-atom split
 * E_i = (1/2) sum_j u_ij [device, N doubles, caller's order; may be NULL]. */
nb_status nb_nonbonded_energy(const nb_system *sys, const nb_params *params, void *workspace,
                              size_t workspace_bytes, double *energy, double *atom_energy,
                              hipStream_t stream);

/* Adjoint of E = sum_b g_b E_b with g = grad_energy [device, B doubles]:
 *   grad_pos[i]    = g_b dE_b/dx_i = -g_b F_i            [device, N*3 doubles or NULL]
 *   grad_charge[i] = g_b dE_b/dq_i = g_b sum_j k_e q_j erfc(beta r)/r   [device, N or NULL]
 *   grad_sigma[t]  = sum_b g_b dE_b/dsigma_t              [device, n_types or NULL]
 *   grad_eps[t]    = sum_b g_b dE_b/deps_t                [device, n_types or NULL]
 * dE/deps_t is reported as 0 for a type with eps_t = 0, where the derivative of
 * sqrt(eps_t eps_j) is unbounded.  Outputs are overwritten, not accumulated. */
nb_status nb_nonbonded_backward(const nb_system *sys, const nb_params *params, void *workspace,
                                size_t workspace_bytes, const double *grad_energy, double *grad_pos,
                                double *grad_charge, double *grad_sigma, double *grad_eps,
                                hipStream_t stream);

/* Vector-Jacobian product of the forces (the double backward of force matching): with
 * v [device, N*3 doubles, caller's order] and L = sum_b sum_{i in b} v_i . F_i,
 *   grad_charge[i] = dL/dq_i       [device, N doubles or NULL]
 *   grad_sigma[t]  = dL/dsigma_t   [device, n_types or NULL]
 *   grad_eps[t]    = dL/deps_t     [device, n_types or NULL; 0 where eps_t = 0]
 * for the same interaction as nb_nonbonded_forces (switch and 1-4 scaling included;
 * direct evaluation whatever nb_params.table says).  Per pair this is the parameter
 * derivative of the force factor times (v_i - v_j) . d_ij, summed in double precision.
 * Requires nb_build_cells on this workspace and a cluster kernel (NB_KERNEL_ATOM is
 * refused).  Outputs are overwritten. */
nb_status nb_nonbonded_force_vjp(const nb_system *sys, const nb_params *params, void *workspace,
                                 size_t workspace_bytes, const double *v, double *grad_charge,
                                 double *grad_sigma, double *grad_eps, hipStream_t stream);

/* Ewald corrections that complete the real-space term of the forces above (section 3:
 * the electrostatics are PME, whose reciprocal part counts every pair, excluded ones
 * included, and every charge with itself):
 *   excluded pairs: -k_e q_i q_j erf(beta r)/r for every pair {i, j} named in either
 *     atom's exclusion row (each pair once, at any distance, minimum image; at r = 0 the
 *     limit -k_e q_i q_j 2 beta/sqrt(pi));
 *   self term: -k_e beta/sqrt(pi) sum_i q_i^2 per system.
 * Writes (does not add to) force [device, N*3 doubles, caller's order: the forces of
 * the excluded-pair term], energy [device, B doubles: both terms, or NULL] and virial
 * [device, 9*B doubles: the excluded-pair term, row-major, or NULL]; force may be NULL only
 * when the batch has no atoms (energies and virials are then zero).  FP64 arithmetic on
 * the caller's positions and charges (either precision).  Requires nb_build_cells on
 * this workspace with the same exclusion lists (it uses the exclusion windows of the
 * build).  A far pair (|i - j| > 64) named in one row only is added to the other atom
 * by an FP64 atomic, so such atoms' forces may vary in the last bits from run to run. */
nb_status nb_ewald_corrections(const nb_system *sys, const nb_params *params, void *workspace,
                               size_t workspace_bytes, double *force, double *energy, double *virial,
                               hipStream_t stream);

/* Reciprocal part of the Ewald sum by smooth particle-mesh Ewald (section 3: the
 * long-range electrostatics are PME with fourth-order interpolation; the method of
 * Essmann et al. 1995).  On a K1 x K2 x K3 grid (grid[3], host, each in [4, 1024], the
 * same for every system of the batch) with cubic B-splines (order 4):
 *   E_b = k_e/(2 pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2 B(m) |FFT(Q)(m)|^2
 * where Q is the charge grid of system b, m = (n1/L1, n2/L2, n3/L3) and B the spline
 * factor.  The m = 0 term is omitted (no neutralising-background term for a charged
 * system).  Writes (does not add to) force [device, N*3 doubles, caller's order],
 * energy [device, B doubles, or NULL] and virial [device, 9*B doubles,
 * W_ab = -dE/d(strain_ab), row-major, or NULL].  FP64 arithmetic (either input
 * precision); ewald_beta > 0 and coulomb_k come from params, which is validated as for
 * the other calls.  `workspace` is its own buffer (not the nonbonded workspace) of
 * nb_pme_workspace_bytes bytes, 256-byte aligned, owned by the caller; it needs no
 * build.  It holds the grids and the work area of the FFTs, so calls with different
 * workspaces may run concurrently on different streams.  The LDS additions of the
 * charge spreading are FP64 atomics, so results may vary in the last bits from run to
 * run.  The FFTs use hipFFT plans (each transforming every system of the batch in one
 * call) made on the first use of a grid shape and batch size on a device, by
 * nb_pme_workspace_bytes (which therefore needs a current HIP device) or
 * nb_pme_reciprocal, and kept until the process ends (only their read-only tables:
 * they allocate no work buffers of their own); at most 32 such plans per process.
 * Returns NB_ERR_HIP if the FFT library refuses a plan or a transform or the 32 are
 * used up. */
nb_status nb_pme_workspace_bytes(const nb_system *sys, const int32_t grid[3] /*[host]*/, size_t *bytes /*[host]*/);
nb_status nb_pme_reciprocal(const nb_system *sys, const nb_params *params, const int32_t grid[3] /*[host]*/,
                            void *workspace, size_t workspace_bytes, double *force, double *energy,
                            double *virial, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): nb_build_cells followed by
 * nb_nonbonded_forces, with the same arguments and results, but with the workspace
 * taken from a scratch array of NB_NOALLOC_SCRATCH_BYTES (16 MiB) that the library holds
 * in device memory on every GPU it runs on, from the loading of the library's code until
 * the process ends.  The caller still passes the outputs.  No hipMalloc, hipFree or
 * other allocating call is made.  Batches whose workspace (nb_workspace_bytes) exceeds
 * NB_NOALLOC_SCRATCH_BYTES are refused with NB_ERR_CAPACITY before any work is enqueued
 * (about 72,000 atoms at the densities of the configurations here).  The first call on a
 * device looks up that device's copy of the array (hipGetSymbolAddress).  Every call on
 * a GPU uses the same array, which keeps the last call's contents (the build rewrites
 * everything the pair kernel reads): calls that overlap on one GPU, on different streams
 * or from different threads, race and must be ordered by the caller.  The device status
 * word of the build cannot be read back (no workspace pointer is handed out). */
#define NB_NOALLOC_SCRATCH_BYTES (16u << 20)
nb_status nb_nonbonded_forces_noalloc(const nb_system *sys, const nb_params *params, double *force,
                                      double *energy, double *virial, hipStream_t stream);

/* ---- Molecular dynamics around the force evaluation ----
 *
 * Section 3 describes production runs in the NVT ensemble: bonded and nonbonded forces,
 * velocity-Verlet integration under a Langevin thermostat, PME electrostatics and
 * constrained bonds to hydrogen, with the speed in ns/day at a 4 fs step reported in
 * Table 5.  The calls below run that loop for every system of a batch on the GPU.
 *
 * Forces: the short-range term of nb_nonbonded_forces (with every nb_params option and
 * kernel variant), with a PME grid also the Ewald corrections (nb_ewald_corrections) and
 * the reciprocal part (nb_pme_reciprocal), plus harmonic bonds E = k (r - r0)^2 and angles
 * E = k (theta - theta0)^2 (minimum image; their forces are added by FP64 atomics, so they
 * may vary in the last bits from run to run).
 *
 * Step (the paper names no splitting; this is Bussi and Parrinello's Langevin velocity
 * Verlet, Phys. Rev. E 75, 056707 (2007)), with c = exp(-gamma dt/2):
 *   v <- c v + sqrt((1 - c^2) kT/m) xi;  v <- v + (dt/2) F/m;  x <- x + dt v, constrained,
 *   and v <- (constrained displacement)/dt;  F <- F(x);  v <- v + (dt/2) F/m;
 *   v <- c v + sqrt((1 - c^2) kT/m) xi';  v constrained.
 * Constraints: rigid 3-site waters (the exact solutions of the SHAKE position and RATTLE
 * velocity equations of each molecule).  Noise: Philox4x32-10 with counter (atom index in
 * the batch, step mod 2^32, step div 2^32, 0 for xi or 1 for xi') and key (seed mod 2^32,
 * seed div 2^32); uniforms (u + 1/2)/2^32; Box-Muller normals x, y from words 0, 1 and z
 * from words 2, 3.  gamma = 0 draws no noise (velocity Verlet with constraints).
 * Units: Angstrom, ps, g/mol, kJ/mol, K (F/m = 100 A/ps^2 per (kJ/mol/A)/(g/mol)).
 * The state is double precision: sys->pos_is_f64 must be 1 (charges double too).
 */
typedef struct {
  const double *mass;           /* [device] N masses (g/mol), > 0 */
  int64_t n_waters;             /* rigid 3-site waters */
  const int32_t *water_o;       /* [device] n_waters indices (in the batch) of their O atoms; the H atoms are
                                   O + 1 and O + 2, in the same system; no atom in two waters */
  double water_r_oh, water_r_hh;/* the held O-H and H-H distances (A); r_hh < 2 r_oh */
  int64_t n_bonds;
  const int32_t *bond_atoms;    /* [device] 2 n_bonds atom indices (in the batch) */
  const double *bond_k;         /* [device] n_bonds, kJ/mol/A^2 */
  const double *bond_r0;        /* [device] n_bonds, A */
  int64_t n_angles;
  const int32_t *angle_atoms;   /* [device] 3 n_angles atom indices i, j, k: the angle at j */
  const double *angle_k;        /* [device] n_angles, kJ/mol/rad^2 */
  const double *angle_theta0;   /* [device] n_angles, rad */
} nb_md_topology;

typedef struct {
  double dt;            /* time step (ps), > 0 */
  double temperature;   /* K, >= 0 */
  double gamma;         /* Langevin friction (1/ps), >= 0; 0: no thermostat */
  uint64_t seed;        /* key of the thermostat noise */
  int32_t pme_grid[3];  /* [host] reciprocal-part grid (as nb_pme_reciprocal; needs ewald_beta > 0);
                           {0, 0, 0}: no reciprocal part and no Ewald corrections */
  int32_t reserved;     /* 0 */
  hipStream_t aux_stream; /* NULL, or a second stream (default priority) on which the reciprocal part
                           runs concurrently with the short-range term: every call then orders it
                           against `stream` with HIP events of its own, so the caller only needs
                           both streams to be usable on the current device */
} nb_md_params;

/* Workspace of the MD calls (it holds a nonbonded workspace, a reciprocal-part workspace
 * and the force parts); with a PME grid it needs a current HIP device (FFT plans). */
nb_status nb_md_workspace_bytes(const nb_system *sys, const nb_params *params, const nb_md_params *md,
                                size_t *bytes /*[host]*/);

/* Total force at sys->pos [device, N*3 doubles, written] and, if energy is not NULL, the
 * energies per system [device, 4*B doubles: short-range, Ewald corrections, reciprocal,
 * bonded].  The MD workspace (256-byte aligned, nb_md_workspace_bytes) is the caller's. */
nb_status nb_md_forces(const nb_system *sys, const nb_params *params, const nb_md_topology *topo /*[host]*/,
                       const nb_md_params *md /*[host]*/, void *workspace, size_t workspace_bytes, double *force,
                       double *energy, hipStream_t stream);

/* n_steps >= 0 steps of the integrator, numbered first_step .. first_step + n_steps - 1
 * (the noise counters), from the positions pos (== sys->pos) and velocities vel [device,
 * N*3 doubles each, updated in place].  The forces at the starting positions are computed
 * first, so consecutive calls continue one trajectory.  If energy is not NULL, the final
 * state's energies per system [device, 5*B doubles: short-range, Ewald corrections,
 * reciprocal, bonded, kinetic].  Velocities need not satisfy the constraints on entry; on
 * return they do. */
nb_status nb_md_run(const nb_system *sys, const nb_params *params, const nb_md_topology *topo /*[host]*/,
                    const nb_md_params *md /*[host]*/, void *workspace, size_t workspace_bytes, double *pos,
                    double *vel, int64_t first_step, int64_t n_steps, double *energy, hipStream_t stream);

/* Synchronises `stream` and returns the NB_STATUS_* bits accumulated in the workspace. */
nb_status nb_read_status(const void *workspace, hipStream_t stream, uint32_t *flags /*[host]*/);

/* Message for the last non-OK return on the calling thread ("" if none). */
const char *nb_last_error(void);

/* Pair-kernel timing, for benchmarks.  nb_pair_timer_start creates `capacity` pairs of
 * HIP events (host call; HIP events only, no device memory) and from then on every
 * nb_nonbonded_forces / _energy / _backward call records one pair on its stream
 * immediately before and after its pair kernel (the launches that follow the first
 * `capacity` are not recorded).  nb_pair_timer_stop waits for the recorded events,
 * returns the summed kernel time in milliseconds and the number of recorded
 * launches, and destroys the events.  Process-wide state: not for concurrent use
 * from several threads.  capacity in [1, 65536]. */
nb_status nb_pair_timer_start(int32_t capacity);
nb_status nb_pair_timer_stop(double *total_ms /*[host]*/, int64_t *launches /*[host]*/);

/* Internal arrays of a built workspace, as byte offsets from its start, for tests
 * and debugging.  Host only.  See the library source for the record formats. */
typedef struct {
  int64_t n_atoms;
  int64_t n_cells;          /* all systems */
  int32_t dims[3];          /* grid of system 0 */
  int64_t off_cell_start;   /* int32 [n_cells + 1] */
  int64_t off_sorted_fixed; /* uint32 x4 [n_atoms]: fixed-point x, y, z and original index */
  int64_t off_sorted_pos64; /* double x4 [n_atoms]: wrapped x, y, z, charge (FP64 data) */
  int64_t off_excl_mask;    /* uint32 x4 [n_atoms], original order: exclusion window bits */
  int64_t off_status;       /* uint32 status word */
  int64_t n_columns;        /* (x, y) columns of all systems */
  int64_t n_clusters_max;   /* upper bound on the number of clusters */
  int64_t off_col_clu_start;/* int32 [n_columns + 1]: first cluster of each column (cluster kernel) */
} nb_layout;

nb_status nb_workspace_layout(const nb_system *sys, const nb_params *params, nb_layout *layout /*[host]*/);

#ifdef __cplusplus
}
#endif

#endif /* NBHIP_H */
