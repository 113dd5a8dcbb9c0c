/*
 * esbgk.h -- C ABI of the MI355X (gfx950) ES-BGK lattice Boltzmann library.
 *
 * The library advances the two-population lattice Boltzmann scheme with a
 * polyatomic ellipsoidal-statistical (ES-BGK) Gaussian target of Hu, Zhang,
 * Du, Jin and Kong, "A lattice Boltzmann scheme with arbitrary Prandtl number
 * and specific heat ratio based on the polyatomic ES-BGK model"
 * (arXiv:1611.02409):
 *
 *   - populations f_i (mass, the paper's g_i) and g_i (internal energy, the
 *     paper's h_i), Section III and the discrete definitions of Section V;
 *   - per cell, the moments rho, rho u, the stress tensor sigma (Eq. Lambda),
 *     T_tr, T_int, T_eq and T_rel (Sections II and V);
 *   - the target G_i = w_i rho sum_{n<=4} a^(n).H^(n)(xi_i)/n! whose Hermite
 *     coefficients come from the general-term formula (Eq. fESCoe, Eq.
 *     GExpansion) with Lambda of Section II;
 *   - collide and stream (Eqs. DiscreteReductionG and DiscreteReductionH),
 *     f_i <- f_i - omega (f_i - G_i), g_i <- g_i - omega (g_i - N_f/2 T_rel G_i),
 *     on a periodic grid.
 *
 * Conventions shared by every entry point
 *   Units: the paper's dimensionless thermal units (Section V): rho0 = T0 = 1,
 *     velocities in units of sqrt(R_g T0).  The lattice velocity of direction
 *     i is xi_i = r c_i with integer c_i; one step moves c_i cells.
 *   Lattices: (D, Q) = (2, 37) Table I; (2, 33) Table II; (3, 39) (three-
 *     dimensional, not in the paper; six shells solved from the degree-7
 *     Gauss-Hermite conditions).
 *   Parameters: tau > 1/2 is the relaxation time in steps, Pr > 0 the
 *     Prandtl number, N_f >= 0 the extra degrees of freedom, so that
 *     gamma = (N_f + D + 2)/(N_f + D) (Eq. Gamma).  The stress relaxes at
 *     1/tau and the heat flux at omega = 1/(1/2 + (tau - 1/2)/Pr); the ES
 *     parameter is nu = (1 - omega_s/omega)/(1 - kappa), which reproduces
 *     Eq. Pr exactly for the lattice transport coefficients (kinematic
 *     viscosity (T/r^2)(tau - 1/2), thermal diffusivity that over Pr, in grid
 *     units) and the paper's rate Pr/tau for large tau.  kappa defaults to
 *     0.2 (Section VI.A).
 *   Fields: host arrays of doubles, row-major with x fastest; a field has
 *     ncell = nx*ny(*nz) values; vector fields (u) hold D such planes in the
 *     order x, y(, z); the pressure tensor holds D(D+1)/2 planes in the order
 *     xx, xy, yy (2D) or xx, xy, xz, yy, yz, zz (3D).
 *   Storage: ESBGK_F32 keeps each population as an FP32 deviation from its
 *     rest-state value; ESBGK_F16_DEV and ESBGK_BF16_DEV keep it as an FP16 or
 *     BF16 deviation multiplied by a per-direction power of two near 1/w_i.
 *     Collision arithmetic is FP32 in all modes.  ESBGK_PULL or-ed into the
 *     storage argument selects the two-copy streaming scheme, and
 *     ESBGK_PLANE_PAD(n) a padding after every plane.  One direction
 *     of all cells forms a plane; the Q planes of a population form a set of
 *     at most 4 GiB (the largest domain: 2^32 / (Q * 4) cells for FP32, and
 *     for FP16/BF16 with N_f > 0, whose f_i and g_i share one 4-byte element;
 *     2^32 / (Q * 2) for FP16/BF16 with N_f = 0).
 *   Errors: every int-returning call returns ESBGK_OK (0) or a negative code
 *     below and sets a thread-local message (esbgk_last_error).  No call
 *     throws or aborts.  A failing call leaves the handle usable unless it
 *     says otherwise.
 *   Threads and streams: a handle is not thread-safe; distinct handles are
 *     independent.  Kernel launches go to the handle's HIP stream; calls
 *     documented as asynchronous return before the GPU has finished.
 */
#ifndef ESBGK_H
#define ESBGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ESBGK_OK 0
#define ESBGK_EINVAL (-1)        /* bad argument                                */
#define ESBGK_EUNSUPPORTED (-2)  /* lattice / storage / size not supported      */
#define ESBGK_ENOMEM (-3)        /* device or host allocation failed            */
#define ESBGK_EDEVICE (-4)       /* a HIP call failed                           */
#define ESBGK_ESTATE (-5)        /* call not valid in the handle's state        */
#define ESBGK_ENONFINITE (-6)    /* non-finite input or result                  */
#define ESBGK_EIO (-7)           /* checkpoint file error                       */

#define ESBGK_F32 0
#define ESBGK_F16_DEV 1
#define ESBGK_BF16_DEV 2

/* Streaming scheme, or-ed into a storage argument.  Without it the populations are one copy updated in place with the A-A
 * pattern: even steps read and write each cell's own slots (writing f_i
 * into slot opp(i)), odd steps read slot opp(i) at x - c_i and write slot i
 * at x + c_i.  With ESBGK_PULL the library keeps two copies: every step
 * reads slot i at x - c_i from the current copy and writes slot i at x of
 * the other one, so every store covers whole aligned cache lines.  Twice
 * the storage; the arithmetic and the results are bit for bit those of
 * A-A. */
#define ESBGK_PULL 0x10

/* Plane padding, or-ed into a storage argument: n (0..255) times 4 KiB of
 * unused bytes after every plane, which changes the distance between the
 * address streams of the Q (or 2Q) planes a step reads and writes at once.
 * The HBM rate of those streams depends on that distance: on MI355X a 4096^2
 * D2Q37 FP32 domain (planes exactly 64 MiB apart) moves 5.46 TB/s unpadded
 * and 5.56-5.60 TB/s with n = 4, and some distances cost a quarter of the
 * rate (a 4096 x 4064 domain unpadded: 3.9-4.1 TB/s).  Results do not
 * depend on it; checkpoints are written unpadded and load into any
 * padding. */
#define ESBGK_PLANE_PAD(n) (((n) & 0xff) << 8)

typedef struct esbgk_lattice esbgk_t;
typedef struct esbgk_batch esbgk_batch_t;

/* Message describing the last failure on the calling thread ("" if none). */
const char *esbgk_last_error(void);

/* Library version string. */
const char *esbgk_version(void);

/* Lattice constants as the library uses them (FP64): c[3*Q] integer
 * velocities (unused components 0), w[Q] weights, *r scale factor,
 * *reach the largest |c| component.  Population i of the library's storage
 * is direction i of this list.  Any output may be NULL.  Section VI
 * (Tables I, II) and the three-dimensional D3Q39 set. */
int esbgk_lattice_info(int D, int Q, int *c, double *w, double *r, int *reach);

/* Relaxation parameters the library derives from (D, N_f, Pr, tau, kappa):
 * out[0] omega (heat-flux rate), out[1] omega_s (stress rate, 1/tau),
 * out[2] nu (ES parameter of Lambda), out[3] gamma (Eq. Gamma).
 * ESBGK_EINVAL if tau <= 1/2, Pr <= 0, N_f < 0, kappa outside [0, 1) or if
 * Lambda could lose positive-definiteness for some admissible stress. */
int esbgk_params(int D, int N_f, double Pr, double tau, double kappa, double out[4]);

/* Create a periodic lattice of dims[0] x dims[1] (x dims[2]) cells.
 * Requires every dim >= the lattice reach and few enough cells that one
 * population set fits in 4 GiB (see Storage above; ESBGK_EUNSUPPORTED
 * otherwise, with the largest cell count in the message).  The library
 * allocates the population storage (2 Q planes, or Q when N_f = 0) and owns
 * it (esbgk_autotune may move it to an allocation with another plane
 * padding); work goes to the default HIP stream until esbgk_set_stream.  The handle starts
 * without a state: call esbgk_init_fields before stepping. */
int esbgk_create(int D, int Q, int N_f, double Pr, double tau, const int64_t *dims, int storage, esbgk_t **out);

/* As esbgk_create, but the populations live in caller-owned device memory
 * dev_buf of at least esbgk_storage_bytes() bytes (256-byte aligned), and
 * work goes to hip_stream (a hipStream_t, or NULL for the default stream).
 * The library never frees dev_buf; it must outlive the handle. */
int esbgk_create_ex(int D, int Q, int N_f, double Pr, double tau, const int64_t *dims, int storage,
                    void *dev_buf, size_t bytes, void *hip_stream, esbgk_t **out);

/* Bytes of population storage a lattice of this shape needs. */
int esbgk_storage_bytes(int D, int Q, int N_f, const int64_t *dims, int storage, size_t *bytes);

/* Set kappa (0 <= kappa < 1; the Section II blend of T_eq into Lambda and
 * T_rel) and re-derive nu.  Allowed at any time; applies to later steps. */
int esbgk_set_kappa(esbgk_t *h, double kappa);

/* Route later work to hip_stream (NULL: default stream).  The caller keeps
 * ownership of the stream. */
int esbgk_set_stream(esbgk_t *h, void *hip_stream);

/* Write the equilibrium state of host fields rho (> 0), u (D planes) and
 * T (> 0): f_i = G_i(rho, u, Lambda = T delta), g_i = (N_f/2) T G_i.
 * Resets the step counter to 0.  Synchronous.  ESBGK_ENONFINITE or
 * ESBGK_EINVAL for non-finite or non-positive rho or T. */
int esbgk_init_fields(esbgk_t *h, const double *rho, const double *u, const double *T);

/* Enqueue n >= 0 collide-and-stream steps (asynchronous).  ESBGK_ESTATE
 * before init.  The call only launches kernels on the handle's stream (no
 * allocation, copy or memset), so it may be captured into a HIP graph on
 * that stream; the handle's step counter, which selects the storage layout
 * for later calls, advances at capture and not at replay, so a captured
 * sequence should hold an even number of steps (the layout it ends in is
 * then the one it starts from). */
int esbgk_step(esbgk_t *h, int64_t n);

/* Diffusely reflecting walls normal to y, for the thermal Couette flow of
 * Sec. VI.A (the wall density of the kinetic boundary condition; the
 * paper's non-equilibrium extrapolation part is not applied).  bottom and
 * top are {u_x, u_y, u_z, T} of the walls at low and high y (u_z ignored in
 * 2D; host memory, read during the call).  The first and last `reach` rows
 * (the largest |c_y| of the lattice) become ghost rows outside the gas;
 * x (and z) stay periodic.  After every step the library sums, per ghost
 * column and in FP64, the mass the gas will stream into the wall, and the
 * wall re-emits it as that density times G(u_w, T_w delta) (f) and
 * (N_f/2) T_w times that (g); on a stepped state the call does this at
 * once.  The first step streams the initial state as given.  Only the gas
 * rows are physical: moments and populations of ghost rows are scratch, and
 * esbgk_totals returns ESBGK_ESTATE while walls are set.  Both NULL removes
 * the walls.  Needs ESBGK_PULL storage and ny >= 2 reach + 1 (else
 * ESBGK_EINVAL); T must be > 0.  The setting is not part of a checkpoint
 * (the wall emission in the saved ghost rows is).  Synchronous. */
int esbgk_set_walls(esbgk_t *h, const double *bottom, const double *top);

/* Open (zero-gradient) ends along x, as for the shock tube of Sec. VI.B
 * (on != 0; 0 restores periodic x).  The first and last `reach_x` columns
 * (the largest |c_x| of the lattice) become ghost columns outside the gas:
 * after every step each ghost cell takes a copy of the stored populations
 * of the nearest gas cell of its row, so the gas next to an end streams in
 * the end column's own post-collision populations; on a stepped state the
 * call does this at once, and the first step streams the initial state as
 * given.  y (and z) stay periodic.  Only the gas columns are physical;
 * esbgk_totals returns ESBGK_ESTATE while the ends are open.  Needs
 * ESBGK_PULL storage, nx >= 2 reach_x + 1 and no walls (else ESBGK_EINVAL;
 * esbgk_set_walls likewise refuses while the ends are open).  Not part of a
 * checkpoint.  Synchronous. */
int esbgk_set_open_x(esbgk_t *h, int on);

/* Plane padding of the handle's storage in bytes (set at creation, or
 * chosen by esbgk_autotune for library-owned storage). */
int esbgk_plane_pad(const esbgk_t *h, int64_t *bytes);

/* Steps taken since init (or loaded from a checkpoint). */
int esbgk_step_count(const esbgk_t *h, int64_t *n);

/* Pre-collision moments at the current step (Section V): rho, u (D planes),
 * T = T_eq, and, if P is not NULL, the central pressure tensor
 * rho sigma (D(D+1)/2 planes).  Any output may be NULL.  Synchronous. */
int esbgk_read_moments(esbgk_t *h, double *rho, double *u, double *T, double *P);

/* Domain totals in FP64: out[0] mass, out[1..D] momentum, out[D+1] total
 * energy sum(1/2 xi^2 f + g) (Section V).  Reduced on the GPU in FP64.
 * Synchronous. */
int esbgk_totals(esbgk_t *h, double *out);

/* Populations of n listed cells (flat indices, x fastest) at the current
 * step, decoded to FP64: f[k*Q + i], g[k*Q + i] (g may be NULL; ignored when
 * N_f = 0).  Synchronous.  For checks of single cells of large runs. */
int esbgk_read_cells(esbgk_t *h, int64_t n, const int64_t *cells, double *f, double *g);

/* All populations at the current step, decoded to FP64, as Q planes of
 * ncell values: f[i*ncell + k] (g likewise, may be NULL).  Synchronous. */
int esbgk_read_populations(esbgk_t *h, double *f, double *g);

/* Overwrite all populations from FP64 planes laid out as in
 * esbgk_read_populations (g ignored when N_f = 0); keeps the step counter.
 * Values are encoded in the handle's storage mode.  Synchronous. */
int esbgk_write_populations(esbgk_t *h, const double *f, const double *g);

/* Checkpoint the raw state (storage, parameters, step counter) to a file /
 * restore it into a handle created with the same lattice, dims, N_f,
 * storage mode and streaming scheme (any plane padding: the file holds the
 * unpadded layout).  Synchronous.  ESBGK_EIO on file errors, ESBGK_EINVAL on
 * a mismatching handle. */
int esbgk_save(esbgk_t *h, const char *path);
int esbgk_load(esbgk_t *h, const char *path);

/* Time n steps on the handle's stream with HIP events around each launch:
 * *total_ms is the elapsed time of the n launches, per_launch_ms (if not
 * NULL, n entries) the time of each.  Synchronous. */
int esbgk_step_timed(esbgk_t *h, int64_t n, double *total_ms, double *per_launch_ms);

/* Launch shape of the step kernels.  parity: 0 = the kernel that reads the
 * even layout, 1 = the odd-layout kernel, -1 = both.  block = work-group
 * size (a multiple of 64 in [64, 512]; 0 = 256); order = work-group order
 * over the cells (0 = default = 1; 1 = dispatch order; 2 = contiguous runs
 * of cells per XCD); policy = cache policy of the population loads and
 * stores (0 = default = 1; 1 = normal; 2 = non-temporal loads and stores;
 * 3 = non-temporal stores, normal loads); cells_per_item =
 * consecutive chunks of `block` cells one work-group sweeps (1..64; 0 = 1).
 * ESBGK_EINVAL otherwise.  Results do not depend on the launch shape. */
int esbgk_set_tile(esbgk_t *h, int parity, int block, int order, int policy, int cells_per_item);
int esbgk_get_tile(const esbgk_t *h, int parity, int *block, int *order, int *policy, int *cells_per_item);

/* Autotune the launch shape of each parity: if cache_path names a file
 * holding entries for this lattice, N_f class, storage and size class, apply
 * them; otherwise time every candidate (block 128/256/512 x both orders x
 * cache policies 1-3 x 1/4/16 chunks per work-group; each launch timed
 * alone) on the handle's own state, apply the fastest shape per parity and
 * append both to cache_path (if not NULL).  With library-owned storage
 * (esbgk_create) it then times plane paddings of 0, 16, 24 and 48 KiB, each
 * on an allocation of its own, and keeps the fastest allocation: the storage
 * moves (device addresses change, so capture graphs of esbgk_step after
 * this call) and the padding goes to the cache too.  Caller-owned storage
 * keeps its layout.  The handle's state is restored bitwise in any case.
 * budget_ms bounds the launch-shape timing (<= 0: no bound).  Needs a
 * second copy of the population storage on the device while it runs, and
 * for library-owned storage room for two more.  Synchronous. */
int esbgk_autotune(esbgk_t *h, double budget_ms, const char *cache_path);

/* Measured ceiling of the step kernels' memory pattern: 74 FP32 planes of
 * `cells` cells read and written once per launch with no arithmetic (1 <=
 * reps timed launches on the default stream, 256 <= cells <= 2.8e7).
 * *gbps counts read plus written bytes and is the best of three placements
 * (in place on each of two buffers, and a copy from one to the other), four
 * occupancies (1, 2, 3 and up to 8 work-groups of 256 per CU), two store
 * cache policies (default and non-temporal) and two plane strides
 * (unpadded, and 16 KiB of padding per plane).
 * Allocates and frees its own buffers (four sets of 37 planes).  A roofline
 * reference next to the published HBM peak, not part of the scheme. */
int esbgk_stream_ceiling(int64_t cells, int reps, double *gbps);

/* The same probe for the stream pattern of another lattice or storage mode:
 * `planes` 4-byte planes in `sets` sets (74, 78 or 66 in two sets: FP32 f
 * and g of D2Q37, D3Q39, D2Q33; 37, 39 or 33 in one set: FP16/BF16 (f, g)
 * pairs, or one population).  ESBGK_EINVAL for other patterns, for cells <
 * 256 and for sets over 4 GiB. */
int esbgk_stream_ceiling_planes(int64_t cells, int planes, int sets, int reps, double *gbps);

/* Release the handle and the memory the library owns.  NULL is a no-op. */
void esbgk_destroy(esbgk_t *h);

/* ------------------------------------------------------------------------
 * Batches: many independent periodic 2D or 3D domains of one lattice and
 * one storage mode, each with its own size and (N_f, Pr, tau, kappa),
 * advanced together by one persistent kernel launch per call.
 * ---------------------------------------------------------------------- */

typedef struct {
    int N_f;
    double Pr, tau, kappa;   /* kappa <= 0 selects the default 0.2 */
    int64_t dims[3];         /* dims[2] ignored in 2D */
} esbgk_domain_desc;

/* Create a batch of n domains of lattice (D, Q).  The library allocates all
 * storage in one device buffer and its own HIP stream.  Same validation per
 * domain as esbgk_create.  storage is ESBGK_F32, ESBGK_F16_DEV or
 * ESBGK_BF16_DEV, or-ed with ESBGK_PULL for two-copy pull streaming (both
 * copies of a domain side by side; twice the memory, bitwise the same
 * results as A-A in place). */
int esbgk_batch_create(int D, int Q, int n, const esbgk_domain_desc *desc, int storage, esbgk_batch_t **out);

/* Route the batch's work to hip_stream (non-NULL; graphs are captured on it). */
int esbgk_batch_set_stream(esbgk_batch_t *b, void *hip_stream);

/* Equilibrium start of domain k (fields as for esbgk_init_fields); only
 * before the batch's first step (ESBGK_ESTATE after). */
int esbgk_batch_init_fields(esbgk_batch_t *b, int k, const double *rho, const double *u, const double *T);

/* Advance every domain by n steps (asynchronous).  mode 0: one persistent
 * kernel launch that loops over all n steps (consecutive steps are ordered
 * by grid-wide barriers; launched through a captured HIP graph);
 * mode 1: one launch per step covering every domain; mode 2: one launch per
 * domain per step (the per-domain loop baseline).  All modes give bitwise
 * identical results.  A mode-0 launch fills the GPU with work-groups that
 * must all be resident at once: the library orders it after the previous
 * mode-0 launch of any batch in the process on the same device, and work
 * on other streams only delays it, but a kernel elsewhere that holds
 * compute units for longer than about a second makes its barrier wait
 * time out (see esbgk_batch_status). */
int esbgk_batch_step(esbgk_batch_t *b, int64_t n, int mode);

/* Launch shape of the batched kernels: block = cells per tile and work-group
 * size (multiple of 64 in [64, 512], 0 = 256); policy as for esbgk_set_tile;
 * window = steps a group of domains advances before the persistent kernel
 * moves to the next group (0 or 1 = step by step); group_bytes = storage
 * budget of one domain group (<= 0 keeps the current one; default: all
 * domains form one group).
 * Results do not depend on any of these. */
int esbgk_batch_set_tile(esbgk_batch_t *b, int block, int policy, int window, double group_bytes);

/* The batch's autotuner: time the persistent mode (a few steps) for each
 * work-group size in {128, 256, 512} and cache policy 0, 2 and 3, on the
 * batch's own state, put that state (and the step count) back bitwise,
 * and keep the fastest shape; window and domain grouping stay as set.
 * With cache_path the choice is looked up first (keyed by lattice,
 * storage, domain count and log2 of the cell count) and appended when
 * measured.  budget_ms bounds the timing (<= 0: no bound).  Needs a second
 * copy of the batch storage on the device while it runs.  Synchronous. */
int esbgk_batch_autotune(esbgk_batch_t *b, double budget_ms, const char *cache_path);

/* Current work-group size and cache policy (0, 2 or 3) of the batched kernels. */
int esbgk_batch_get_tile(const esbgk_batch_t *b, int *block, int *policy);

/* esbgk_batch_step bracketed by HIP events on the batch's stream; *ms is
 * the elapsed time.  Synchronous. */
int esbgk_batch_step_timed(esbgk_batch_t *b, int64_t n, int mode, double *ms);

/* Wait for the batch's queued work. */
int esbgk_batch_sync(esbgk_batch_t *b);

/* Per-domain read-outs, as the single-domain calls (synchronous). */
int esbgk_batch_read_moments(esbgk_batch_t *b, int k, double *rho, double *u, double *T, double *P);
int esbgk_batch_totals(esbgk_batch_t *b, int k, double *out);
int esbgk_batch_read_populations(esbgk_batch_t *b, int k, double *f, double *g);

/* Total cells over all domains, and population bytes one step moves
 * (read + write) over all domains. */
int esbgk_batch_info(const esbgk_batch_t *b, int64_t *cells, double *bytes_per_step);

/* Persistent-kernel diagnostics of the last mode-0 call (synchronous):
 * *status 0 = ran to completion, 1 = a bounded barrier wait timed out (the
 * kernel then stopped early and the state is invalid). */
int esbgk_batch_status(esbgk_batch_t *b, int *status);

void esbgk_batch_destroy(esbgk_batch_t *b);

#ifdef __cplusplus
}
#endif
#endif /* ESBGK_H */
