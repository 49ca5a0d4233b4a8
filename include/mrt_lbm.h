/*
 * mrt_lbm.h -- C ABI of the MI355X (gfx950) library for the D3Q19
 * non-orthogonal multiple-relaxation-time lattice Boltzmann step with the
 * pseudopotential multiphase force (Li, Du, Fei, Luo & Yu, arXiv:1805.08643).
 *
 * Model, in the paper's notation (Sec. II):
 *   lattice velocities e_a of Eq. (2); variable fbar = f - G/2 of Eq. (3);
 *   moments m = M fbar with the non-orthogonal M of Eq. (12) (basis
 *   Eqs. (7)-(10)); relaxation m* = m - Lambda (m - m_eq) + (I - Lambda/2) S
 *   (Eq. (4)) with Lambda of Eq. (11), m_eq of Eq. (13), S of Eq. (14) and the
 *   thermodynamic-consistency term of Eq. (16); fbar* = M^-1 m*; streaming
 *   Eq. (5); density and velocity Eq. (6); interaction force Eq. (15) with the
 *   square-root pseudopotential on the Carnahan-Starling EOS of Eq. (58) or
 *   the exponential pseudopotential; wetting ghost layer Eq. (57).
 *   The orthogonal Gram-Schmidt operator the paper compares against is
 *   selected by LBM_OP_ORTH.
 *
 * Conventions
 *   - Lattice units: dt = dx = c = 1, c_s^2 = 1/3.
 *   - Node index i = (z * ny + y) * nx + x, x fastest.  Per-node fields are
 *     flat arrays of N = nx*ny*nz doubles; vector fields are three such
 *     planes back to back (x, y, z components: "SoA").
 *   - Populations in the canonical form are fbar_a(x, t) after streaming,
 *     stored f[a * N + i] for a = 0..18 in the order of Eq. (2).
 *   - Every pointer argument named dev_* or documented as "device" is a
 *     device (HBM) pointer, typically a torch tensor's data_ptr(); the caller
 *     owns it.  Host pointers are documented as such.
 *   - All work is enqueued on the HIP stream given at creation and is
 *     asynchronous unless stated ("synchronises").
 *   - Functions return lbm_status.  Parameters are validated before any HIP
 *     call; on error nothing is launched and lbm_last_error() (thread-local)
 *     holds a message.  No C++ exception crosses this boundary.
 */
#ifndef MRT_LBM_H
#define MRT_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
enum {
    LBM_OK = 0,
    LBM_ERR_INVALID_ARG = -1,      /* parameter out of range, null pointer */
    LBM_ERR_BUFFER_TOO_SMALL = -2, /* workspace or buffer smaller than required */
    LBM_ERR_HIP = -3,              /* a HIP runtime call failed */
    LBM_ERR_NONFINITE = -4,        /* diagnostics found a NaN/Inf population */
    LBM_ERR_UNSUPPORTED = -5       /* valid request the library does not implement */
};

/* Collision operator. */
enum { LBM_OP_NONORTH = 0, /* Eqs. (7)-(14), (16): the paper's model */
       LBM_OP_ORTH = 1     /* Gram-Schmidt orthogonal D3Q19 basis (comparison) */ };

/* Population storage in HBM.  Arithmetic is FP64 for F64 storage and FP32
 * otherwise.  F16S stores h_a = (fbar*_a - w_a rho_ref) * 2^f16_exp in IEEE
 * binary16 with w = 1/3, 1/18, 1/36 by velocity class: the expression is
 * evaluated exactly from the FP32 population and rounded once to nearest
 * even; loading gives h_a 2^-f16_exp + w_a rho_ref rounded once to FP32.  The
 * power-of-two factor only moves h into the normal range of binary16. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16S = 2, LBM_STORE_F16N = 3 };
/* F16N (binary16 relative to the pulling node) stores every population that
 * arrives at node x as h_a in binary16, standing for the value
 * w_a rt(x) + h_a 2^-f16_exp exactly, where rt(x) is the density of x at the
 * step that wrote the state (the sum of its 19 populations in FP32), itself
 * rounded to binary16 and kept in a twentieth plane: element 19 N + i of the
 * state holds rt of node i.  A node's populations then differ from their
 * shifts only by what streaming and collision changed in one step, instead of
 * by the whole liquid-vapour density contrast of F16S.  rho_ref is ignored.
 *   The step works on the deviations h_a 2^-f16_exp (exact in FP32) and the
 * density rt + their sum; the rest state's moments enter the collision
 * analytically.  Its stores round stochastically: the FP32 value of
 * (fbar*_a - w_a rt(x)) 2^f16_exp gets a 13-bit dither added to its bits and
 * is truncated toward zero to binary16, so a value rounds up with probability
 * equal to its fraction of a binary16 unit and changes smaller than half a
 * unit per step are kept in expectation instead of stagnating.  The dither
 * hashes a 32-bit seed, the index of the node whose population is stored and
 * the direction.  The seed sits after the planes (element 20 N, as a 32-bit
 * word followed by 12 zero bytes; the buffer holds 20 N + 8 elements): each
 * step reads it from the source and writes seed + 1 to the destination, and
 * lbm_init_fields, lbm_init_droplets and lbm_write_populations set it to 0
 * (so that a saved state holds no uninitialised bytes), so results are
 * deterministic and the same in plain launches, graph replays, batches and
 * lbm_step_noalloc.
 *   lbm_write_populations computes (f_a - w_a rt) 2^f16_exp in FP64 (the
 * product and the difference each rounded once) and rounds it once to
 * binary16 (to nearest); lbm_read_populations returns w_a rt + h_a
 * 2^-f16_exp in FP64 (product and sum each rounded once).  F16N runs the split
 * step only (nx a multiple of 4, walls only on z; batches too); its step moves
 * 40 instead of 38 values of 2 bytes per node. */

/* Pseudopotential form (text after Eq. (15)). */
enum { LBM_PSI_SQRT_CS = 0, /* psi = sqrt(2 (p_EOS - rho/3) / G), C-S p_EOS, Eq. (58) */
       LBM_PSI_EXP = 1      /* psi = psi0 exp(-rho0 / rho) */ };

typedef struct lbm_params {
    int32_t nx, ny, nz;     /* lattice size, each >= 1 (nz >= 2 with walls) */
    int32_t wall_z;         /* 0: periodic in z; 1: half-way bounce-back walls at
                               z = -1/2 and z = nz - 1/2 (x, y always periodic) */
    int32_t op;             /* LBM_OP_* */
    int32_t storage;        /* LBM_STORE_* */
    int32_t psi_form;       /* LBM_PSI_* */
    int32_t f16_exp;        /* F16S, F16N: stored value is (fbar - w rho_ref) * 2^f16_exp
                               (F16N: w rt(x)), in [-24, 24]; pick it so the largest
                               |fbar - w rho_ref| scaled stays below 2^15 (ignored
                               otherwise) */
    double rho_ref;         /* F16S shift density (ignored otherwise) */
    /* Relaxation rates, Eq. (11); each in (0, 2).  ORTH also uses s_eps (energy
     * square) and s_m (cubic m_x,y,z rows). */
    double s_e, s_nu, s_q, s_pi, s_eps, s_m;
    double G;               /* interaction strength, Eq. (15); < 0 for SQRT_CS */
    double eos_a, eos_b, eos_R; /* C-S constants, Eq. (58) */
    double T_over_Tc;       /* T = T_over_Tc * 0.37733 a / (b R) */
    double psi0, rho0;      /* exponential form constants */
    double sigma;           /* Eq. (16) constant */
    double gravity[3];      /* body acceleration g; body force rho g */
    double theta_wall_deg;  /* prescribed contact angle theta_a, Eq. (57) */
    double ghost_rho_min;   /* lower clamp of the Eq. (57) ghost density */
    /* Density-dependent kinematic viscosity for runs with nu_V != nu_L
     * (Sec. IV.D varies nu_V / nu_L without giving the rule; this is the
     * library's reading).  nu_ratio = 0 or 1: s_nu everywhere.  Otherwise
     * nu_L = (1/s_nu - 1/2)/3 (Eq. (54)), nu_V = nu_ratio nu_L, and a node of
     * density rho takes nu = nu_V + t (nu_L - nu_V) with
     * t = (rho - visc_rho_V) / (visc_rho_L - visc_rho_V) clamped to [0, 1];
     * its stress rows relax at 1 / (3 nu + 1/2).  nu_ratio must be >= 0 and
     * finite; when it is active, 0 <= visc_rho_V < visc_rho_L. */
    double nu_ratio, visc_rho_L, visc_rho_V;
    /* Half-way bounce-back walls at x = -1/2, nx - 1/2 (wall_x = 1) and
     * y = -1/2, ny - 1/2 (wall_y = 1), for single-phase runs only
     * (psi_form = LBM_PSI_EXP with G = 0; else LBM_ERR_UNSUPPORTED): the
     * lid-driven cavity of Appendix B.  The face y = ny - 1/2 moves with the
     * tangential velocity lid_u (lid_u[1] must be 0; nonzero lid_u needs
     * wall_y): a population reflected there gains
     * -2 w_a lid_rho (e_a . lid_u) / c_s^2 (a the direction that hit the
     * face, w = 1/18 axis, 1/36 diagonal), lid_rho > 0 when lid_u != 0.
     * These runs use their own step kernel (one node per thread, no psi) in
     * every step mode; batched runs must be periodic in x and y. */
    int32_t wall_x, wall_y;
    double lid_u[3];
    double lid_rho;
    /* Failure detection (the instability of Sec. IV.A at too small a
     * viscosity): with diag_every = K > 0, lbm_step checks the populations
     * for NaN / Inf every time the step count reaches a multiple of K (one
     * reduction on the device and one synchronisation of the stream) and
     * returns LBM_ERR_NONFINITE at the first check that finds any, the state
     * left at that step.  0: no checks.  Must be >= 0. */
    int32_t diag_every;
    /* Readings of the orthogonal comparison operator (LBM_OP_ORTH), which the
     * paper names but does not print (Secs. IV.A-B); ignored otherwise.
     * orth_meq: 0 = m_eq = M_orth f_eq of the textbook D3Q19 equilibrium,
     *   i.e. eps_eq = rho (3 - 11/2 |u|^2) and pi_eq = -p_eq / 2; 1 = the
     *   free parameters of the Gram-Schmidt D3Q19 model set to
     *   eps_eq = -475/63 rho |u|^2 and pi_eq = 0 (the stability-tuned choice
     *   for that basis); the source rows follow the equilibrium
     *   (S_eps = 2 w_epsj F.u, S_pi = w_xx S_p).
     * orth_sigma: rows that take the Eq. (16) term: 0 = the e row only
     *   (x 19; the reading that reproduces the paper's orthogonal Table II:
     *   rho_V rising with nu); 1 = e (x 19) and eps (x -16), the image of the
     *   non-orthogonal correction, which equals it for s_eps = s_e. */
    int32_t orth_meq;
    int32_t orth_sigma;
    int32_t reserved1;
} lbm_params;

/* Launch shape of the fused step: tx * ty threads per block, one thread per
 * (x, y) column of a tx x ty tile, marching cz planes in z. */
typedef struct lbm_tile {
    int32_t tx, ty, cz, reserved;
} lbm_tile;

/* One droplet of the Eq. (59) initial condition. */
typedef struct lbm_droplet {
    double center[3];
    double r0;
    double u[3];            /* velocity scaled by the liquid fraction */
} lbm_droplet;

/* Region selection for the Laplace-law sums: "inside" is |x - c| < r_in,
 * "outside" is |x - c| > r_out (minimum-image distance on periodic axes). */
typedef struct lbm_diag_request {
    double center[3];
    double r_in, r_out;
} lbm_diag_request;

typedef struct lbm_diag {
    double mass;            /* sum rho (FP64) */
    double momentum[3];     /* sum (sum_a e_a fbar_a + F/2) (FP64) */
    double max_u;           /* max |u| */
    double p_in, p_out;     /* sums of p = rho/3 + G psi^2/2 in the two regions */
    double rho_in, rho_out; /* sums of rho in the two regions */
    double n_in, n_out;     /* node counts of the two regions */
    int64_t nonfinite;      /* populations that are NaN or Inf */
    int64_t step;           /* time steps taken so far */
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

/* Paper defaults: c_s^2 = 1/3 implied; conserved rates 1; C-S b = 4, R = 1,
 * a = 0.5; G = -1; sigma = 0; theta = 90 deg; F32 storage, non-orthogonal,
 * periodic.  nx = ny = nz = 32.  Rates s_e = s_nu = s_q = s_pi = s_eps =
 * s_m = 1. */
void lbm_params_default(lbm_params *p);

/* Device bytes needed by lbm_create for these parameters: two population
 * buffers of 19 N elements (20 N + 8 for F16N), a psi buffer of N, wall planes
 * and diagnostics partials, each 256-byte aligned. */
lbm_status lbm_workspace_bytes(const lbm_params *p, size_t *bytes);

/* Create a lattice on the current device.  dev_ws: device buffer of at least
 * lbm_workspace_bytes bytes, owned by the caller and kept alive until
 * lbm_destroy.  hip_stream: a hipStream_t (may be NULL = default stream),
 * borrowed.  The library allocates host memory only.  Populations are left
 * undefined until an init call. */
lbm_status lbm_create(const lbm_params *p, void *dev_ws, size_t ws_bytes, void *hip_stream,
                      lbm_ctx **out);
lbm_status lbm_destroy(lbm_ctx *ctx);

/* fbar(x, 0) = M^-1 m_eq(rho(x), u(x)) (Eq. (13)), i.e. the equilibrium of
 * the chosen operator.  rho: device, N doubles; u: device, 3N doubles. */
lbm_status lbm_init_fields(lbm_ctx *ctx, const double *rho, const double *u);

/* Same, with rho and u from the Eq. (59) tanh profile of each droplet
 * (host array of n <= 8): at each node the droplet with the largest profile
 * gives rho, and u = u_d (rho - rho_V) / (rho_L - rho_V). */
lbm_status lbm_init_droplets(lbm_ctx *ctx, const lbm_droplet *d, int32_t n, double rho_L,
                             double rho_V, double W);

/* Advance nsteps time steps (asynchronous unless diag_every > 0): each step is
 * the update of Sec. II -- density and pseudopotential (Eq. (6), Eq. (58)),
 * interaction force (Eq. (15), Eq. (57) at walls), velocity (Eq. (6)),
 * collision in moment space (Eqs. (4), (11)-(14), (16)) and pull streaming
 * with periodic wrap or half-way bounce-back (Eq. (5)).  With graph steps set
 * (lbm_set_graph_steps), runs of that many steps replay a captured hipGraph. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Replay steps from captured hipGraphs of k steps each (k >= 1), or plain
 * launches (k = 0, the default): lbm_step then launches one graph per k steps
 * (captured on first use on a stream of the library, one graph per buffer
 * parity) and the rest step by step.  Bit for bit the same results; it cuts
 * the launch cost of small lattices.  Changing the tile, the step mode, the
 * store policy or the write check drops the captured graphs.  Steps are not
 * replayed from graphs while kernel timing (lbm_set_timing) is on.
 * k < 0: LBM_ERR_INVALID_ARG. */
lbm_status lbm_set_graph_steps(lbm_ctx *ctx, int32_t k);

/* One time step for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * step of lbm_step (Sec. II, Eqs. (3)-(6), (15), (57)) from the populations
 * in dev_src to dev_dst, with no context and no allocation of host or device
 * memory.
 *   p: the lattice parameters (validated as by lbm_create).
 *   dev_src, dev_dst: distinct device buffers of 19 N storage elements each
 *     (20 N + 8 for F16N, whose seed word dev_src supplies and dev_dst
 *     receives incremented),
 *     256-byte aligned, in the layout of the raw state (lbm_save_state):
 *     element a * N + i holds direction a of node i, in the storage format of
 *     p->storage; owned by the caller.  dev_src is read, dev_dst written.
 *   hip_stream: hipStream_t (NULL = default stream), borrowed; asynchronous.
 * It runs the step kernel and launch shape that a new context with these
 * parameters uses, so its result is bit for bit that of lbm_step.  Scratch
 * (the wall-plane densities and the Eq. (57) ghost psi planes, walls only)
 * lives in a device array inside the library, LBM_NOALLOC_SCRATCH_BYTES on
 * every GPU the library runs on, held until the process ends.  A walled
 * lattice whose planes need more (6 nx ny values, each plane set 256-byte
 * aligned) returns LBM_ERR_UNSUPPORTED before any HIP call.  The first call
 * on a device looks up that device's array address (no allocation).  Calls
 * that overlap on one GPU share its scratch and race: serialise them (one
 * stream, or events). */
#define LBM_NOALLOC_SCRATCH_BYTES (32 << 20)
lbm_status lbm_step_noalloc(const lbm_params *p, const void *dev_src, void *dev_dst, void *hip_stream);

/* Macroscopic fields of the current state, Eq. (6): rho (N), u (3N),
 * p = rho/3 + G psi^2/2 (N); device FP64 outputs, any may be NULL. */
lbm_status lbm_read_fields(lbm_ctx *ctx, double *rho, double *u, double *p);

/* Canonical populations fbar_a(x, t) (19 N device doubles) out / in.
 * Storage rounds to the storage precision; with a moving lid the
 * populations reflected off it are stored without the lid term and read
 * back with it, so a round trip may differ there in the last bit. */
lbm_status lbm_read_populations(lbm_ctx *ctx, double *f);
lbm_status lbm_write_populations(lbm_ctx *ctx, const double *f);

/* FP64 global sums of the current state (see lbm_diag): mass and momentum
 * (Eq. (6), with F/2), max |u|, and the sums of p = rho/3 + G psi^2 / 2 and
 * rho inside and outside a sphere for the Laplace law (Sec. IV.B); fixed
 * summation order, so the same state gives the same bits.  req may be NULL
 * (no Laplace sums).  out: host pointer.  Synchronises the stream.  Returns
 * LBM_ERR_NONFINITE (with out filled) when any population is not finite. */
lbm_status lbm_diagnostics(lbm_ctx *ctx, const lbm_diag_request *req, lbm_diag *out);

/* Raw state (storage-format populations plus the step counter) to/from a
 * device buffer of lbm_state_bytes bytes; resuming is bit-identical. */
lbm_status lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
lbm_status lbm_save_state(lbm_ctx *ctx, void *dev_buf, size_t bytes);
lbm_status lbm_load_state(lbm_ctx *ctx, const void *dev_buf, size_t bytes);

/* Launch shape.  set validates (tx in [1, 1024], tx * ty <= 1024, cz >= 1,
 * halo ring 2 (tx + ty) + 4 <= tx * ty).  autotune times `trials` steps of
 * each candidate shape (output written to the scratch buffer only, so the
 * state is unchanged), keeps the fastest, and reports it.  Synchronises. */
lbm_status lbm_set_tile(lbm_ctx *ctx, const lbm_tile *t);
lbm_status lbm_get_tile(const lbm_ctx *ctx, lbm_tile *t);
lbm_status lbm_autotune(lbm_ctx *ctx, int32_t trials, lbm_tile *best);

/* Step implementation (all of one time step, Sec. II and Eq. (5)).
 * LBM_STEP_FUSED: one kernel per step, tiles marching in z with psi and its
 * halo in LDS, one node per thread.  LBM_STEP_SLABS: per z-slab of
 * slab_planes planes, a psi pass then a collide pass that re-reads the slab
 * (sized to stay in the last-level cache) and reads psi from a global array.
 * LBM_STEP_PAIRS: the fused kernel with two x-adjacent nodes per thread and
 * one wide access per direction for both; FP32 and F16S storage with even nx.
 * LBM_STEP_QUADS: four x-adjacent nodes per thread, one 8-byte access per
 * direction; F16S storage with nx a multiple of 4.  LBM_STEP_SPLIT: 8-byte
 * groups of nodes (four F16S or two FP32 per thread) with the block split by
 * wave into pullers (global loads, psi, populations into LDS) running three
 * planes ahead of colliders (collision from LDS, stores), so memory and
 * arithmetic overlap; F16S or F16N with nx a multiple of 4 or FP32 with even nx; tile
 * width a multiple of the group size and at most 256, at most 256 groups and
 * 1024 nodes, (tx + 2)(ty + 2) <= 1548 (1300 for F16N), and a halo ring 2 (tx + ty) + 4 of at
 * most 512 nodes for F16S or 768 for FP32 (tuned: 128 x 8 nodes for F16S,
 * 128 x 4 for FP32).
 * A mode that does not apply
 * returns LBM_ERR_UNSUPPORTED.  With 2 or 4 nodes per thread the tile width
 * must be a multiple of that count (lbm_set_tile returns LBM_ERR_INVALID_ARG
 * otherwise); switching to a mode whose kernel cannot run the current tile
 * replaces the tile by the mode's default (rows of up to 128 nodes).
 * slab_planes is used by LBM_STEP_SLABS only but must be >= 1.
 * All modes give the same populations bit for bit.  A new context uses
 * LBM_STEP_SPLIT where it applies, else LBM_STEP_PAIRS where that applies,
 * else LBM_STEP_FUSED. */
enum { LBM_STEP_FUSED = 0, LBM_STEP_SLABS = 1, LBM_STEP_PAIRS = 2, LBM_STEP_QUADS = 3, LBM_STEP_SPLIT = 4 };
lbm_status lbm_set_step_mode(lbm_ctx *ctx, int32_t mode, int32_t slab_planes);
/* Current step mode and slab size (slab_planes may be NULL). */
lbm_status lbm_get_step_mode(const lbm_ctx *ctx, int32_t *mode, int32_t *slab_planes);

/* Average device time of one step's kernels (fused mode: the step kernel;
 * slab mode: the psi and collide passes of all slabs) over the steps launched
 * since the last call, measured with HIP events on the context's stream when
 * timing is enabled (lbm_set_timing(ctx, 1)).  Synchronises. */
lbm_status lbm_set_timing(lbm_ctx *ctx, int32_t enable);

/* Write check, a debug aid for the streaming of Eq. (5): each step must
 * write all 19 populations of every node.  With enable != 0, every step first
 * fills the destination population buffer with all-ones bits (NaN in FP64,
 * FP32 and F16S storage).  A node the step fails to write then shows up as
 * non-finite in lbm_diagnostics and in the populations.  Costs one extra
 * write pass per step, outside the timed region of lbm_set_timing; kernels
 * only, so a captured step stays capturable. */
lbm_status lbm_set_write_check(lbm_ctx *ctx, int32_t enable);

/* Cache policy of the split step's population stores (LBM_STEP_SPLIT; other
 * step modes always store cached).  LBM_STORE_AUTO (the default) stores
 * non-temporally when the two population arrays together exceed the GPU's
 * 256 MiB last-level cache, where cached stores would evict the lines the next
 * plane's reads need; LBM_STORE_CACHED and LBM_STORE_STREAM force either
 * policy.  Results are bit for bit the same under every policy; only the
 * speed differs.  An unknown policy returns LBM_ERR_INVALID_ARG. */
enum { LBM_STORE_AUTO = 0, LBM_STORE_CACHED = 1, LBM_STORE_STREAM = 2 };
lbm_status lbm_set_store_policy(lbm_ctx *ctx, int32_t policy);
lbm_status lbm_kernel_time(lbm_ctx *ctx, double *avg_ms, int64_t *launches);

int64_t lbm_step_count(const lbm_ctx *ctx);
const char *lbm_status_string(lbm_status s);
const char *lbm_last_error(void);

/* ---------------------------------------------------------------------------
 * Batched independent runs (periodic lattices, common op and storage): one
 * persistent launch advances every run by one step; nsteps launches are
 * captured once in a hipGraph and replayed.
 * ------------------------------------------------------------------------- */
lbm_status lbm_batch_workspace_bytes(const lbm_params *runs, int32_t n, size_t *bytes);
lbm_status lbm_batch_create(const lbm_params *runs, int32_t n, void *dev_ws, size_t ws_bytes,
                            void *hip_stream, lbm_batch **out);
lbm_status lbm_batch_destroy(lbm_batch *b);
lbm_status lbm_batch_init_droplets(lbm_batch *b, int32_t run, const lbm_droplet *d, int32_t n,
                                   double rho_L, double rho_V, double W);
lbm_status lbm_batch_init_fields(lbm_batch *b, int32_t run, const double *rho, const double *u);
/* graph_steps > 0: capture that many steps in a hipGraph and replay it;
 * 0: plain launches. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps, int32_t graph_steps);
lbm_status lbm_batch_read_fields(lbm_batch *b, int32_t run, double *rho, double *u, double *p);
lbm_status lbm_batch_read_populations(lbm_batch *b, int32_t run, double *f);
/* Diagnostics of run `run`, as lbm_diagnostics gives them for a single
 * lattice (Sec. IV.B sums; FP64, fixed order); synchronises the stream.
 * LBM_ERR_NONFINITE (out still filled) if that run holds NaN or Inf. */
lbm_status lbm_batch_diagnostics(lbm_batch *b, int32_t run, const lbm_diag_request *req, lbm_diag *out);
/* Status of every run: status[k] = LBM_OK, or LBM_ERR_NONFINITE when the
 * populations of run k hold NaN or Inf.  status: host array of
 * lbm_batch_runs(b) entries, owned by the caller.  Returns LBM_OK when all
 * runs are finite, LBM_ERR_NONFINITE (message names the first such run)
 * otherwise, or the first HIP error.  Synchronises the stream. */
lbm_status lbm_batch_status(lbm_batch *b, lbm_status *status);
/* Number of runs in the batch (0 for NULL). */
int32_t lbm_batch_runs(const lbm_batch *b);
/* Persistent grid size (blocks), per-run tiles and step kernel (one or two
 * nodes per thread, or the split step, where they apply) chosen by timing candidates;
 * synchronises; state unchanged. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t trials, int32_t *best_blocks);
lbm_status lbm_batch_set_blocks(lbm_batch *b, int32_t blocks);
/* Nodes per work item (a run's tile holds about this many nodes: whole rows
 * of up to 128 nodes times the z run that reaches it), in [1, 2^24]; rebuilds
 * the work list and drops captured graphs, and caps the grid at the new tile
 * count.  With lbm_batch_set_step_mode and lbm_batch_set_blocks it restores a
 * shape that lbm_batch_autotune chose (the tuning cache of the Python
 * binding does).  Results are bit for bit the same for every value. */
lbm_status lbm_batch_set_item_nodes(lbm_batch *b, int32_t item_nodes);
/* Current step mode, nodes per work item and grid size; any pointer may be NULL. */
lbm_status lbm_batch_get_tuning(const lbm_batch *b, int32_t *mode, int32_t *item_nodes, int32_t *blocks);
/* Step kernel of the batch: LBM_STEP_FUSED, LBM_STEP_PAIRS (two nodes per
 * thread; FP32/F16S storage and even nx in every run) or LBM_STEP_SPLIT
 * (pulling and colliding waves; FP32 with even nx or F16S with nx a multiple
 * of 4 in every run; the only mode of F16N batches); otherwise
 * LBM_ERR_UNSUPPORTED.  A new batch uses
 * LBM_STEP_SPLIT where it applies to every run, else LBM_STEP_PAIRS where that
 * applies, else LBM_STEP_FUSED.  Rebuilds the work list and drops captured
 * graphs; results are bit for bit the same in all modes. */
lbm_status lbm_batch_set_step_mode(lbm_batch *b, int32_t mode);
/* Store policy of the batch's split step, as lbm_set_store_policy, judged on
 * the whole population pool of the batch.  Drops captured graphs. */
lbm_status lbm_batch_set_store_policy(lbm_batch *b, int32_t policy);
lbm_status lbm_batch_get_step_mode(const lbm_batch *b, int32_t *mode);
lbm_status lbm_batch_kernel_time(lbm_batch *b, double *avg_ms, int64_t *launches);
int64_t lbm_batch_nodes(const lbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MRT_LBM_H */
