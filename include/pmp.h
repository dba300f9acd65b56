/*
 * libpmp — particle-mesh-particle interactions on one MI355X (gfx950).
 *
 * Implements the data-parallel hot path of He et al. (2025), "A GPU-optimised
 * particle-mesh-particle algorithm" (Quokka), Sec. 2.2:
 *
 *   pmp_deposit      Step 1  particles -> zeroed, ghost-zoned buffer mesh
 *                            (eq. "delta_u_buf"), atomic adds
 *   pmp_ghost_fold   Step 2  ghost zones -> owning cells (periodic images and
 *                            neighbouring boxes held by this GPU)
 *   pmp_sink_update  Step 4  sinks gain the limited removal
 *   pmp_apply        Steps 3 + 5  cell-wise limiter, then U := U + dU_lim
 *
 * Calling order for one step: deposit, ghost_fold, sink_update (only with
 * sinks; it reads the state before the mesh update), apply.  pmp_step runs
 * all of them; pmp_graph_build/pmp_graph_launch capture and replay several
 * steps as one HIP graph.
 *
 * Conventions for every function:
 *  - returns PMP_OK (0) or a negative PMP_E* code; never aborts, never throws;
 *    pmp_last_error() returns a message for the calling thread's last error;
 *  - pointers named "device" must be device memory (hipMalloc / PyTorch CUDA
 *    tensors) readable and writable by the GPU the context was created on;
 *    pointers named "host" are ordinary host memory;
 *  - the caller owns every array it passes; the library never frees them and
 *    keeps no pointer to them after the call returns (the graph functions
 *    excepted, see there);
 *  - stream: a hipStream_t passed as void* (NULL = the null stream); work is
 *    enqueued asynchronously and no call synchronises the stream except
 *    pmp_get_status and pmp_autotune;
 *  - data-dependent problems found on the GPU (a particle outside its box, a
 *    stencil reaching beyond the ghost zone, fixed-point overflow, NaN input,
 *    an infeasible energy floor) do not abort: the offending contribution is
 *    skipped and a bit is set in the status word read by pmp_get_status.
 *
 * Units and layout (Sec. 2.1, "Formulation of the problem"):
 *  - positions are in cell units of the global index space: a particle at x
 *    lies in cell floor(x); cell (i,j,k) has its centre at (i+1/2, j+1/2,
 *    k+1/2); dx is the cell edge and V = dx^3;
 *  - box b owns global cells [lo_b, lo_b + n_b) (x, y, z); boxes must not
 *    overlap; the domain is periodic along all three axes;
 *  - state = concatenation over boxes, in box order, of [5][nz][ny][nx]
 *    arrays (rho, px, py, pz, E), x fastest; float or double;
 *  - buffer = concatenation over boxes of [F][nz+2g][ny+2g][nx+2g]: the F
 *    channels present (pmp_layout.channels) in the order rho, px, py, pz, E,
 *    K (sink removal, >= 0); float, double, or int64 fixed point with
 *    value = q * 2^-40;
 *  - each particle kind is a set of device float64 arrays grouped by box,
 *    with a device int64 CSR array box_off[nbox+1] (particles of box b are
 *    [box_off[b], box_off[b+1])); floor(x) must lie in box b.
 */
#ifndef PMP_H
#define PMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMP_OK 0
#define PMP_EINVAL (-1)       /* bad argument (null pointer, bad enum, size mismatch) */
#define PMP_ERANGE (-2)       /* geometry: overlapping boxes, box outside the domain,
                                 ghost width smaller than a kernel's reach */
#define PMP_EDEVICE (-3)      /* a HIP runtime call failed */
#define PMP_ENOMEM (-4)       /* device or host allocation failed */
#define PMP_EUNSUPPORTED (-5) /* valid request this build does not implement */

/* status-word bits (pmp_status.flags) */
#define PMP_FLAG_OUTSIDE 0x1u   /* particle's host cell not in its box (skipped) */
#define PMP_FLAG_REACH 0x2u     /* stencil member outside the ghost zone (skipped) */
#define PMP_FLAG_OVERFLOW 0x4u  /* fixed-point value outside (-2^62, 2^62) */
#define PMP_FLAG_NAN 0x8u       /* non-finite particle or state value seen */
#define PMP_FLAG_FLOOR 0x10u    /* energy floor infeasible: E raised (counted in fall) */
#define PMP_FLAG_CAPACITY 0x20u /* binned path: tile entry list full (entries skipped) */

/* PMP_ACC_F64R: the reproducibility mode of App. A.1.  The buffer is FP64;
 * every addition to a buffer element also adds eps |sum after the addition|
 * (eps = 2^-52) to that element's error bound, and once the element's
 * deposits are complete its lowest 52 + M + ceil(log2(bound / |sum|))
 * mantissa bits (clamped to [0, 52]) are cleared, M = margin_bits.  Binned
 * path only (deposit_path 1), tiles never split. */
typedef enum { PMP_ACC_F32 = 0, PMP_ACC_F64 = 1, PMP_ACC_FIX64 = 2, PMP_ACC_F64R = 3 } pmp_acc_t;
typedef enum { PMP_STATE_F32 = 0, PMP_STATE_F64 = 1 } pmp_state_t;

typedef struct pmp_ctx pmp_ctx;

/* Mesh description, copied into the context by pmp_create. */
typedef struct {
  int32_t nbox;        /* number of boxes (>= 1) */
  const int32_t *lo;   /* host [nbox][3]: first owned global cell (x, y, z) */
  const int32_t *n;    /* host [nbox][3]: owned cells per axis (>= 1) */
  int32_t ghost;       /* ghost width g (>= 1 when CIC particles are deposited,
                          >= floor(r + 1/2) for a sphere of radius r) */
  int32_t domain[3];   /* periodic domain in cells */
  double dx;           /* cell edge (> 0) */
  int32_t acc;         /* pmp_acc_t: buffer accumulator type */
  int32_t state;       /* pmp_state_t: state element type */
  int32_t with_sinks;  /* 1: buffer has the removal channel K */
  int32_t channels;    /* buffer channels present, PMP_CH_* bits; 0 = rho, p and E
                          (+ K with sinks).  A channel no particle kind deposits
                          into is identically zero and need not be stored:
                          CIC needs RHO, supernovae RHO | E, sinks K; absent
                          channels read as zero in the apply. */
  int32_t margin_bits; /* PMP_ACC_F64R: the safety margin M, 0 .. 52 (the
                          paper's example: 28); ignored otherwise */
} pmp_layout;

#define PMP_CH_RHO 0x1
#define PMP_CH_MOM 0xe   /* px, py, pz together */
#define PMP_CH_E 0x10
#define PMP_CH_K 0x20

/* CIC mass particles (Sec. 2.2: PM deposit using steps 1, 2 and 5). */
typedef struct {
  const double *x, *y, *z, *m;  /* device [n] */
  int64_t n;
  const int64_t *box_off;       /* device [nbox+1] */
} pmp_cic;

/* Supernova particles: mass m and energy e spread uniformly over the cells
 * whose centres lie within radius r (Sec. 3.2.1, eq. "du" with full coverage
 * and no momentum term). */
typedef struct {
  const double *x, *y, *z, *m, *e, *r;  /* device [n] */
  int64_t n;
  const int64_t *box_off;               /* device [nbox+1] */
  double r_max;                         /* host: largest r, for the ghost check */
} pmp_sn;

/* Supernova remnants with the variant of the TIGRESS prescription of
 * Sec. 3.2.1 (eqs. "du", "dp", "psnr"), deposited by pmp_deposit_snr.  Code
 * units throughout: nh_per_rho converts a mass density to the number density
 * of H nuclei in cm^-3 (1 / (mu_H m_H)); msf_coef and psnr_coef are the
 * shell-formation mass and the terminal momentum at n_H = 1 cm^-3 (1679 Msun
 * and 2.8e5 Msun km/s in the paper); eps_k the kinetic fraction of the
 * Sedov-Taylor phase (0.28). */
typedef struct {
  const double *x, *y, *z;        /* device [n]: position (cells) */
  const double *m, *e;            /* device [n]: ejecta mass M_ej, supernova energy E_sn */
  const double *vx, *vy, *vz;     /* device [n]: velocity of the exploding particle */
  int64_t n;
  const int64_t *box_off;         /* device [nbox+1] */
  double r_k;                     /* kernel radius r_K (cells), 0 .. 16 */
  int32_t sub;                    /* sample points per axis for the covered fraction:
                                     1, 2, 4, 8 or 16 */
  double nh_per_rho, msf_coef, psnr_coef, eps_k;  /* > 0, > 0, >= 0, >= 0, finite */
} pmp_snr;

/* Sink request rates (pmp_sinks.rate). */
typedef enum {
  PMP_SINK_FRACTION = 0,  /* the fraction a of the kernel gas mass, Gaussian width r_gauss */
  PMP_SINK_BONDI = 1      /* the Bondi-Hoyle-Lyttleton rate, width r_acc per sink */
} pmp_sink_rate_t;

/* Sink particles (Sec. 3.1.1).  Each removes gas from the cells whose centres
 * lie within r_k, spread with Gaussian weights exp(-d^2/r_acc^2) normalised
 * over those cells (eqs. "kernel", "kernel_wgt"); a cell's removal is at least
 * rho - rho_Tr (eq. "accretion_function").  The requested mass is
 *   PMP_SINK_FRACTION: a times the kernel gas mass sum rho V, r_acc = r_gauss;
 *   PMP_SINK_BONDI: mdot dt with mdot = 4 pi rho_inf r_BH^2
 *     (lambda^2 c_inf^2 + v_inf^2)^(1/2) and r_BH = G m / (v_inf^2 + c_inf^2)
 *     (eqs. "rbh", "mdot"), where over the kernel cells v_inf is the length of
 *     the mass-weighted mean gas velocity minus the sink velocity, c_inf the
 *     mass-weighted mean of c_s = (gamma (gamma-1) e_int / rho)^(1/2) (e_int =
 *     E - |p|^2/(2 rho), negative values taken as 0) and rho_inf the mean
 *     density (kernel mass over kernel volume); the request is capped at the
 *     kernel gas mass (also when v_inf = c_inf = 0), and r_acc = r_BH / dx
 *     clamped to [1/4, r_k/2] cells (r_k/2 when the rate is not finite).
 * The kernel sums are taken on the 2^-40 grid, so they do not depend on the
 * order of summation (PMP_FLAG_OVERFLOW past 2^22 per term).  Any box
 * layout: sinks are grouped by box like the other kinds (box_off), the
 * kernel reads the state of whichever box owns each (periodically wrapped)
 * cell, the removal goes to the sink's own box (its ghost zone where the
 * kernel leaves the box; the fold moves it to the owners), and Step 4 reads
 * eta from the owners.  A kernel cell that no box owns is skipped and raises
 * PMP_FLAG_REACH. */
typedef struct {
  const double *x, *y, *z, *a;  /* device [n]; a is read by PMP_SINK_FRACTION only */
  int64_t n;
  const int64_t *box_off;       /* device [nbox+1] */
  double r_k, r_gauss;          /* host scalars, cells; r_gauss: PMP_SINK_FRACTION only */
  int32_t rate;                 /* pmp_sink_rate_t */
  const double *m, *vx, *vy, *vz;  /* device [n], PMP_SINK_BONDI: sink mass and velocity */
  double G, dt, gamma, lambda;  /* host, PMP_SINK_BONDI: gravitational constant, time step,
                                   adiabatic index (>= 1), BHL lambda (e^(3/2)/4 in the
                                   paper); G, dt, lambda >= 0 and finite, r_k >= 1/2 */
} pmp_sinks;

/* Limiter parameters (Sec. 3.1.1 removal limiter, Sec. 3.2.1 eq. "lambda").
 * The Truelove density rho_Tr (Sec. 3.1.1, eq. "truelove") enters the sink
 * removal k = max(M_req w / (W V), rho - rho_Tr), the removal limiter and
 * sink creation.  With truelove_J = 0 it is the constant rho_tr; with
 * truelove_J > 0 every cell has its own,
 *   rho_Tr = J^2 pi c_s^2 / (G dx^2),  c_s^2 = gamma (gamma - 1) e_int / rho,
 * e_int = E - |p|^2 / (2 rho) from the cell's state (negative values as 0,
 * c_s = 0 where rho <= 0), and rho_tr is ignored (J = 1/4 in the paper). */
typedef struct {
  double rho_floor;   /* density never drops below this by removal */
  double rho_tr;      /* constant Truelove density (+inf disables the term) */
  double cap;         /* largest removed fraction per step (0.25 in the paper) */
  int32_t eint_mode;  /* 0: e_int >= 0; 1: specific e_int may not drop */
  double truelove_J;  /* 0: constant rho_tr; > 0 (finite): per-cell rho_Tr with this J */
  double G;           /* gravitational constant of the per-cell rho_Tr (> 0, finite) */
  double gamma;       /* adiabatic index of the per-cell rho_Tr (>= 1, finite) */
} pmp_limits;

/* Device-side diagnostics accumulated since the last reset. */
typedef struct {
  uint32_t flags;     /* PMP_FLAG_* */
  uint32_t reserved;
  int64_t touched;    /* apply: cells with K > 0 */
  int64_t bind;       /* apply: cells where the removal limiter binds */
  int64_t lam;        /* apply: cells with lambda < 1 */
  int64_t fall;       /* apply: cells where the floor was infeasible */
} pmp_status;

/* Kernel tuning; pmp_create fills defaults, pmp_autotune overwrites. */
typedef struct {
  int32_t deposit_path;  /* 0: zero fill, then direct global atomic adds;
                            1: particles binned into tiles of the padded box
                            their stencil touches, each tile accumulated in
                            LDS by one workgroup and stored once (no global
                            atomics, no separate zero fill) */
  int32_t tile_x;        /* tile edge along x: 16, 32, 64, 128 or 256 cells (long x
                            tiles give long contiguous state rows in the fused apply) */
  int32_t tile_yz;       /* tile edge along y and z: 2, 4 or 8 cells */
  int32_t tile_block;    /* threads per tile workgroup: 64 .. 1024 */
  int32_t block;         /* threads per block of the streaming kernels */
  int32_t grid_per_cu;   /* cap on blocks per CU for grid-stride launches */
  int32_t sn_lanes;      /* lanes cooperating on one supernova: 16, 32 or 64 */
  int32_t tile_grid_per_cu; /* cap on tile workgroups per CU (0: one per tile) */
  int32_t chunk_cic;     /* binned path: a tile holding more CIC entries than
                            this (64 .. 2^24) is split into chunks of at most
                            this many, each accumulated in LDS by its own
                            workgroup; the last chunk to finish sums the
                            chunks' partial tiles in chunk order and stores */
  int32_t chunk_sn;      /* the same threshold for supernova entries (16 .. 2^24) */
  int32_t fuse_apply;    /* 1: pmp_step without sinks on the binned path applies
                            Steps 3 + 5 inside the tile pass for owned cells at
                            least g from every box face (no ghost image reaches
                            them), then folds and applies the shell cells in one
                            kernel; results are those of the separate calls.
                            The buffer's interior cells are left unwritten.
                            2: owner tiles, no ghost zone and no fold: tiles
                            cover owned cells only, each particle is binned into
                            every tile (of any box) that a periodic image of its
                            stencil reaches, and the tile pass applies every
                            owned cell from its complete LDS sum (Steps 2, 3
                            and 5 fused; the same sums as the fold, added in
                            another order: fixed point bit for bit, floats
                            rounded once).  The buffer is not written; in a
                            step with sinks the tiles a sink kernel may reach
                            are stored instead, the sinks add their removal
                            to the owning cells, and after the sink update
                            those tiles are applied; no fold runs.  Needs every tile extent along an axis to
                            be at most the domain less 2g cells, the binned
                            path and not PMP_ACC_F64R; where that does not hold
                            the step runs as with 1. */
  int32_t count_lanes;   /* binned path: lanes counting one supernova's sphere
                            members (its candidate rows dealt round them):
                            1, 2, 4, 8 or 16 */
} pmp_tuning;

/* Create a context on the current HIP device.  Copies the layout, checks the
 * geometry (PMP_ERANGE on overlap or boxes outside the domain) and builds the
 * ghost-fold plan.  Allocates device memory for the box table, the fold plan
 * and the status word. */
int pmp_create(pmp_ctx **out, const pmp_layout *L);
void pmp_destroy(pmp_ctx *ctx);

/* Element counts of the state and buffer arrays for this layout (host out). */
int pmp_sizes(const pmp_ctx *ctx, int64_t *state_elems, int64_t *buffer_elems,
              int64_t *owned_cells);

/* Scratch of the deposits (the binned path's two-level sort, supernova
 * records and split-tile partials; the sinks' kernel sums), which the
 * context otherwise allocates itself on first use.  pmp_workspace_size
 * writes to *bytes (host) the device bytes (a multiple of 256) a caller-owned workspace needs
 * for deposits of at most max_cic CIC particles, max_sn supernovae of
 * radius at most max_sn_radius (cells) and max_sinks sinks, for the current
 * tuning (the tile shape changes it: call again after pmp_set_tuning or
 * pmp_autotune).  PMP_EINVAL on negative counts, PMP_ERANGE where the
 * deposit itself would be out of range. */
int pmp_workspace_size(const pmp_ctx *ctx, int64_t max_cic, int64_t max_sn,
                       double max_sn_radius, int64_t max_sinks, size_t *bytes);

/* Hand the context a caller-owned device workspace (dev_ptr: 256-byte
 * aligned, at least 256 bytes; the caller keeps ownership and keeps it alive
 * while the context uses it).  The context frees its own scratch and from
 * then on carves every scratch array from the workspace: pmp_deposit,
 * pmp_sink_update, pmp_step, pmp_step_per_box and pmp_graph_build allocate
 * nothing, and a deposit whose scratch does not fit returns PMP_ERANGE with
 * the bytes it needs.  Calls on one context share the workspace (as they
 * share the buffer).  dev_ptr NULL returns to library-owned scratch.
 * PMP_EINVAL on misalignment or while a built graph exists (it holds scratch
 * addresses).  pmp_set_tuning (a new tile shape) and pmp_autotune (a state
 * copy) still allocate; the tuner skips tile shapes whose scratch does not
 * fit the workspace.  Synchronises the device. */
int pmp_set_workspace(pmp_ctx *ctx, void *dev_ptr, size_t bytes);

/* Step 1 (Sec. 2.2, eq. "delta_u_buf").  Zeroes the device buffer, then adds
 * every particle's deposition function with atomic adds.  state (device) is
 * read by sinks only (may be NULL without sinks).  Any of cic, sn, sinks may
 * be NULL.  limits is read for rho_tr (Truelove term) when sinks are given.
 * In PMP_ACC_FIX64 every contribution is rounded to the 2^-40 grid (half to
 * even) and each particle's rounding residue goes to its host cell, so the
 * buffer total equals the particle total exactly and the result does not
 * depend on execution order. */
int pmp_deposit(pmp_ctx *ctx, void *buf, const void *state, const pmp_cic *cic,
                const pmp_sn *sn, const pmp_sinks *sinks, const pmp_limits *limits,
                void *stream);

/* Step 1 for supernova remnants (Sec. 3.2.1, eqs. "du", "dp", "psnr"):
 * adds each remnant's deposition function to a buffer that pmp_deposit has
 * filled (call it after pmp_deposit, before pmp_ghost_fold).  Per remnant s:
 *   kernel   cells with a covered fraction w > 0, w = the share of the cell's
 *            sub^3 sub-cell centres within r_K (squared distance <= r_K^2);
 *            the host cell alone (w = 1) when no sample point is that close;
 *   sums     on the 2^-40 grid: V_snr = sum w V, M_gas = sum w rho V,
 *            P_gas = sum w p V, the state read in place in the box that owns
 *            each (periodically wrapped) cell;
 *   regime   M_snr = M_gas + M_ej, n_H = nh_per_rho M_snr / V_snr,
 *            R_M = M_snr / (msf_coef n_H^-0.26); |p_rad| = psnr_coef
 *            n_H^-0.17 if R_M > 1 (MC), sqrt(2 M_ej eps_k E_sn) if
 *            0.027 < R_M <= 1 (ST), else 0 (EJ);
 *   deposit  v_COM = (P_gas + M_ej v_s) / M_snr, E_kin = M_ej |v_s|^2 / 2; per
 *            cell with a = w / V_snr and rhat the unit vector from the
 *            remnant to the cell centre (0 at the remnant):
 *            d rho = a M_ej, d p = w ((rho + M_ej / V_snr) v_COM - p) +
 *            a |p_rad| rhat, d E = a (E_sn + E_kin) + v_COM . a |p_rad| rhat.
 * The powers come from the library's own log and exp (same bits as the
 * reference implementation).  In PMP_ACC_FIX64 every term is rounded on the
 * 2^-40 grid and the rounding residues of the mass and of the injected energy
 * go to the host cell (else the first kernel cell in (k, j, i) order), so
 * they land exactly.  The layout needs the rho, momentum and E channels.
 * state (device) is the state the deposit reads (before the step); info
 * (device float64 [4][n], may be NULL) receives V_snr, M_snr, n_H and
 * |p_rad| per remnant.  Errors: PMP_EINVAL (arguments, missing channels),
 * PMP_ERANGE (floor(r_K + 1 - 1/(2 sub)) > ghost width),
 * PMP_EUNSUPPORTED (PMP_ACC_F64R). */
int pmp_deposit_snr(pmp_ctx *ctx, void *buf, const void *state, const pmp_snr *snr,
                    double *info, void *stream);

/* Step 2 (Sec. 2.2; App. A.2).  Adds every ghost cell into the owned cell of
 * the box that holds its periodic image; each owned cell gathers its
 * contributions in one fixed order (source box lo z, y, x, then periodic
 * shift z, y, x), so the fold is deterministic in every accumulator type. */
int pmp_ghost_fold(pmp_ctx *ctx, void *buf, void *stream);

/* Step 4 (Sec. 2.2).  For each sink, re-evaluates its removal k_c over its
 * kernel and writes dm = sum_c eta_c k_c V and dp = sum_c eta_c k_c V p_c/rho_c
 * to the device float64 arrays dm, dpx, dpy, dpz [sinks->n], where
 * eta_c = Kl_c / K_c from the folded buffer and the state before Step 5.
 * Must follow pmp_ghost_fold and precede pmp_apply; needs the same sinks and
 * limits as pmp_deposit. */
int pmp_sink_update(pmp_ctx *ctx, const void *state, const void *buf, const pmp_sinks *sinks,
                    const pmp_limits *limits, double *dm, double *dpx, double *dpy,
                    double *dpz, void *stream);

/* Steps 3 + 5.  In place on the device state: per owned cell, in double
 * precision, the removal K is limited to Kl = min(max(min(K, cap rho),
 * rho - rho_tr), rho - rho_floor) (Sec. 3.1.1) and removes the fraction Kl/rho
 * of the cell; sources are added, the momentum source scaled by the largest
 * lambda in [0, 1] keeping e_int at its floor (Sec. 3.2.1, eq. "lambda").
 * eta (device, may be NULL) receives Kl/K per owned cell (1 where K = 0),
 * float64, in state cell order. */
int pmp_apply(pmp_ctx *ctx, void *state, const void *buf, const pmp_limits *limits,
              double *eta, void *stream);

/* Sink creation (Sec. 3.1.2), after a step, on any box layout that tiles the
 * periodic domain.  A cell becomes a sink when
 *   (1) rho > rho_Tr, the cell's Truelove density (limits: the constant, or
 *       the cell's own with truelove_J > 0);
 *   (2) it is the densest cell among those whose centres lie within r_k
 *       (cells) of its centre, periodic (equal densities ranked by the
 *       global linear cell index, x fastest, the lower index counting as
 *       denser);
 *   (3) no sink lies within r_k of its centre: none of the existing sinks
 *       (existing: positions x, y, z and n are read, may be NULL) is at
 *       squared distance <= r_k^2 from the cell centre or one of its
 *       periodic images, and, where buf is given with the removal channel,
 *       the folded removal K is zero there (no kernel reached it).
 * All tests read the state before any creation, so the result does not
 * depend on the order of the cells.  Each new sink sits at its cell centre
 * (global cell units) with mass (rho - rho_Tr) V and momentum mass p / rho;
 * the cell keeps its velocity and specific energy (rho -> rho_Tr,
 * p -> (p / rho) rho_Tr, E -> (E / rho) rho_Tr), updated in place in the
 * device state of the box that owns it.
 *   out   device float64 [7][max_new]: x, y, z, m, px, py, pz of the new
 *         sinks in increasing global linear cell index;
 *   work  device int64 [2 max_new + 1], caller-owned scratch; work[0]
 *         receives the number of qualifying cells.  When it exceeds max_new,
 *         nothing is created and state and out are left alone (call again
 *         with a larger list).
 * max_new in [0, 65536], r_k in [0, 16] and floor(r_k) at most every axis
 * length of the domain.  Allocates nothing.  Errors: PMP_EINVAL (arguments,
 * limits), PMP_ERANGE (boxes that leave cells of the domain unowned). */
int pmp_sink_create(pmp_ctx *ctx, void *state, const void *buf, const pmp_sinks *existing,
                    double r_k, const pmp_limits *limits, int64_t max_new, double *out,
                    int64_t *work, void *stream);

/* pmp_sink_create for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * passes and results, with the key list and rank accumulators held in a
 * static device array of the library (2 * 65536 + 1 int64, 1 MiB, one copy
 * per GPU, kept until the process ends) instead of a caller's work array.
 *   count  device int64 [1]: receives the number of qualifying cells (as
 *          work[0] of pmp_sink_create); nothing is created when it exceeds
 *          max_new.
 * Other arguments and limits as pmp_sink_create (max_new at most 65536,
 * else PMP_EINVAL).  Calls no hipMalloc, hipFree or allocating routine.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (on different streams, or from several threads) race and must be
 * serialised by the caller. */
int pmp_sink_create_noalloc(pmp_ctx *ctx, void *state, const void *buf,
                            const pmp_sinks *existing, double r_k, const pmp_limits *limits,
                            int64_t max_new, double *out, int64_t *count, void *stream);

/* One whole step: deposit, fold, sink update (if sinks), apply.  sink_out
 * (device) is four float64 arrays [4][sinks->n] (dm, dpx, dpy, dpz) or NULL
 * without sinks. */
int pmp_step(pmp_ctx *ctx, void *state, void *buf, const pmp_cic *cic, const pmp_sn *sn,
             const pmp_sinks *sinks, const pmp_limits *limits, double *sink_out, void *stream);

/* The per-box launch form of pmp_step, kept as the baseline the batched
 * launches are measured against: every kernel is launched once per box over
 * that box's cells and particles only (zero fill, direct CIC and supernova
 * atomics, fold, apply), as a code without batching would.  Same results as
 * pmp_step with deposit_path 0.  cic_off and sn_off are host copies of the
 * kinds' box_off arrays (NULL when the kind is absent).  No sinks. */
int pmp_step_per_box(pmp_ctx *ctx, void *state, void *buf, const pmp_cic *cic,
                     const pmp_sn *sn, const pmp_limits *limits, const int64_t *cic_off,
                     const int64_t *sn_off, void *stream);

/* Capture nsteps consecutive pmp_step calls into one HIP graph kept by the
 * context (replacing any previous one).  The device pointers are baked into
 * the graph and must stay valid until the graph is rebuilt or the context is
 * destroyed.  Enqueues nothing on stream; uses it only to order the capture. */
int pmp_graph_build(pmp_ctx *ctx, int nsteps, void *state, void *buf, const pmp_cic *cic,
                    const pmp_sn *sn, const pmp_sinks *sinks, const pmp_limits *limits,
                    double *sink_out, void *stream);
/* Replay the captured graph on stream. */
int pmp_graph_launch(pmp_ctx *ctx, void *stream);

/* Synchronise the context's device, copy the status to *out (host), and
 * clear it if reset != 0. */
int pmp_get_status(pmp_ctx *ctx, pmp_status *out, int reset);

int pmp_get_tuning(const pmp_ctx *ctx, pmp_tuning *out);
int pmp_set_tuning(pmp_ctx *ctx, const pmp_tuning *t);

/* Autotuner: times whole steps (2 warm-up, 5 timed, HIP events) for each
 * candidate tuning on the given inputs and keeps the fastest.  Stage 1: the
 * direct (global atomic) path and the binned (LDS-privatised) path with a set
 * of tile shapes and workgroup sizes, with and without the fused apply (steps
 * without sinks).  Stage 2, if the binned path won: the split thresholds
 * chunk_cic / chunk_sn, the persistent tile grid cap and (with supernovae)
 * count_lanes, each around the winner so far.  The steps run on a scratch
 * copy of the state (the
 * caller's state is left as it was; the buffer and sink_out are overwritten).
 * Synchronises the stream; allocates and frees the scratch copy.  best_ms
 * (host, may be NULL) receives the winning step time. */
int pmp_autotune(pmp_ctx *ctx, void *state, void *buf, const pmp_cic *cic, const pmp_sn *sn,
                 const pmp_sinks *sinks, const pmp_limits *limits, double *sink_out,
                 void *stream, double *best_ms);

/* Phase profiler (the per-routine timers of Sec. 4.6, on the GPU): after
 * pmp_profile_begin, every kernel the context launches outside graph capture
 * is bracketed by HIP events on its stream, for up to max_launches launches
 * per phase.  pmp_profile_end synchronises, writes the summed kernel time in
 * milliseconds and the launch count of each phase to the host arrays ms and
 * launches [PMP_NPHASE] (either may be NULL) and stops profiling. */
#define PMP_NPHASE 10
#define PMP_PHASE_ZERO 0          /* direct path: zero fill of the buffer */
#define PMP_PHASE_CIC 1           /* direct path: CIC atomics */
#define PMP_PHASE_SN 2            /* direct path: supernova atomics */
#define PMP_PHASE_SINK_DEPOSIT 3
#define PMP_PHASE_FOLD 4          /* ghost fold; in a fused step (fuse_apply 1), the
                                     shell cells' fold + limiter + apply (none
                                     with owner tiles) */
#define PMP_PHASE_SINK_UPDATE 5
#define PMP_PHASE_APPLY 6
#define PMP_PHASE_BIN 7           /* binned path: two-level sort of (particle, tile)
                                     pairs, supernova member counts and shares,
                                     chunk table of split tiles (several launches) */
#define PMP_PHASE_TILE 8          /* binned path: the tile kernel alone (LDS
                                     accumulation and store; in a fused step also
                                     the interior cells' limiter + apply) */
#define PMP_PHASE_SNR 9           /* supernova remnants (pmp_deposit_snr) */
int pmp_profile_begin(pmp_ctx *ctx, int max_launches);
int pmp_profile_end(pmp_ctx *ctx, double *ms, int64_t *launches);

/* Bandwidth calibration: copy bytes from device src to device dst with a
 * plain streaming kernel (16-byte loads and stores). */
int pmp_stream_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Bandwidth calibration variants (measurement support): variant 0 is
 * pmp_stream_copy; 1 moves groups of 1024 16-byte vectors per 256-thread
 * workgroup, four coalesced loads per thread before nontemporal stores
 * (bytes a multiple of 16384, 16-byte aligned pointers); 2 is the runtime's
 * device-to-device hipMemcpyAsync. */
int pmp_copy_bench(void *dst, const void *src, size_t bytes, int variant, void *stream);

/* Global-atomic throughput microbenchmark (measurement support: the peak the
 * atomic deposits are measured against; no part of the method).  Enqueues
 * one kernel that performs n_ops atomic adds of 1 into the device array dst
 * of `slots` elements (a power of two): type 0 int64, 1 float, 2 double;
 * pattern 0 op i -> element i mod slots (each wavefront's 64 ops on
 * consecutive elements), 1 a multiplicative hash of i mod slots (scattered
 * addresses), 2 element 0 for every op (all contend for one address).  The
 * caller times it (events on stream).  PMP_EINVAL on bad arguments. */
int pmp_atomic_bench(void *dst, int64_t slots, int type, int pattern, int64_t n_ops,
                     void *stream);

const char *pmp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
