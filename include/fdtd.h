/*
 * fdtd.h -- C-ABI of libfdtd, the MI355X (gfx950) hot path of a
 * differentiable FDTD solver (TorchFDTD, arXiv 2609.30039).
 *
 * The library advances one or more independent 3-D Yee domains
 *   E^{n+1} = E^n + S eps^-1 C^-(H^{n+1/2}) + s^{n+1},
 *   H^{n+3/2} = H^{n+1/2} - S C^+(E^{n+1})            (Section 2.1, Eq. 1)
 * with convolutional PML memories in absorbing faces and PEC outer walls
 * (Section 2.2), per-node real or diagonal permittivity and a dispersive
 * box of 1 to 16 Lorentz or Drude poles integrated by the trapezoidal ADE
 * (Section 2.3), soft electric sources and point / plane-spectrum monitors
 * (Section 2.4), and runs the discrete adjoint of that step (Section 3.1,
 * Eq. 3) with accumulation of dJ/deps.  Checkpoint slots serve the binomial replay of Section 3.2.
 *
 * Conventions shared by every call:
 *   - unit mesh (h = 1), c = 1: dt = S, frequencies are given as omega*dt;
 *   - field arrays are [nz][ny][nx], x fastest; boxes are half-open [lo, hi)
 *     in cell indices (i, j, k);
 *   - Ex[k][j][i] sits at (i+1/2, j, k), Ey at (i, j+1/2, k), Ez at
 *     (i, j, k+1/2), Hx at (i, j+1/2, k+1/2), Hy at (i+1/2, j, k+1/2),
 *     Hz at (i+1/2, j+1/2, k); E at index N_a is a zero ghost, H at -1 too;
 *     E tangential to a low face (index 0 along another axis) is held at 0;
 *   - forward step t (t = 0, 1, ...) maps u^t -> u^{t+1}; E^{t+1} is sampled
 *     at time (t+1) dt and H^{t+3/2} at (t+3/2) dt; plane spectra are
 *     X(w) = sum_n x^n exp(-i w t_n) with that half-step offset kept.
 *
 * Ownership: the handle owns all device memory (hipMalloc); every host array
 * passed in is copied during the call and never retained.  All device work is
 * enqueued on the stream given at create; only calls returning host data
 * synchronise (that stream only).  A handle is not thread-safe; distinct
 * handles are independent.
 *
 * Errors: every call returns an int status, never aborts or throws.
 *   FDTD_E_INVALID, FDTD_E_STATE, FDTD_E_RANGE leave the handle usable;
 *   FDTD_E_DEVICE (a HIP error) poisons it: every later call except
 *   fdtd_destroy and fdtd_last_error returns FDTD_E_DEVICE.
 */
#ifndef FDTD_H_
#define FDTD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FDTD_OK = 0,
    FDTD_E_INVALID = -1,   /* bad argument or descriptor */
    FDTD_E_UNSTABLE = -2,  /* CFL eta > 0.99 (Eq. 2), non-finite eps or eps below 1
                              (the step bound of Eq. 2 is the vacuum one; Section 2.3
                              admits eigenvalues >= 1), anisotropic eps inside an
                              absorbing face violating the principal-axis rule of
                              Section 2.3, a pole with omega_dt <= 0, gamma_dt < 0, a
                              negative Lorentz strength, a Lorentz omega_0 dt >= 2
                              (its recursion then has a root outside the unit disc)
                              or a non-finite parameter */
    FDTD_E_NOMEM = -3,     /* device memory request above budget, refused before allocating */
    FDTD_E_DEVICE = -4,    /* HIP runtime error; handle poisoned */
    FDTD_E_STATE = -5,     /* wrong step index for an adjoint step, empty or corrupt slot */
    FDTD_E_RANGE = -6      /* index out of range (domain, component, slot, monitor, buffer size) */
};

enum { FDTD_F32 = 0, FDTD_F64 = 1, FDTD_BF16 = 2 };
/* permittivity kinds.  ISO: one value per cell (each E edge takes its
   cell's value); DIAG: three values per cell, one per E component; TENSOR
   (Section 2.3): a symmetric tensor at each grid node (the corner where the
   edges Ex, Ey, Ez of index (i,j,k) start), six values xx, yy, zz, xy, xz, yz,
   applied to the curl through the node assembly S = (1/8) sum over the eight
   octants of R^T eps^-1 R (an edge takes half of each end node's diagonal
   entry and a quarter of each off-diagonal entry times the sum of the two
   edges of that axis meeting it there).  Every node's tensor must have all
   eigenvalues >= 1; inside an absorbing face (node index along the normal in
   the slab) the normal must be a principal axis (zero off-diagonal entries
   with it) whose eigenvalue is the largest or the smallest: else
   FDTD_E_UNSTABLE, checked node by node.  On a periodic axis the node
   tensors repeat past the seam (the node past the last one is the first)
   and the edges past it take the Bloch factor.  TENSOR domains take no
   dispersive box, no reversible mode and no fused kernels (FDTD_E_INVALID),
   and one scratch curl of 3 field arrays each.  Their
   gradient (Section 3.1 through the assembly, which is its own transpose)
   is dJ/deps of the six stored entries of each node tensor in the gradient
   box, an off-diagonal entry counting as one parameter for both of its
   matrix entries. */
enum { FDTD_EPS_ISO = 0, FDTD_EPS_DIAG = 1, FDTD_EPS_TENSOR = 2 };
enum { FDTD_SRC_POINT = 0, FDTD_SRC_PLANE_Z = 1 };
enum { FDTD_MON_PROBE = 0, FDTD_MON_FLUX_Z = 1, FDTD_MON_PATCH_Z = 2 };
/* field components for get/set: 0..5 = Ex..Hz of the forward state,
   6..11 = the adjoint (cotangent) Ex..Hz */
enum { FDTD_EX = 0, FDTD_EY, FDTD_EZ, FDTD_HX, FDTD_HY, FDTD_HZ, FDTD_ADJ = 6 };
/* step_forward flags */
enum { FDTD_RECORD = 1u, FDTD_REPLAY = 2u };
/* monitor ops */
enum { FDTD_MON_GET = 0, FDTD_MON_FLUX = 1, FDTD_MON_SET_COTANGENT = 2, FDTD_MON_RESET = 3 };
/* kernel family.  AUTO and SPLIT: one E launch and one H launch per step,
   updating the state in place; FUSED: one pass per step over tiles, writing
   the other state set; ONEPASS: the split kernels on the blocks that meet an
   absorbing slab, a wall or a dispersive box, and one z-marching pass that
   advances E and H together on every other block (interior blocks), writing
   the other state set.  Results are bitwise identical; the speed depends on
   the geometry (the package's autotuner picks per workload).  ONEPASS takes
   the split launch shapes (tile_rows 4 or 8) and no reversible mode. */
enum { FDTD_KERNEL_AUTO = 0, FDTD_KERNEL_SPLIT = 1, FDTD_KERNEL_FUSED = 2, FDTD_KERNEL_ONEPASS = 3 };

#define FDTD_MAX_SOURCES 4
#define FDTD_MAX_MONITORS 8
#define FDTD_MAX_POLES 16

/* One pole of a dispersive medium (Section 2.3: up to sixteen Drude or
   Lorentz poles, trapezoidal auxiliary differential equation).  A Lorentz
   pole has strength delta_eps, resonance omega_dt = omega_0 dt and damping
   gamma_dt; a Drude pole has plasma frequency omega_dt = omega_p dt and
   damping gamma_dt (delta_eps unused): the Lorentz recursion with omega_0 -> 0
   and delta_eps omega_0^2 -> omega_p^2.  fdtd_create returns FDTD_E_INVALID
   for n_poles outside 1..FDTD_MAX_POLES or an unknown kind, and
   FDTD_E_UNSTABLE for omega_dt <= 0, gamma_dt < 0, a negative Lorentz
   delta_eps, a Lorentz omega_dt >= 2 or a non-finite parameter.  Each
   pole's two history arrays cost 6 words per box cell. */
enum { FDTD_POLE_LORENTZ = 0, FDTD_POLE_DRUDE = 1 };

typedef struct {
    int32_t kind;                  /* FDTD_POLE_LORENTZ | FDTD_POLE_DRUDE */
    double delta_eps;              /* Lorentz pole strength */
    double omega_dt;               /* Lorentz omega_0 dt | Drude omega_p dt, > 0 */
    double gamma_dt;               /* damping gamma * dt (full rate), >= 0 */
} fdtd_pole_desc;

typedef struct {
    int32_t lo[3], hi[3];          /* cell box; eps_inf of each cell is its permittivity */
    int32_t n_poles;               /* 1..FDTD_MAX_POLES; the poles' polarisation currents add */
    fdtd_pole_desc poles[FDTD_MAX_POLES];
} fdtd_lorentz_desc;

typedef struct {
    int32_t kind;                  /* FDTD_SRC_POINT | FDTD_SRC_PLANE_Z */
    int32_t comp;                  /* 0..2: Ex, Ey, Ez */
    int32_t pos[3];                /* point (i,j,k); plane uses pos[2] = k, whole plane */
    const double *waveform;        /* host; waveform[t] is added at forward step t */
    int32_t n_waveform;            /* steps beyond the end add nothing */
} fdtd_source_desc;

typedef struct {
    int32_t kind;                  /* FDTD_MON_PROBE | FDTD_MON_FLUX_Z | FDTD_MON_PATCH_Z */
    int32_t comp;                  /* probe / patch component 0..5 */
    int32_t pos[3];                /* probe (i,j,k); planes use pos[2] = k */
    int32_t rect[4];               /* plane rectangle i0, i1, j0, j1 */
    const double *omega_dt;        /* host; n_freq frequencies omega*dt */
    int32_t n_freq;
} fdtd_monitor_desc;

typedef struct {
    int32_t n[3];                  /* nx, ny, nz cells, absorbing cells included */
    double courant;                /* S = c dt / h; S*sqrt(3) must be <= 0.99 */
    int32_t pml[6];                /* absorbing cells at xlo, xhi, ylo, yhi, zlo, zhi */
    double pml_m, pml_kappa_max, pml_sigma_max, pml_alpha_max;   /* grading */
    int32_t eps_kind;              /* FDTD_EPS_ISO | FDTD_EPS_DIAG | FDTD_EPS_TENSOR */
    int32_t eps_lo[3], eps_hi[3];  /* box where eps is given (TENSOR: a box of nodes) */
    const double *eps;             /* host [ncomp][bz][by][bx], ncomp 1 (ISO), 3 (DIAG) or 6 (TENSOR:
                                      xx, yy, zz, xy, xz, yz); values (eigenvalues) >= 1 */
    double eps_bg;                 /* permittivity outside the box, >= 1 */
    int32_t n_lorentz;             /* 0 or 1 */
    fdtd_lorentz_desc lorentz;
    int32_t n_sources;             /* <= FDTD_MAX_SOURCES */
    fdtd_source_desc sources[FDTD_MAX_SOURCES];
    int32_t n_monitors;            /* <= FDTD_MAX_MONITORS */
    fdtd_monitor_desc monitors[FDTD_MAX_MONITORS];
    int32_t grad;                  /* 1: this domain takes part in the adjoint */
    int32_t grad_lo[3], grad_hi[3];/* box where dJ/deps accumulates */
    int32_t periodic[3];           /* 1: Bloch-periodic axis (Section 2.2): no PEC wall, and the node past
                                      the last one is the first one times bloch_sign.  x and y only, with no
                                      absorbing cells on that axis, split kernels; with a gradient (the
                                      adjoint scatters across the seam with the same real factor, its own
                                      conjugate) no reversible mode: else FDTD_E_INVALID */
    int32_t bloch_sign[3];         /* real Bloch factor exp(i k L) of a periodic axis: +1 (periodic) or -1
                                      (anti-periodic); ignored on other axes */
} fdtd_domain_desc;

typedef struct {
    int32_t dtype;                 /* FDTD_F32 | FDTD_F64: field and coefficient arithmetic */
    int32_t n_ckpt;                /* checkpoint slots */
    int32_t ckpt_storage;          /* FDTD_F32 (= dtype width) | FDTD_BF16 (per-array scale) */
    int32_t ckpt_checksum;         /* 1: store a checksum per slot, verify on restore */
    int32_t max_steps;             /* length of probe traces and adjoint seed range */
    int32_t kernel;                /* FDTD_KERNEL_* */
    int32_t dft_block;             /* time samples buffered before a DFT flush (0: default) */
    int32_t graph_chunk;           /* steps per captured hipGraph (0: no graph) */
    int32_t tile_rows;             /* fused kernels: rows per wave, 2 | 4 | 8 (0: 2); split kernels:
                                      rows per 256-thread block, 4 (64 columns; 0 = 4) or 8 (32) */
    int32_t tile_kz;               /* z planes per block (0: default) */
    void *stream;                  /* hipStream_t; NULL = default stream */
    double mem_budget_bytes;       /* refuse with FDTD_E_NOMEM above this (0: device free memory) */
    int32_t reversible;            /* 1: reversible mode (see fdtd_step_reverse); admissible only when
                                      every domain with a gradient has no dispersive box and its gradient
                                      box lies between the absorbing slabs, one cell clear of a low slab
                                      (else FDTD_E_INVALID); needs max_steps >= 1 and keeps
                                      (max_steps + 1) x 4 x (the box's face areas) interface values */
    /* optional device allocator for the handle's one pool (e.g. the caching
       allocator of the caller's framework, so that its memory accounting sees
       the pool): alloc(ctx, bytes) returns device memory or NULL (then
       FDTD_E_NOMEM), release(ctx, p) takes it back at fdtd_destroy; both NULL:
       hipMalloc / hipFree.  Called on the handle's stream's device. */
    void *(*alloc)(void *ctx, size_t bytes);
    void (*release)(void *ctx, void *p);
    void *alloc_ctx;
} fdtd_options;

typedef struct fdtd_s *fdtd_t;

/* Create a handle advancing n_domains independent domains together
   (n_domains > 1: one launch covers all of them through a tile table).
   Validates the CFL bound (Eq. 2), eps positivity and the absorbing-face
   tensor rule, estimates device memory and refuses above budget, then
   allocates and uploads.  State starts at zero with forward step 0. */
int fdtd_create(const fdtd_domain_desc *domains, int32_t n_domains, const fdtd_options *opt, fdtd_t *out);

/* Release all device memory of the handle (after draining its stream). */
int fdtd_destroy(fdtd_t h);

/* Advance every domain n_steps forward steps (Eq. 1 with absorbers,
   dispersion, sources).  FDTD_RECORD accumulates monitors; FDTD_REPLAY
   leaves them untouched (checkpoint replay must not double count). */
int fdtd_step_forward(fdtd_t h, int32_t n_steps, uint32_t flags);

/* Start the reverse sweep at m = n_total: zero the cotangent state and the
   gradient accumulators and inject dJ/du^{n_total} from the cotangents set
   with FDTD_MON_SET_COTANGENT. */
int fdtd_adjoint_begin(fdtd_t h, int32_t n_total);

/* n_steps adjoint steps of Eq. 3.  Each step m -> m-1 requires the forward
   state u^{m-1} (forward step index == m-1, else FDTD_E_STATE; so n_steps
   is 1 unless the caller replays in between), applies the transposes of
   Section 3.1 in reverse order, accumulates dJ/deps from u^{m-1} inside the
   gradient box, and adds dJ/du^{m-1}. */
int fdtd_step_adjoint(fdtd_t h, int32_t n_steps);

/* Reversible mode (Section 3.2, the absorbing-face variant).  The box R of
   each domain with a gradient, between its absorbing slabs, is lossless and
   nondispersive, so Eq. 1 can be stepped backward there:
     H^{m-1/2} = H^{m+1/2} + S C^+(E^m),  E^{m-1} = (E^m - s^m) - S eps^-1 C^-(H^{m-1/2}).
   Every forward step records, on the device, the fields just outside R that
   these backward steps read (H on R's low faces, E on its high faces), so the
   interior reconstruction needs nothing from the absorbers.  fdtd_step_reverse
   takes n_steps such backward steps: the forward step index goes from m to
   m - n_steps and the forward state inside R becomes u^{m-n_steps} up to
   round-off; outside R it is left undefined (the adjoint reads the forward
   state only inside the gradient box).  The reverse sweep then alternates
   fdtd_step_reverse(h, 1) and fdtd_step_adjoint(h, 1) without checkpoints.
   Forward steps are launched one by one in this mode (no captured chunks).
   FDTD_E_STATE without reversible mode, or when the interface of a step was
   not recorded since the last reset, set_field or set_eps. */
int fdtd_step_reverse(fdtd_t h, int32_t n_steps);

/* Copy the full forward state u^n (fields, absorber memories, Lorentz
   history) and n into slot (Section 3.2).  BF16 storage scales each array by
   its max-abs value and rounds to nearest even; an array whose max-abs value
   is below the smallest normal float is stored as zeros.  FP32/FP64 slots
   swap buffers with the working set, so a save copies nothing. */
int fdtd_checkpoint_save(fdtd_t h, int32_t slot);

/* Make the slot's state current: u := slot, forward step := slot's n.
   FDTD_E_STATE for an empty slot or (with checksums) a mismatch. */
int fdtd_checkpoint_restore(fdtd_t h, int32_t slot);

/* Plane-spectrum monitor access for domain `domain`, monitor `monitor`:
   GET            host_buf <- complex128 [n_freq][ncomp][j1-j0][i1-i0]
                  (flux: ncomp 4 = Ex, Ey, Hx, Hy with H averaged over planes
                  k and k-1; patch: ncomp 1); probes: double [n_recorded].
   FLUX           host_buf <- double [n_freq], Re sum (Ex Hy* - Ey Hx*).
   SET_COTANGENT  host_buf -> same layout as GET: dJ/dRe X + i dJ/dIm X
                  (probes: dJ/dsample, double [max_steps]).
   RESET          zero the spectra / trace (host_buf unused). */
int fdtd_monitor_dft(fdtd_t h, int32_t domain, int32_t monitor, int32_t op, void *host_buf, size_t bytes);

/* Copy one component (FDTD_EX..FDTD_HZ, + FDTD_ADJ for the cotangent) of one
   domain to/from a host array of nx*ny*nz elements of the handle's dtype. */
int fdtd_get_field(fdtd_t h, int32_t domain, int32_t comp, void *host_buf, size_t bytes);
int fdtd_set_field(fdtd_t h, int32_t domain, int32_t comp, const void *host_buf, size_t bytes);

/* dJ/deps over the gradient box: double [ncomp][gz][gy][gx], ncomp 1 (ISO),
   3 (DIAG: per E component) or 6 (TENSOR: xx, yy, zz, xy, xz, yz at the
   nodes).  FDTD_E_RANGE if bytes is below ncomp * cells * 8. */
int fdtd_get_grad(fdtd_t h, int32_t domain, double *host_buf, size_t bytes);

/* Replace the permittivity of a domain (same layout as the descriptor). */
int fdtd_set_eps(fdtd_t h, int32_t domain, const double *eps, size_t bytes);

/* Zero the forward state and monitors, forward step := 0. */
int fdtd_reset(fdtd_t h);

/* Current forward step n and adjoint index m (-1 before fdtd_adjoint_begin). */
int fdtd_get_step(fdtd_t h, int32_t *fwd_n, int32_t *adj_m);

/* The probe trace of monitor `probe` (a FDTD_MON_PROBE) of domain `domain`:
   its first n samples (n <= max_steps), sample t taken after forward step t
   + 1, as FDTD_MON_GET returns them. */
int fdtd_probe_trace(fdtd_t h, int32_t domain, int32_t probe, double *host_buf, int32_t n);

/* Watchdog: the sum of squares of domain `domain`'s six fields in the
   current state, reduced on the device in FP64 in a fixed order, into
   *energy.  Returns FDTD_E_UNSTABLE (after writing the sum) when it is not
   finite: a NaN or an infinity somewhere in the fields, from a diverged run
   or non-finite input.  The FDTD_MON_FLUX op of fdtd_monitor_dft returns
   FDTD_E_UNSTABLE the same way when a flux value is not finite. */
int fdtd_field_energy(fdtd_t h, int32_t domain, double *energy);

/* Bytes of device memory held by the handle. */
int fdtd_get_memory(fdtd_t h, double *bytes);

/* Timing of the stepping kernels with HIP events recorded on the handle's
   stream around every forward/adjoint stepping launch:
   op 1 = enable and clear, 0 = disable, 2 = synchronise and return the
   summed kernel time (ms) and the number of timed launches since enable. */
int fdtd_kernel_timing(fdtd_t h, int32_t op, double *total_ms, int64_t *launches);

/* Bandwidth calibration: copy `bytes` (a multiple of 4) between two device
   buffers allocated for the call, `reps` times, on the default stream, and
   return the mean kernel time per copy in ms (HIP events).  Used to scale
   hardware byte counters against a plain copy of known size. */
int fdtd_copy_probe(size_t bytes, int32_t reps, double *ms_per_copy);

/* Failure injection for tests of checksum validation: overwrite 32-bit word
   `word` of checkpoint slot `slot` with `value`. */
int fdtd_checkpoint_corrupt(fdtd_t h, int32_t slot, size_t word, uint32_t value);

/* Poynting flux through a z-plane from its spectra (Section 2.4), reduced
   on the device: flux[f] = Re sum_p (Ex Hy* - Ey Hx*) over the n_pts plane
   points, for spectra laid out as fdtd_monitor_dft GET returns those of a
   flux monitor: complex128 [n_freq][4][n_pts], components Ex, Ey, Hx, Hy (H
   already averaged over planes k and k-1).  `spectra` (read) and `flux`
   (double [n_freq], written) are device pointers owned by the caller.  The
   sums run in a fixed order with no atomics, so the result depends only on
   the inputs.  Work is enqueued on `stream` (a hipStream_t, NULL = the
   default stream); the call does not synchronise unless it allocates.
   Partial sums need FDTD_FLUX_WORKSPACE_BYTES(n_freq, n_pts) bytes of
   device memory: pass a caller-owned `workspace` of `workspace_bytes` >=
   that, or NULL, and the call then takes them with hipMalloc and frees them
   after synchronising the stream.  Returns FDTD_E_INVALID for a null
   spectra/flux pointer, n_freq < 1 or n_pts < 1, FDTD_E_RANGE for a
   workspace below the size, FDTD_E_NOMEM if the allocation fails and
   FDTD_E_DEVICE for a launch error; fdtd_last_error(NULL) holds the message.
   fdtd_monitor_dft FLUX uses the same reduction. */
#define FDTD_FLUX_POINTS_PER_BLOCK 4096
#define FDTD_FLUX_MAX_BLOCKS 256
#define FDTD_FLUX_BLOCKS(n_pts) \
    ((n_pts) >= (int64_t)FDTD_FLUX_POINTS_PER_BLOCK * FDTD_FLUX_MAX_BLOCKS ? FDTD_FLUX_MAX_BLOCKS \
     : (int)(((n_pts) + FDTD_FLUX_POINTS_PER_BLOCK - 1) / FDTD_FLUX_POINTS_PER_BLOCK))
#define FDTD_FLUX_WORKSPACE_BYTES(n_freq, n_pts) ((size_t)(n_freq) * (size_t)FDTD_FLUX_BLOCKS(n_pts) * 8u)
int fdtd_flux_reduce(const double *spectra, int32_t n_freq, int64_t n_pts, double *flux, void *workspace,
                     size_t workspace_bytes, void *stream);

/* fdtd_flux_reduce for callers that cannot allocate device memory: code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc.  Same arguments and results as fdtd_flux_reduce (bitwise), but
   the partial sums live in a file-scope device array of
   FDTD_FLUX_SCRATCH_BYTES that every GPU the library runs on holds until the
   process ends, so the call allocates nothing and never synchronises.  It
   returns FDTD_E_RANGE when FDTD_FLUX_WORKSPACE_BYTES(n_freq, n_pts) exceeds
   that size (n_freq * blocks <= 8192), FDTD_E_INVALID for a null pointer,
   n_freq < 1 or n_pts < 1, FDTD_E_DEVICE for a HIP error.  All calls on one
   GPU share its array: calls that overlap on one GPU (other streams or
   threads) race and must be serialised by the caller. */
#define FDTD_FLUX_SCRATCH_BYTES 65536
int fdtd_flux_reduce_noalloc(const double *spectra, int32_t n_freq, int64_t n_pts, double *flux, void *stream);

/* Message of the last failing call on this handle (or, when h is NULL, of
   the last failing create or handle-free call); valid until the next call. */
const char *fdtd_last_error(fdtd_t h);

/* ---------------------------------------------------------------------------
   Host-streamed causal slabs (Section 4.2): one domain whose state lives in
   host memory, advanced slab by slab in a device workspace of a few slabs'
   planes, for domains beyond the device's memory.

   The domain is cut along z (the slowest axis of the field layout, so every
   host<->device transfer is one contiguous copy per state array) into
   ceil(nz / slab_planes) slabs whose cores split nz as evenly as possible.
   One pass advances the domain by K = steps_per_pass steps: each slab in turn
   is copied from host bank A (time t) over its core and K + 1 halo planes per
   cut side, stepped K times with the resident kernels, and its core is copied
   to host bank B (time t + K); the banks then swap.  A cut face acts as a
   wall, and a wrong value moves at most one plane per step, so every core
   plane equals the resident solution bit for bit (same kernels, same
   operands).  Device memory scales with (W + 2K + 2) nx ny, host memory with
   the two banks (2 x the resident state) plus eps^-1 in the field type.

   Supported: everything the resident forward path supports on the domain
   (scalar, diagonal or tensor eps, a dispersive box, absorbing faces on every
   side, periodic x/y, sources, probe and plane monitors), and with grad set
   the reverse sweep (fdtd_stream_reverse) over the same slabs.  With a
   gradient the host keeps, by default, one forward bank per pass boundary
   (bank j holds time j K; ceil(max_steps / K) + 1 banks), or with
   host_banks = B >= 4 only B forward banks: the state at time t, time 0 and
   the snapshots of a binomial schedule over passes (Section 3.2's
   checkpointing applied to the block checkpoints); the reverse sweep then
   regenerates the other block starts by streamed forward passes from the
   nearest snapshot.  Two cotangent banks besides, and passes are exactly K
   steps except the last one.  An absorbing z face
   must lie wholly inside or wholly outside each slab's extent: a slab that
   would cut one is refused (FDTD_E_INVALID; raise slab_planes).  Monitors
   belong to the slab whose core holds their plane; their spectra and probe
   traces accumulate on the device across slabs and passes.  The device
   workspace and monitor accumulators are admitted against mem_budget_bytes
   (0: the device's free memory) and the host banks against
   host_budget_bytes (0: no limit besides the pinned allocation itself), both
   before anything is allocated (FDTD_E_NOMEM). */
typedef struct {
    int32_t dtype;                 /* FDTD_F32 | FDTD_F64 */
    int32_t slab_planes;           /* W: most core planes of one slab, >= 1 */
    int32_t steps_per_pass;        /* K: steps a slab advances per visit, >= 1 (halo K + 1 per cut side) */
    int32_t max_steps;             /* probe trace length */
    int32_t tile_rows, tile_kz;    /* split-kernel launch shape of the slab steps (0: defaults) */
    void *stream;                  /* hipStream_t; NULL = default stream */
    double mem_budget_bytes;       /* device budget (0: free memory) */
    double host_budget_bytes;      /* pinned host budget for the banks and eps^-1 (0: unchecked) */
    int32_t overlap;               /* 1: two workspaces on two streams, so that one slab's transfers run
                                      beside the other slab's steps (twice the device workspace) */
    int32_t local_slots;           /* reverse sweep: forward states a slab keeps on the device while it
                                      reverses a block (binomial schedule); 0 or >= K: every state */
    int32_t host_banks;            /* with a gradient: forward banks on the host, 0 (one per pass
                                      boundary) or >= 4 (binomial over passes); else FDTD_E_INVALID */
} fdtd_stream_options;

typedef struct {
    int32_t n_slabs;
    int32_t halo;                  /* planes per cut side */
    int32_t max_extent;            /* planes of the largest slab, halos included */
    int32_t step;                  /* steps advanced so far */
    double device_bytes;           /* workspace + monitor accumulators */
    double host_bytes;             /* pinned: two state banks + eps^-1 */
    double resident_bytes;         /* what the resident handle of the same domain would allocate */
    int32_t materials_resident;    /* 1: eps^-1 is kept on the device (the budget held it beside the
                                      workspaces); 0: each visit uploads its planes from pinned memory */
    int32_t replay_passes;         /* streamed forward passes the last reverse sweep ran to regenerate
                                      block starts (0 with one bank per pass boundary) */
} fdtd_stream_info;

typedef struct fdtd_stream_s *fdtd_stream_t;

/* Validates the domain as fdtd_create would (same error codes), plans and
   admits the slabs, allocates, and zeroes the state (time 0).  The
   descriptor's arrays are copied; the caller may free them afterwards. */
int fdtd_stream_create(const fdtd_domain_desc *domain, const fdtd_stream_options *opt, fdtd_stream_t *out);
int fdtd_stream_destroy(fdtd_stream_t h);
/* Advances n_steps (passes of steps_per_pass steps, the last one shorter). */
int fdtd_stream_step(fdtd_stream_t h, int32_t n_steps);
/* Field comp 0..5 (Ex..Hz) of the current state, [nz][ny][nx] of the dtype. */
int fdtd_stream_get_field(fdtd_stream_t h, int32_t comp, void *host_buf, size_t bytes);
/* op FDTD_MON_GET: spectra (layout of fdtd_monitor_dft) or the probe trace;
   FDTD_MON_FLUX: flux per frequency of a flux monitor, reduced on the device. */
int fdtd_stream_monitor(fdtd_stream_t h, int32_t monitor, int32_t op, double *host_buf, size_t bytes);
/* Back to time 0: state and monitors zeroed. */
int fdtd_stream_reset(fdtd_stream_t h);
/* Cotangent dJ/d(observation) of monitor `monitor` (layout of
   FDTD_MON_SET_COTANGENT), kept until replaced; FDTD_E_STATE without grad. */
int fdtd_stream_set_cotangent(fdtd_stream_t h, int32_t monitor, const double *host_buf, size_t bytes);
/* Reverse sweep (Eq. 3, Section 3.1) over the forward steps done since the
   reset, block by block from the last: each slab replays its block from the
   block's starting bank with every state kept in the workspace, runs the
   transposed steps from the cotangent state at the block's end (loaded over
   its extent, seeded by every monitor whose plane the extent holds), and
   returns its core's cotangent state and dJ/deps.  The gradient equals the
   resident sweep's up to the order of its FP64 sums.  FDTD_E_STATE without
   grad or without forward steps. */
int fdtd_stream_reverse(fdtd_stream_t h);
/* dJ/deps of the last reverse sweep over the gradient box, double
   [ncomp][gz][gy][gx] as fdtd_get_grad; FDTD_E_STATE if the forward has
   moved since or no sweep ran. */
int fdtd_stream_get_grad(fdtd_stream_t h, double *host_buf, size_t bytes);
int fdtd_stream_get_info(fdtd_stream_t h, fdtd_stream_info *out);
/* Message of the last failing call on h (NULL: of a failing create). */
const char *fdtd_stream_last_error(fdtd_stream_t h);

#ifdef __cplusplus
}
#endif
#endif /* FDTD_H_ */
