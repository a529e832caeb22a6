/*
 * esp.h -- long-range (k-space) electrostatics by Ewald summation with
 * prolate spheroidal wave functions (ESP), on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Methods, "A general Ewald split", eq. task): N point charges q_i at
 * r_i in a periodic box (cubic of side L, orthorhombic with sides L, Ly, Lz,
 * or a triclinic cell with tilts xy, xz, yz), sum q_i = 0, kernel 1/(4 pi r) (nondimensionalised; multiply by the
 * Coulomb constant of your unit system).
 * The library evaluates the spectral (smooth, long-range) part of the split
 * 1/(4 pi r) = S(r) + L(r) (eq. kernelsplitting) with the PSWF splitting kernel
 * (eq. pswf), using the five-step method (eqs. spread, FFT, diagonal scaling,
 * IFFT, interp) with the influence function of eq. pk and analytic-derivative
 * forces. For each particle it returns
 *     phi_i = u~^s_i - q_i S(0)                  (self-corrected potential),
 *     F_i   = -q_i grad u~^s(r_i)                (AD forces),
 *     E     = (1/2) sum_i q_i phi_i              (computed in k-space, FP64).
 * Adding the local part u^l_i (eq. localpart, kernel L(r) for r < rc, zero
 * beyond; see esp_local_kernel) gives the full Coulomb potential of eq. task;
 * with esp_params.local = 1 the library adds it on the device, and
 * esp_params.method = 1 selects the classical method (Gaussian split,
 * B-spline window) on the same kernels. The m = 0 Fourier mode is dropped
 * (tin-foil boundary).
 *
 * Conventions shared by every entry point
 *   - Status codes: every call returns ESP_OK or a negative esp_status and
 *     never throws; esp_last_error() gives a thread-local message.
 *   - Device pointers: pos, q, phi, F are device memory on the plan's device,
 *     owned by the caller, valid for the duration of the call (and until the
 *     plan's stream reaches the call for the _async variant). They must not
 *     alias one another. Element type follows the plan precision: float for
 *     precision 32, double for precision 64.
 *   - Layouts: pos is N x 3 row-major (x, y, z per particle); q, phi are N;
 *     F is N x 3 row-major. Positions may lie anywhere: they are wrapped into
 *     [0, L). For a batch, the arrays of the systems are concatenated in system
 *     order.
 *   - The plan owns all scratch memory (grids, sorted particles, tables).
 *     The caller may supply the HIP stream the plan enqueues on
 *     (esp_params.stream, esp_plan_set_stream); otherwise the plan creates
 *     its own. PyTorch or any other allocator only supplies the caller's
 *     buffers and, optionally, the stream.
 *   - Thread safety: calls on different plans may run concurrently; calls on
 *     one plan must be serialised by the caller.
 */
#ifndef ESP_H
#define ESP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ESP_OK = 0,
    ESP_E_INVALID = -1,      /* bad argument (NULL, N < 1, box <= 0, tol out of range) */
    ESP_E_UNSUPPORTED = -2,  /* grid, window or cutoff outside the built range */
    ESP_E_NOT_NEUTRAL = -3,  /* |sum q| > 1e-6 sum |q|: results computed but meaningless */
    ESP_E_NOMEM = -4,        /* device allocation failed */
    ESP_E_DEVICE = -5,       /* HIP runtime error (message in esp_last_error) */
    ESP_E_BUSY = -6          /* serving: queue full / budget exhausted for this request */
} esp_status;

/* Parameters. On input (esp_plan_create_ex, esp_plan_query) a zero field means
 * "choose for me"; on output every field is resolved.
 *
 * Default rules (Methods, parameter selection; Table 2; eq. pswfparameters):
 *   c      solves psi_0^c(1) = tol (psi L2-normalised on [-1,1]);
 *   P      Table 2's P_esp for the largest tabulated eps not above tol
 *          (5 above 1e-3; +3 per decade below 1e-5, at most 12);
 *   nf     smallest even 2^a 3^b with L/nf <= h_max;
 *   rc     kappa * c * h / pi;
 *   c1     argmin over [0.9c, 1.4c] of the aliasing estimate (eq. errorformula);
 *   degree smallest polynomial degree whose piecewise fit of the window is
 *          within 0.05*tol of psi_0^{c1} (relative to its peak). */
typedef struct {
    int    nf;            /* grid points per side: even, 2^a 3^b, 8..144 */
    int    P;             /* window width in grid points, 4..12 */
    int    degree;        /* window polynomial degree, 4..16 */
    int    precision;     /* 32 (default) or 64 */
    int    tile;          /* particle bin edge in grid points, 8..16, rounded down to a
                             divisor of nf >= 8 (0: chosen per plan; reported by
                             esp_plan_get_params, 0 from esp_plan_query) */
    int    fft_passes;    /* 0: three FFT passes (x-planes, x-columns, x-planes);
                             1: one block per system for the whole 3D FFT where
                             the half spectrum fits in LDS (nf <= 32 in FP32,
                             <= 24 in FP64), three passes otherwise. Both are
                             deterministic; esp_plan_autotune may pick either. */
    double c;             /* splitting-kernel shape parameter: PSWF c (method 0) or the
                             Gaussian's alpha (method 1, default log(1/tol)) */
    double c1;            /* window PSWF shape parameter (method 0; 0 for method 1) */
    double rc;            /* cutoff radius of the local part */
    double h_max;         /* default-grid spacing bound (0: 1.25, length units) */
    double kappa;         /* default-cutoff margin (0: 1.2) */
    /* outputs only */
    double L;             /* box side */
    double h;             /* grid spacing L/nf */
    double tol;           /* requested tolerance */
    double s0;            /* self constant S(0) = chi(0)/(4 pi rc) */
    int    force_method;  /* forces (Methods, force paragraph): 0 analytic derivatives of
                             the window in the interpolation ("AD", default); 1 spectral
                             derivatives of the scaled spectrum ("ik": three more
                             gradient grids, each interpolated with the window) */
    int    local;         /* 1: also evaluate the local part u^l of the split (eq.
                             localpart, kernel L(r) inside rc) on the device, so that
                             phi, F and E are the full Coulomb values of eq. task
                             (needs rc <= L/2); 0: the long-range part only */
    int    method;        /* 0: ESP (PSWF splitting kernel and PSWF window, default);
                             1: the classical method (Methods, classical fast Ewald
                             methods, eq. cem): Gaussian splitting kernel
                             chi(t) = 2 sqrt(alpha/pi) exp(-alpha t^2), t = r/rc, and the
                             cardinal B-spline of order P as window, with the defaults
                             alpha = log(1/tol) and nf = 2 ceil(alpha L/(pi rc)) of eq.
                             cemparameters (rounded up to a supported grid), P = 5 and
                             rc the ESP cutoff at the same tolerance. Same kernels and
                             outputs; a baseline on the same hardware. */
    double Ly, Lz;        /* box sides along y and z (0: equal to L, a cubic box).
                             A non-cubic (orthorhombic) box keeps a cubic index grid
                             nf^3 with spacing L_d/nf per axis; nf follows the longest
                             side and rc the coarsest spacing; the influence function
                             becomes a per-system table. Set by esp_plan_create from
                             box[1], box[2]; outputs always hold the three sides. */
    double xy, xz, yz;    /* tilts of a triclinic cell (0: orthorhombic or cubic): the
                             lattice vectors are a = (L, 0, 0), b = (xy, Ly, 0) and
                             c = (xz, yz, Lz), the columns of an upper-triangular H.
                             The index grid nf^3 then runs over fractional coordinates
                             s = H^-1 r (grid point l at H l / nf); nf and the default rc
                             follow the longest lattice vector, and the local part needs
                             rc at most half the smallest distance between lattice
                             planes. Forces F = -q H^-T grad_s, by either force_method
                             (ik: derivatives along the fractional coordinates) and with
                             either method. Positions may lie anywhere (each is wrapped
                             into the cell). */
    void*  stream;        /* hipStream_t the plan enqueues on. Input of esp_plan_create_ex /
                             esp_batch_create (the batch takes reqs[0].stream): the
                             caller's stream, which the plan then uses and never
                             destroys; NULL: the plan creates and owns a stream of its
                             own. Output: the stream in use. See esp_plan_set_stream. */
    int    deterministic; /* 1: results are bitwise reproducible run to run and do not
                             depend on which other systems share a batch or a served step.
                             FP32 plans always are (the spread sums in 64-bit fixed point,
                             every other sum has a fixed order). FP64 plans are not: their
                             spread adds with FP64 LDS atomics, whose order varies, so
                             runs agree to rounding only. Input 0 (either) or 1 (required:
                             ESP_E_UNSUPPORTED for precision 64); output as described. */
} esp_params;

typedef struct esp_plan esp_plan;

/* ---- host-only queries (no device use; safe on machines without a GPU) ---- */

/* Resolve parameters for a box of sides box[0..2] (cubic or orthorhombic, or
 * a triclinic cell with req->xy, xz, yz), N particles and tolerance tol in
 * [1e-8, 1e-2]. req may be NULL. */
esp_status esp_plan_query(const double box[3], int64_t N, double tol,
                          const esp_params* req, esp_params* out);

/* Window polynomials used by the spread and gather kernels (eq. pswf, SI
 * kernel approximated by piecewise polynomials on intervals of length h).
 * For a particle at grid coordinate u, l0 = floor(u - P/2) + 1 and
 * y = u - P/2 - floor(u - P/2) - 1/2 in [-1/2, 1/2); the weight of grid point
 * l0 + j (j = 0..P-1) is sum_m coef[j*(degree+1) + m] y^m, approximating
 * psi_0^{c1}(2 (u - l0 - j)/P). coef must hold P*(degree+1) doubles. */
esp_status esp_window_coeffs(const esp_params* resolved, double* coef);

/* Influence function in factored form (eq. pk) of a cubic box: for Fourier
 * index m in [-nf/2, nf/2)^3,
 *   p_m = TS[mx^2+my^2+mz^2] * Tphi[|mx|] Tphi[|my|] Tphi[|mz|].
 * TS holds 3*(nf/2)^2 + 1 doubles (TS[0] = 0), Tphi holds nf/2 + 1 doubles.
 * Non-cubic boxes and cells use a per-system table built on the host at plan
 * creation; Tphi is still their per-axis factor. */
esp_status esp_influence_tables(const esp_params* resolved, double* TS, double* Tphi);

/* Local kernel of the split (eq. kernelsplitting), for pairing with a
 * short-range code: L(r) and dL/dr at the n radii r[] (r > 0). */
esp_status esp_local_kernel(const esp_params* resolved, const double* r, int64_t n,
                            double* Lr, double* dLr);

/* Piecewise polynomials the device evaluates for the local part, in grid
 * units (lengths divided by h; rho = rc/h). For 0 < r < rho, with
 * x = r^2/rho^2, piece k = min(floor(K x), K-1) and y = K x - k - 1/2:
 *   h L(h r)          = 1/(4 pi r) - sum_m A[k*(degree+1) + m] y^m,
 *   h^2 L'(h r) / r   = -1/(4 pi r^3) - sum_m B[k*(degree+1) + m] y^m.
 * A and B must hold ESP_LOCAL_COEF_MAX doubles each; *pieces = K and
 * *degree are written. Host only. */
#define ESP_LOCAL_COEF_MAX 104
esp_status esp_local_coeffs(const esp_params* resolved, double* A, double* B, int* pieces, int* degree);

/* Precompute (host, process-wide cache) the parameter classes of every grid
 * size 8..nf_max (even 2^a 3^b) for the default rules at each tolerance in
 * tols[ntol], using `threads` host threads (0: up to 16). A class holds the
 * window polynomials, influence tables and c1 search of one (grid, tolerance)
 * pair; the first plan or served request of a class otherwise pays for it
 * (~0.1 s). */
esp_status esp_warm_tables(const double* tols, int ntol, int nf_max, int threads);

/* ---- single-system plans ---- */

/* box[0..2]: the sides L, Ly, Lz (all equal for a cubic box); a triclinic
 * cell adds its tilts through req->xy, xz, yz. */
esp_status esp_plan_create(const double box[3], int64_t N, double tol, esp_plan** out);
esp_status esp_plan_create_ex(const double box[3], int64_t N, double tol,
                              const esp_params* req, esp_plan** out);

/* Batched plan: nsys independent systems of sides L[s] (with reqs[s].Ly, Lz for
 * orthorhombic ones and reqs[s].xy, xz, yz for triclinic ones), N[s] particles and
 * tolerances tol[s]; req (may be NULL) applies to every system, or reqs[s]
 * (may be NULL) per system. One call evaluates all systems with one launch per
 * pipeline phase (systems grouped by window width P). */
esp_status esp_batch_create(int nsys, const double* L, const int64_t* N, const double* tol,
                            const esp_params* reqs, esp_plan** out);

esp_status esp_plan_get_params(const esp_plan* plan, int sys, esp_params* out);
int        esp_plan_num_systems(const esp_plan* plan);
/* Stream (hipStream_t) the plan enqueues on: the caller's (esp_params.stream)
 * or the plan's own. */
void*      esp_plan_stream(const esp_plan* plan);
/* Enqueue all later work of the plan on `stream` (hipStream_t of the plan's
 * device; NULL selects the device's null stream, on which graph capture is
 * not possible). The call waits for the work already enqueued on the current
 * stream, so the plan's scratch is never used by two streams at once; a
 * stream the plan created stays alive until esp_plan_destroy. The caller
 * keeps `stream` alive while the plan uses it. A captured graph is kept (it
 * is launched on whichever stream is current). */
esp_status esp_plan_set_stream(esp_plan* plan, void* stream);

/* Evaluate potentials, forces and energy (Methods, five-step method; AD
 * forces). phi and/or F may be NULL to skip writing them. E is a HOST array
 * of nsys doubles (or NULL); when non-NULL the call waits for the stream and
 * checks neutrality, otherwise it returns after enqueueing. */
esp_status esp_longrange(esp_plan* plan, const void* pos, const void* q,
                         void* phi, void* F, double* E);

/* Same, never waiting: E_dev (device, nsys doubles, or NULL) receives the
 * energies; call esp_plan_sync to wait and check neutrality. */
esp_status esp_longrange_async(esp_plan* plan, const void* pos, const void* q,
                               void* phi, void* F, double* E_dev);
esp_status esp_plan_sync(esp_plan* plan);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: work issued while a stream is captured into a HIP graph, tight
 * serving loops, harnesses that forbid allocation): one evaluation of a single
 * system, as esp_plan_create_ex followed by esp_longrange and
 * esp_plan_destroy, with no device allocation. Every buffer of the pipeline
 * comes from one fixed block of ESP_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends; a system whose buffers do not
 * fit (the message states the bytes it needs) returns ESP_E_UNSUPPORTED. The
 * 300,000-atom water box at tol 1e-5 (grid 96, P = 8) needs about 26 MB.
 * box, N, tol, req: as esp_plan_create_ex (req may be NULL; req->stream is
 * ignored). pos, q, phi, F: as esp_longrange (device, caller-owned; phi or
 * F may be NULL). E: HOST, one double, or NULL. stream: the hipStream_t to
 * run on (NULL: the null stream). The call waits for the stream before it
 * returns and checks neutrality (ESP_E_NOT_NEUTRAL). Results are those of
 * esp_longrange on a plan with the same parameters (bin edge: req->tile, or
 * the default of a single-system plan).
 * Every call on one GPU uses that GPU's block: calls that overlap in time on
 * one GPU (from several host threads, or on several streams) race and
 * corrupt each other's results, so the caller serialises them. The block's
 * previous contents never matter (every buffer is written before it is
 * read within a call), so nothing is cleared between calls. */
#define ESP_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
esp_status esp_longrange_noalloc(const double box[3], int64_t N, double tol, const esp_params* req,
                                 const void* pos, const void* q, void* phi, void* F, double* E, void* stream);

/* Batched evaluation (Methods, five-step method, applied to many independent
 * systems at once): esp_longrange on a plan made by esp_batch_create. pos, q,
 * phi, F hold the systems' arrays concatenated in system order (device, plan
 * precision); E (HOST, nsys doubles, or NULL) receives each system's energy,
 * and when non-NULL the call waits and checks every system's neutrality
 * (ESP_E_NOT_NEUTRAL names the first offending system). Every system's
 * results are bitwise those it gets alone. Same errors as esp_longrange. */
esp_status esp_batch_longrange(esp_plan* batch, const void* pos, const void* q,
                               void* phi, void* F, double* E);

/* Short-range kernel of the plan's split for pairing with a short-range code
 * (Methods: eq. kernelsplitting, L(r) = 1/(4 pi r) - S(r) for r < rc and 0
 * beyond; eq. localpart sums q_j L(r_ij) over pairs within rc). Host only;
 * system 0 of a batch (esp_plan_get_params and esp_local_coeffs give any
 * other system's). coef (room for 2 * ESP_LOCAL_COEF_MAX doubles) receives
 * the two piecewise polynomials of esp_local_coeffs, A then B right after
 * it, each (*npieces) x (*degree + 1), in grid units of the plan (lengths divided by
 * its h = L/nf): for 0 < r < rc/h, with x = r^2 h^2/rc^2,
 * k = min(floor(K x), K-1), y = K x - k - 1/2,
 *   h L(h r)        = 1/(4 pi r)   - sum_m A[k][m] y^m,
 *   h^2 L'(h r) / r = -1/(4 pi r^3) - sum_m B[k][m] y^m.
 * The polynomials match L and L' to 1e-12 of their peak. */
esp_status esp_plan_shortrange_coeffs(const esp_plan* plan, double* coef, int* npieces, int* degree);

/* Autotuner of the bin edge T (batching: tile and bin sizes picked by
 * measurement). Systems are grouped by (grid size, window width); for each
 * group, largest total particle count first, every admissible T (divisors of
 * the grid size in [8, 16] whose spread tile and bin histogram fit in the
 * 160 KB LDS) is timed over `reps` full steps on the caller's data (pos, q,
 * phi, F as for esp_longrange_async, device, concatenated in system order)
 * with the other groups held at their current T, in three interleaved
 * sweeps of the candidates; the candidate with the fastest sweep is kept,
 * unless the group's current choice is within 2% of it.
 * Where the one-block FFT applies (fft_passes), both FFT paths are timed for
 * every T. The plan is then rebuilt with the choice: its scratch is reallocated and
 * a captured graph is dropped (recaptured on the next graph call). tiles_out
 * (nsys ints, may be NULL) receives the chosen T per system. Blocks until
 * done. Results depend on T only through rounding: the fold of the bins'
 * overlapping tiles into the grid adds in an order set by T, and the 32-bit
 * fixed-point spread (FP32, P <= 6) rounds each term to a unit set by its
 * bin's particle count (together about 1e-6 relative in FP32 forces, 1e-15 in
 * FP64). Within a bin the fixed-point sums are exact, so no result depends on
 * the order of the particles. */
esp_status esp_plan_autotune(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, int reps,
                             int* tiles_out);

/* Capture the whole pipeline for fixed buffers into a HIP graph and replay it
 * on every later esp_longrange call with the same pointers (0 disables). */
esp_status esp_plan_set_graph(esp_plan* plan, int enable);

void esp_plan_destroy(esp_plan* plan);

/* ---- diagnostics ---- */

/* Run the pipeline of a single-system plan up to one stage and copy the plan's
 * grid buffer (device, caller-owned) out:
 *   stage 1: b   real grid after spreading (eq. spread)
 *   stage 2: b^  spectrum after the forward FFT
 *   stage 3: c^  spectrum after diagonal scaling
 *   stage 4: c   real grid after the inverse FFT
 * Real grids are nf x nf x (nf+2) (last axis padded); spectra are
 * nf x nf x (nf/2+1) complex (interleaved re, im), the half spectrum along the
 * last axis, index k meaning mode k or k - nf. Element type follows the plan
 * precision. If grid_in (nf x nf x (nf+2) real) is non-NULL it replaces the
 * spread grid and pos/q are ignored (stages 2..4). */
esp_status esp_debug_stage(esp_plan* plan, const void* pos, const void* q,
                           const void* grid_in, int stage, void* grid_out);

/* The interpolation stage alone (eq. interp, AD forces) on a single-system
 * long-range plan (local = 0, force_method = 0): bins the particles as
 * esp_longrange does, takes grid_c (device, nf x nf x (nf+2) reals of the
 * plan precision, last axis padded) as the potential grid c, and writes
 *   phi_i = sum_l phi~(r_i - h l) c_l - q_i S(0),
 *   F_i   = -q_i grad_r sum_l phi~(r_i - h l) c_l
 * to phi and F (device, caller order; either may be NULL). Waits for the
 * stream. ESP_E_UNSUPPORTED for batches, local or ik plans. */
esp_status esp_debug_gather(esp_plan* plan, const void* pos, const void* q, const void* grid_c,
                            void* phi, void* F);

/* Time each pipeline phase: runs the full pipeline `reps` times on the plan's
 * stream with a HIP event between consecutive phases and writes the mean
 * milliseconds of each phase to ms[0..ESP_NUM_PHASES-1] (names from
 * esp_phase_name). Each timed pass follows an untimed one, so the phases
 * are not charged for host launch latency. Waits for the stream. */
#define ESP_NUM_PHASES 10
esp_status esp_plan_profile(esp_plan* plan, const void* pos, const void* q, void* phi, void* F,
                            int reps, double* ms);
int         esp_num_phases(void);
const char* esp_phase_name(int phase);

/* Time each launch of the spread or the gather phase (phase = index of
 * "spread" or "gather" in esp_phase_name): a plan with several pipeline
 * lanes launches one kernel per (lane, window width) there. Runs the
 * pipeline `reps` times on the plan's stream, the phase's launches one
 * after another with a HIP event around each, and writes for launch k <
 * *count (at most `max`) its mean milliseconds to ms[k], its particle count
 * to particles[k], the grid points of its systems (sum of n^3) to points[k]
 * and its workgroup count to blocks[k] (host arrays of `max` entries). Each
 * timed pass follows an untimed one. ESP_E_INVALID for other phases. Waits
 * for the stream. */
esp_status esp_plan_profile_launches(esp_plan* plan, const void* pos, const void* q, void* phi, void* F, int reps,
                                     int phase, int max, double* ms, int64_t* particles, int64_t* points,
                                     int64_t* blocks, int* count);

/* ---- serving: continuous batching of independent long-range solves ----
 *
 * A server owns one HIP stream, one scheduler thread and a device arena of
 * hbm_budget_bytes. Each request is a cubic system (FP32) that is evaluated
 * for nsteps consecutive MD steps; its positions stay resident on the device
 * and move between steps by a seeded drift (each coordinate by
 * drift * (2u - 1), u the SplitMix64 variate of the counter
 * (step << 40) + 3 i + c + 1 added to seed in multiples of 0x9E3779B97F4A7C15,
 * wrapped into [0, L)), so a host can reproduce every step. Requests are
 * admitted in arrival order while their state fits the arena and fewer than
 * max_active run; every scheduler iteration evaluates one step of every
 * admitted request with one launch per pipeline phase, so requests that
 * arrive while others run join the next iteration and their work overlaps on
 * the device. Results of one request do not depend on which others share
 * its launches (the spread sums in fixed point). Requests larger than the
 * whole budget are refused at submission with ESP_E_BUSY. All server calls
 * are thread-safe. Errors of server calls are reported by
 * esp_server_last_error. */
typedef struct esp_server esp_server;

typedef struct {
    size_t hbm_budget_bytes;  /* device memory for request state (0: 16 GiB), allocated at creation */
    int    max_active;        /* most requests admitted at once (0: 4096) */
    int    keep_outputs;      /* 1: keep each request's last-step phi and F for esp_server_fetch */
} esp_server_opts;

typedef struct {
    double       L;           /* cubic box side */
    int64_t      N;           /* particles (>= 2) */
    double       tol;         /* force tolerance, parameters as for esp_plan_create */
    const float* pos;         /* HOST, N x 3, copied by esp_server_submit */
    const float* q;           /* HOST, N, copied by esp_server_submit */
    int          nsteps;      /* steps to evaluate (>= 1) */
    double       drift;       /* drift amplitude per coordinate and step (0: static) */
    uint64_t     seed;        /* drift stream */
    uint64_t     tag;         /* returned in the result */
} esp_request;

typedef struct {
    uint64_t id, tag;
    int      status;          /* ESP_OK, ESP_E_NOT_NEUTRAL, or ESP_E_BUSY (never admitted) */
    int      nsteps;
    int64_t  N;
    int      nf, P;
    double   t_submit, t_admit, t_done;  /* seconds since the server was created */
    double   E_first, E_last;            /* energies of the first and the last step */
} esp_result;

typedef struct {
    int64_t submitted, admitted, completed, failed, active, waiting, iterations;
    double  particle_steps;   /* sum of N * nsteps over completed requests */
    double  busy_s;           /* scheduler host time enqueueing steps and handling their
                                 results (not waiting for the device) */
    double  span_s;           /* first submission to last completion */
    double  p50_latency_s, p99_latency_s, max_latency_s;  /* t_done - t_submit */
    size_t  bytes_in_use, bytes_peak;
    double  build_s;          /* scheduler host time assembling launch sets */
    double  admit_s;          /* scheduler host time admitting (incl. uploads) */
    double  step_s;           /* enqueue-to-results time of the steps, summed (iterations
                                 overlap: the next is enqueued before the previous
                                 one's results are taken) */
} esp_server_stats;

esp_status esp_server_create(const esp_server_opts* opts, esp_server** out);
/* Enqueue a request (never waits for the device); *id identifies its result. */
esp_status esp_server_submit(esp_server* server, const esp_request* req, uint64_t* id);
/* Move up to max finished results into out[]; *n receives how many. */
esp_status esp_server_poll(esp_server* server, esp_result* out, int max, int* n);
/* Copy a finished request's last-step outputs (HOST phi[N], F[N x 3]) once;
 * needs keep_outputs. */
esp_status esp_server_fetch(esp_server* server, uint64_t id, float* phi, float* F);
/* Wait until no request is queued or running (ESP_E_BUSY on timeout). */
esp_status esp_server_wait(esp_server* server, double timeout_s);
esp_status esp_server_get_stats(esp_server* server, esp_server_stats* out);
void       esp_server_destroy(esp_server* server);
const char* esp_server_last_error(void);

/* Message for the last failing call on this thread ("" if none). */
const char* esp_last_error(void);
/* Library version string. */
const char* esp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* ESP_H */
