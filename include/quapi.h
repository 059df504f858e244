/*
 * quapi.h -- C ABI of the MI355X (gfx950) QUAPI tensor-propagator library.
 *
 * The library propagates the reduced density matrix of an open quantum
 * system in the Feynman-Vernon model (Dattani 2012, Sec. II "Setting"):
 * given the system coordinate vector s, the system Hamiltonian H, the
 * spectral density J(omega) of the harmonic bath and its temperature, the
 * initial density matrix rho(0), and the convergence parameters
 * {dt, Delta k_max}, it returns rho(t_k) at the grid times t_k = k dt
 * (Sec. II, last paragraph; Sec. IV 'allPoints' / 'justFinalPoint').
 *
 * Method (Sec. II, exact path-sum equation with the discretized influence
 * functional and the eta_kk' definitions, evaluated by the tensor-propagator
 * scheme named in the Introduction):
 *   setup   G(t) = double time integral of the bath response alpha(t), by
 *           FP64 quadrature over J on the GPU; the eta classes as second
 *           differences of G; U = exp(-i H dt); K = U (x) conj(U); the
 *           influence-factor tables.  All on the device, in FP64.
 *   step    the augmented density tensor over the last Delta k_max path
 *           points (N^L complex entries, N = M^2, L = Delta k_max) is
 *           multiplied by K and the influence factors of the new point and
 *           its oldest index is summed out; rho(t_n) is extracted on
 *           selected steps from the same pass.
 *
 * Units: hbar = k_B = 1; kT is in the energy units of H, time in their inverse.
 *
 * Conventions common to every call:
 *   - Complex numbers are interleaved (re, im) doubles.  Matrices are M x M,
 *     row-major, in the basis of the coupling coordinate ordered as s.
 *   - Liouville index o = a*M + b for the path pair (s+ = s[a], s- = s[b]);
 *     rho(t)[a][b] is element o of an output block of M*M complex values.
 *   - A call never throws or aborts across the ABI; it returns a status and
 *     leaves a message for quapi_last_error().
 *   - One context is used by one thread at a time (QUAPI_ERR_STATE when a
 *     second call overlaps).  Distinct contexts may run concurrently, each on
 *     its own HIP stream.
 */
#ifndef QUAPI_H
#define QUAPI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct quapi_ctx quapi_ctx;   /* opaque; owned by the library */

typedef enum {
    QUAPI_OK = 0,
    QUAPI_ERR_INVALID = 1,   /* malformed argument (message says which) */
    QUAPI_ERR_NOMEM = 2,     /* the working set does not fit in free device memory */
    QUAPI_ERR_DEVICE = 3,    /* HIP runtime / kernel launch failure, or no device */
    QUAPI_ERR_STATE = 4      /* overlapping use of one context */
} quapi_status;

/* Precision of the augmented density tensor.  G, eta, U, K and the influence
 * tables are always FP64, and rho is always reduced in FP64 with compensated
 * sums.  The per-block and per-thread factor products are formed in FP64 and
 * rounded once to the arithmetic type. */
typedef enum {
    QUAPI_C128 = 0,          /* stored in complex128, FP64 products */
    QUAPI_C64 = 1,           /* stored in complex64, FP32 products with FP32 accumulation; the
                                K entries of the diagonal rows (a, a) are rounded to FP32 values
                                whose column sums are exactly delta_cd, so the rounding of K
                                does not change the trace of rho from step to step, and the
                                rows of the diagonal points, which carry the trace, sum their
                                FP32 values exactly and round each product once */
    QUAPI_C64_F64 = 2        /* stored in complex64; each loaded value is widened and every
                                product and sum is FP64, rounded to complex64 on store */
} quapi_dtype;

typedef enum {
    QUAPI_BATH_OHMIC = 0,    /* J(w) = (pi/2) xi w exp(-w / omega_c) */
    QUAPI_BATH_TABLE = 1     /* J tabulated at n_tab nodes, piecewise linear in w through
                                the anchor J(0) = 0, and zero beyond the last node */
} quapi_bath_kind;

/* Spectral density of the bath (Sec. II, spectral-distribution equation). */
typedef struct {
    int kind;                 /* quapi_bath_kind */
    double xi, omega_c;       /* OHMIC: xi >= 0, omega_c > 0 */
    const double *omega;      /* TABLE: n_tab nodes, strictly increasing, omega[0] > 0 */
    const double *J;          /* TABLE: J(omega[i]) >= 0 */
    int n_tab;                /* TABLE: >= 1, <= 1,000,000 */
} quapi_bath;

/* The problem statement (Sec. II, last paragraph).  Every pointer is read
 * during quapi_create only; the caller keeps ownership. */
typedef struct {
    int M;                    /* system dimension, 1 <= M <= 4 */
    const double *s;          /* M coupling-coordinate eigenvalues (the basis order) */
    const double *H;          /* M*M complex, Hermitian (tolerance 1e-12 of max |H_ij|) */
    const double *rho0;       /* M*M complex initial density matrix */
    quapi_bath bath;
    double kT;                /* >= 0; kT = 0 takes coth(w / 2kT) = 1 */
    double dt;                /* > 0 */
    int dk_max;               /* memory length L = Delta k_max, 1 <= L <= 30 */
    int dtype;                /* quapi_dtype */
    /* Driven system (optional; the model's Rabi frequency may depend on time,
     * Sec. III): n_H Hamiltonians, each M*M complex and Hermitian like H.  The
     * bare propagator of step k (interval (t_{k-1}, t_k]) is exp(-i H_t[k-1] dt)
     * for k <= n_H and uses H_t[n_H-1] after that.  NULL / n_H = 0: H for every
     * step.  A driven context computes every interval's propagator during
     * quapi_create, rewrites the tables that carry K before every step, and
     * runs one step per launch. */
    const double *H_t;
    int n_H;                  /* 0 <= n_H <= 1,000,000 */
} quapi_params;

/* Device bytes that quapi_create needs for these parameters (the two
 * ping-pong tensors of N^L entries dominate; factor tables and rho
 * reduction scratch add less than 0.2% of that plus 4 MB, and a driven
 * system 2 * n_H * M*M * 16 bytes for its Hamiltonians and propagators).
 * Validates the parameters; needs no GPU.  INVALID on malformed parameters
 * or size overflow. */
quapi_status quapi_footprint(const quapi_params *p, size_t *device_bytes);

/* The paper's primary memory cost (primary-memory-cost equation, Sec. II):
 * 64 * M^(2 (dk_max + 1)) bytes, i.e. four complex128 arrays of
 * M^(2 (dk_max + 1)) entries, which the paper's program stores.  This library
 * stores two arrays of M^(2 dk_max) entries instead.  Returns 0 on overflow
 * or bad arguments.  Needs no GPU. */
size_t quapi_paper_pmc_bytes(int M, int dk_max);

/* Create a propagation context and run the whole setup on the device:
 * quadrature of G(t) at t = j dt/2 (j = 0 .. 2L+2), the eta classes, U, K,
 * the influence tables, and the initial tensor.
 *   hip_stream  hipStream_t to run on (borrowed; must outlive the context),
 *               or NULL for a stream owned by the context.
 *   workspace   device memory of ws_bytes >= quapi_footprint() bytes
 *               (borrowed, e.g. a torch tensor's data_ptr; must outlive the
 *               context and be 256-byte aligned), or NULL for the library to
 *               allocate.  With NULL, NOMEM is returned when the footprint
 *               exceeds free device memory (or the QUAPI_FAKE_HBM_BYTES
 *               environment cap), the paper's "did not fit on the GPU".
 *   out         receives the context (NULL on failure).
 * Blocks until the setup has finished on the device.  For M = 4 the
 * full-window steps contract the oldest point once per distinct s_a - s_b
 * of the new point (a, b) where the levels allow it (evenly spaced levels
 * do); QUAPI_STEP16_CLASSES=0 in the environment at creation keeps one
 * contraction per new point (the results differ by rounding only). */
quapi_status quapi_create(const quapi_params *p, void *hip_stream, void *workspace,
                          size_t ws_bytes, quapi_ctx **out);

/* Advance the context by n_steps >= 0 time steps, from its current global
 * step c to c + n_steps, and return rho at the selected global steps.
 *   sel      strictly increasing global step indices k with c < k <= c + n_steps,
 *            or k == 0 (rho(t_0) = rho0); NULL selects every k in (c, c + n_steps]
 *            (the paper's 'allPoints'); {c + n_steps} is 'justFinalPoint'.
 *   n_sel    length of sel (ignored when sel is NULL).
 *   rho_out  host buffer of n_out * M*M complex (n_out = n_sel, or n_steps when
 *            sel is NULL), written in selection order; caller-owned.
 * Blocking: returns when the results are on the host.
 * Results are deterministic.  For M = 2 full-window steps run in fused groups
 * of F = quapi_fused_steps() steps fixed by the global step number:
 * (L+1 .. L+F), (L+F+1 .. L+2F), ...  A sequence of calls gives bit-identical
 * results to one call when every call ends at step c <= L or with c - L a
 * multiple of F (otherwise the steps of a split group run one by one, or as
 * one two-step launch when a call ends two steps into a three-step group, and
 * round differently, within 1e-15).  F is chosen as quapi_set_fused_steps
 * describes. */
quapi_status quapi_propagate(quapi_ctx *ctx, int n_steps, const int *sel, int n_sel,
                             double *rho_out);

/* As quapi_propagate, but enqueues the work on the context's stream and
 * returns at once; rho_out_dev is device memory of n_out * M*M complex128
 * (caller-owned; valid once the stream has reached this point). */
quapi_status quapi_propagate_async(quapi_ctx *ctx, int n_steps, const int *sel, int n_sel,
                                   void *rho_out_dev);

/* Path filtering: Sim's on-the-fly filtering of the tensor propagator, which
 * the paper names in its Introduction as the way to cut the memory of the
 * augmented tensor.  Read here as: every entry of the tensor whose magnitude
 * is not above theta is dropped as soon as it is formed (the initial tensor
 * and the tensor after every step), so the paths it stands for take no
 * further part; theta = 0 drops exact zeros only and gives the unfiltered
 * result.  The kept entries are stored as (flat index, value) pairs sorted
 * by index, in two buffers of `capacity` entries, so the memory follows the
 * kept count instead of N^L, and N^dk_max may reach 2^62.
 *
 * quapi_create_filtered: as quapi_create (its own device allocation; hip_stream
 *   borrowed or NULL), with theta >= 0 finite and 1 <= capacity <= 2^38.
 *   The context works with quapi_propagate,
 *   quapi_propagate_async, quapi_step_count, quapi_get_setup, timing and
 *   quapi_destroy; every step runs as its own sequence of launches (no fused
 *   steps, mirror mode, persistent path or graphs), and quapi_read_tensor,
 *   quapi_restore and quapi_tensor_size refuse it (INVALID).
 *   When a step keeps more than `capacity` entries, the entries beyond it are
 *   lost, a sticky overflow flag is set on the device, and the results from
 *   that step on are wrong: quapi_propagate then returns QUAPI_ERR_NOMEM, and
 *   after quapi_propagate_async the caller reads the flag with
 *   quapi_filter_stats.  Deterministic (integer scans, fixed-order sums).
 * quapi_filtered_footprint: device bytes of such a context (about
 *   capacity * (2 * (8 + sizeof(complex)) + 2) plus a few MB of tables);
 *   needs no GPU.
 * quapi_filter_stats: waits for the context's stream, then gives the entries
 *   kept after the last step and the overflow flag (0 or 1).
 * quapi_filter_read: waits for the stream, then copies kept entries
 *   [first, first + count) in index order: keys (flat index, oldest point
 *   fastest, as quapi_read_tensor's positions) and vals (count complex128,
 *   interleaved); INVALID when the range exceeds the kept entries.
 * All return INVALID for NULL arguments and for contexts that are not
 * filtered (stats, read); STATE while another call runs on the context. */
quapi_status quapi_filtered_footprint(const quapi_params *p, size_t capacity, size_t *device_bytes);
quapi_status quapi_create_filtered(const quapi_params *p, double theta, size_t capacity, void *hip_stream,
                                   quapi_ctx **out);
quapi_status quapi_filter_stats(quapi_ctx *ctx, long long *entries, int *overflow);
quapi_status quapi_filter_read(quapi_ctx *ctx, size_t first, size_t count, long long *keys, double *vals);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * propagation -- the setup of quapi_create, n_steps steps from step 0 and
 * rho at the selected steps, as quapi_propagate_async -- with its entire
 * working set (both tensors, the factor tables and the rho reduction
 * buffers) in a static device array of 64 MiB that the library holds on each
 * GPU until the process ends.  It calls no hipMalloc or hipFree and creates
 * no streams or events: every kernel runs on hip_stream (NULL: the null
 * stream).
 *   p, n_steps, sel, n_sel   as quapi_create / quapi_propagate (global steps
 *                            0 < k <= n_steps, or k = 0 for rho0)
 *   rho_out_dev              device memory of n_out * M*M complex128,
 *                            caller-owned, written in selection order
 * Blocks until the work has finished on hip_stream, then returns; the result
 * equals quapi_create + quapi_propagate_async on the same parameters, bit for
 * bit (the same kernels run in the same order; no captured graphs).
 * Every call on one GPU uses that GPU's one array, which keeps the last call's
 * contents: calls from different threads of a process on one GPU are
 * serialized by the library, and a call must not overlap other work that
 * reads or writes it (there is none outside this call).
 * Errors: QUAPI_ERR_INVALID for malformed parameters or selection, NULL
 * rho_out_dev with outputs selected, or a working set (quapi_footprint)
 * above 64 MiB (e.g. M = 2 beyond dk_max = 10 at complex128); QUAPI_ERR_DEVICE
 * for runtime or launch failures. */
quapi_status quapi_propagate_static(const quapi_params *p, int n_steps, const int *sel, int n_sel,
                                    void *rho_out_dev, void *hip_stream);

/* The persistent path.  A context whose tensor has at most 2^14 entries
 * (N^L; M = 2 up to dk_max = 7, M = 3 up to 4, M = 4 up to 3) runs every
 * step of a call in one launch, one workgroup per context: the tensor stays
 * in LDS when both of its buffers fit there (M = 2 up to dk_max = 6),
 * otherwise in the context's two buffers in HBM, which stay in the L2 cache
 * at these sizes; a step costs a workgroup barrier instead of kernel
 * launches.  Not for driven contexts, contexts whose launch width is pinned
 * (quapi_set_fused_steps != 0) or mirror mode 2.  Results do not depend on
 * how a run is split into calls or batched.
 *   quapi_persistent:  *mode = 0 (multi-block kernels), 1 (persistent, tensor
 *                      in LDS) or 2 (persistent, tensor in HBM).
 * Errors: QUAPI_ERR_INVALID for NULL arguments. */
quapi_status quapi_persistent(const quapi_ctx *ctx, int *mode);

/* Advance n_ctx contexts in as few launches as possible: the serving loop's
 * batched form of quapi_propagate_async (the paper's many runs that differ
 * in a parameter, Sec. IV).  Every context must be on the persistent path
 * (quapi_persistent != 0), and all must have the same M and dtype (their
 * memory lengths, baths, Hamiltonians and step counts may differ); one
 * workgroup runs one context, up to 32 contexts per launch.  Context k
 * advances n_steps[k] >= 0 steps and writes rho to device memory
 * rho_out_dev[k] (caller-owned, complex128, N values per output):
 *   rho_mode[k] = 0 none, 1 every step (n_steps[k] outputs, 'allPoints'),
 *                 2 the last step only (one output, 'justFinalPoint').
 * Enqueued on the first context's stream, after the work already queued on
 * every context's stream; later work on any of the contexts' streams runs
 * after it.  Returns at once.  Each context's results equal those of its
 * own quapi_propagate calls over the same steps, bit for bit.
 * Errors: QUAPI_ERR_INVALID for NULL arguments, a repeated or unsuitable
 * context, mixed M or dtype, negative steps, rho_mode outside 0..2 or a NULL
 * output buffer with outputs; QUAPI_ERR_STATE when a context is in use;
 * QUAPI_ERR_DEVICE on launch failure. */
quapi_status quapi_propagate_batch(quapi_ctx *const *ctxs, int n_ctx, const int *n_steps, const int *rho_mode,
                                   void *const *rho_out_dev);

/* Global step index the context has reached (0 after create). */
quapi_status quapi_step_count(const quapi_ctx *ctx, int *step);

/* Test hooks: copy setup results to host (complex values interleaved).
 *   what = QUAPI_SETUP_G     G(j dt/2), j = 0 .. 2L+2                  (2L+3 values)
 *          QUAPI_SETUP_ETA   eta classes: self interior, self end, then
 *                            lag[1..L], init[1..L], fin[1..L], fin_init[1..L] (4L+2)
 *          QUAPI_SETUP_U     exp(-i H dt), M x M row-major             (M*M)
 *          QUAPI_SETUP_K     K[o', o] = U[a',a] conj(U[b',b]), N x N      (N*N)
 *   out_len  number of doubles available at out (INVALID when too small). */
enum { QUAPI_SETUP_G = 0, QUAPI_SETUP_ETA = 1, QUAPI_SETUP_U = 2, QUAPI_SETUP_K = 3 };
quapi_status quapi_get_setup(const quapi_ctx *ctx, int what, double *out, size_t out_len);

/* Copy entries [first, first + count) of the current augmented tensor to
 * host as complex128 (a test hook; the whole tensor is the checkpoint that
 * quapi_restore takes back).
 * Layout after global step c >= 1: the tensor holds path points
 * max(0, c-L+1) .. c, flat index sum_j o_{p0 + j} N^j (oldest point fastest),
 * N^min(c+1, L) entries (complex64 storage is widened to complex128).
 * INVALID when the range exceeds the tensor; QUAPI_ERR_STATE while another
 * call runs on the context. */
quapi_status quapi_read_tensor(const quapi_ctx *ctx, size_t first, size_t count, double *out);

/* Resume from a checkpoint.  The state a context carries from one call to
 * the next is its step count c and its tensor (the factor tables depend only
 * on the parameters); quapi_step_count and quapi_read_tensor (first = 0,
 * count = quapi_tensor_size) read it out.  quapi_restore puts such a state
 * into a context created from the same parameters: step = c >= 0, tensor =
 * N^min(c+1, L) complex values interleaved (re, im) in the layout of
 * quapi_read_tensor, host memory, read only during the call (for complex64
 * storage each value is rounded to complex64, so a state read from a
 * complex64 context goes back unchanged).  The next quapi_propagate continues
 * with step c+1 and gives the same results, bit for bit, as the context the
 * state was read from would have given (the fused groups are fixed by the
 * global step number).  The call waits for the context's queued work first.
 * Errors: QUAPI_ERR_INVALID for NULL arguments, step < 0 or a count other
 * than N^min(step+1, L); QUAPI_ERR_STATE while another call runs on the
 * context; QUAPI_ERR_DEVICE when the copy fails. */
quapi_status quapi_restore(quapi_ctx *ctx, int step, const double *tensor, size_t count);

/* Number of entries in the current tensor (N^min(c+1, L)). */
quapi_status quapi_tensor_size(const quapi_ctx *ctx, size_t *entries);

/* Full-window steps that one launch advances for this context (3, 2 or 1),
 * the group size of the determinism rule of quapi_propagate.
 * Errors: QUAPI_ERR_INVALID for NULL arguments. */
quapi_status quapi_fused_steps(const quapi_ctx *ctx, int *steps);

/* Choose the full-window steps per launch: 1, 2 (N = 4, L >= 3), 3 (N = 4,
 * L >= 4), or 0 for the default: 3 at complex128 and QUAPI_C64 from L = 13,
 * else 2 where available, else 1; always 1 for a driven context.  Every choice gives the same results to within rounding (the
 * fused kernels apply the same factors in another order); use it to pin the
 * kernel, e.g. in tests.  It takes effect from the next call.
 * Errors: QUAPI_ERR_INVALID for an unavailable width; QUAPI_ERR_STATE while
 * another call runs on the context. */
quapi_status quapi_set_fused_steps(quapi_ctx *ctx, int steps);

/* Mirror mode of the full-window kernels: the three-step kernel (M = 2,
 * L >= 4), the two-step kernel (M = 2, L >= 3) and the single step (M = 2, 3,
 * 4; L >= 2).  Swapping the forward and
 * backward path of every point maps the path sum of Sec. II to its complex
 * conjugate: K = U (x) U* and every influence factor go to their conjugates,
 * and so does rho(0) when it is Hermitian.  So the tensor entry of the
 * mirrored paths is the conjugate of the entry itself, and a pass reads and
 * writes only the entries not above their mirror (flat index, each digit
 * (a, b) -> (b, a)) -- about half the bytes.  rho at every step is unchanged
 * up to rounding.  On by default where available.  The single step and the
 * two-step kernel use it for tensors above 2^22 entries only (smaller steps
 * are bound by their launches, and mirror mode takes three); the three-step
 * kernel always.  The entries above their mirror are filled in (one pass
 * over the tensor) before anything that reads the whole tensor: a kernel
 * that does not take mirror mode, quapi_read_tensor.
 *   quapi_mirror:      *enabled = the mode: 0 off, 1 on (default), 2 on at every size.
 *   quapi_set_mirror:  enable = 0, 1 or 2 as above.
 * Errors: QUAPI_ERR_INVALID for NULL arguments, enable outside 0..2, or enable > 0 where it is not
 * available (M other than 2, 3 or 4, L = 1, or rho0 not exactly Hermitian);
 * QUAPI_ERR_STATE while another call runs on the context. */
quapi_status quapi_mirror(const quapi_ctx *ctx, int *enabled);
quapi_status quapi_set_mirror(quapi_ctx *ctx, int enable);

/* Kernel timing with HIP events on the context's stream. */
typedef struct {
    double setup_ms;          /* device time of the setup kernels in quapi_create */
    double step_ms;           /* summed duration of full-window step kernels (n >= L) */
    long long step_launches;  /* number of those launches (in mirror mode: of their groups of three) */
    long long step_steps;     /* full-window steps they covered (a fused launch covers two or three) */
    double grow_ms;           /* summed duration of growth-step kernels (n < L) */
    long long grow_launches;
    double finalize_ms;       /* summed duration of the kernels that sum rho over blocks */
    long long finalize_launches;
    /* step_ms / step_launches split by the full-window steps a launch covers:
     * index 1 single steps, 2 two-step launches, 3 three-step launches (index
     * 0 unused).  A launch in mirror mode counts its group of three kernels. */
    double width_ms[4];
    long long width_launches[4];
} quapi_timing;

/* enable != 0 records an event pair around every propagation kernel launch. */
quapi_status quapi_set_timing(quapi_ctx *ctx, int enable);
/* Waits for the stream, returns the accumulated timings, and resets them
 * (setup_ms is kept). */
quapi_status quapi_get_timing(quapi_ctx *ctx, quapi_timing *out);

/* Measurement aid, not part of the method: enqueue one device copy of
 * `bytes` from src to dst (both device memory, 16-byte aligned, bytes a
 * multiple of 16) on hip_stream (NULL: the null stream).  Each block of 512
 * threads copies one contiguous chunk of chunk_bytes (a multiple of 16,
 * >= 8192) with 16-byte accesses; nontemporal != 0 marks the loads
 * nontemporal.  Timing it with events on the stream gives the attainable
 * HBM read+write rate that the step kernels are compared with.  Returns
 * QUAPI_ERR_INVALID for bad arguments, QUAPI_ERR_DEVICE when the launch
 * fails; the call does not wait for the copy. */
quapi_status quapi_copy_bandwidth(const void *src, void *dst, size_t bytes, size_t chunk_bytes,
                                  int nontemporal, void *hip_stream);

/* Release the context and everything it allocated (not a caller workspace). */
quapi_status quapi_destroy(quapi_ctx *ctx);

/* Message of the last failed call on ctx, or of the calling thread's last
 * failed call when ctx is NULL.  Valid until the next call. */
const char *quapi_last_error(const quapi_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* QUAPI_H */
