/*
 * lw.h -- C ABI of the MI355X (gfx950) radiation spectral synthesis library.
 *
 * The library evaluates, on one GPU, the discretised Lienard-Wiechert
 * spectral integral that the paper accumulates in situ for a sample of PIC
 * particles (Section 2.2, "Radiation Spectral Synthesis": the discretised
 * Rybicki-Lightman expression for d^2W/(dOmega domega), integrated over
 * emission time with the retarded phase phi' = t' - n.r(t')/c, seen by far
 * observers at arbitrary orientation, on log or linear frequency bins,
 * summed over particles).  In the paper's units c = m_e = q_e = 1:
 *
 *   kappa_k  = 1 - n.beta_k
 *   g_k      = n x ((n - beta_k) x betadot_k) / kappa_k^2
 *   A_p(n,w) = sum_k g_k exp(i w (t_k - n.r_k)) dt_p
 *   S(s,n,w) += sum_{p in species s} w_p q_p^2 |A_p(n,w)|^2 / (4 pi^2)
 *
 * S is the energy radiated per unit frequency and solid angle (incoherent
 * synthesis, one of the two options of Section 2.2).
 *
 * Conventions
 *   - Every call returns lw_status; nothing throws across the ABI.  After a
 *     failure lw_last_error() describes it.
 *   - Pointers named host_* are host memory; every pointer in lw_batch and
 *     the workspace/per-particle pointers are device memory on the context's
 *     device.  The caller owns them and keeps them valid until the stream has
 *     passed the call.  The context owns its grids and the accumulator S.
 *   - Calls that launch work are asynchronous and ordered on the context's
 *     stream (a hipStream_t passed as void*; NULL = the default stream).
 *   - Data errors detected on the device (|beta| >= 1, non-finite samples, a
 *     species index outside [0, n_species)) record the lowest offending
 *     particle index; the offending sample (or particle, for a bad species)
 *     contributes nothing and the next lw_read_spectra returns LW_ERANGE.
 *   - A context is not thread safe; use one context per host thread.
 */
#ifndef LW_H
#define LW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LW_OK = 0,
  LW_EINVAL = -1,       /* bad argument (message in lw_last_error) */
  LW_ENOMEM = -2,       /* device allocation failed or workspace too small */
  LW_EDEVICE = -3,      /* HIP runtime error */
  LW_ESTATE = -4,       /* call out of order (e.g. accumulate before grids are set) */
  LW_ERANGE = -5,       /* |beta| >= 1 or non-finite sample seen on the device */
  LW_EUNSUPPORTED = -6  /* option not available */
} lw_status;

/* Arithmetic of the accumulation.
 *   LW_PATH_FP32: retarded time, kappa, g and the phase w*tau reduced to a
 *     turn fraction in FP64; phase factors and the sum over samples in FP32,
 *     with FP64 partial sums every 16 samples.
 *   LW_PATH_MFMA_F16 / LW_PATH_MFMA_BF16: the sum over samples as a dense
 *     contraction on the matrix cores -- each particle's integrand is spread
 *     onto a uniform retarded-time grid per frequency band, contracted with
 *     a shared table of phase factors e^{i w q h} in FP16 (BF16), FP32
 *     accumulation, then deconvolved (see lw_set_mfma_options).
 *   LW_PATH_AUTO: the library picks one of the above per call: the FP16
 *     matrix-core path (hi/lo operands unless lw_set_mfma_options chose one
 *     product) when no per-particle output is asked for and the frequency
 *     list has at least LW_AUTO_MIN_FREQUENCIES points (where that path
 *     measured faster than the FP32 path), the FP32 path otherwise.  Each of
 *     the two keeps its own stated error. */
typedef enum { LW_PATH_FP32 = 0, LW_PATH_MFMA_F16 = 1, LW_PATH_MFMA_BF16 = 2, LW_PATH_AUTO = 3 } lw_path;
#define LW_AUTO_MIN_FREQUENCIES 256

/* Particle batch (structure of arrays, device pointers, borrowed).
 * Particle p owns samples offsets[p] .. offsets[p+1]-1 (offsets non-decreasing,
 * offsets[0] may be > 0, every offset within the sample arrays); sample k of
 * particle p is at time t0[p] + k*dt[p].  beta = (bx,by,bz) = v/c,
 * betadot = (ax,ay,az) = d(beta)/dt, r = (x,y,z).  species may be NULL (all
 * particles in species 0).  flags: 0, or LW_BATCH_F64_ACCEL when ax, ay, az
 * point to double arrays (they are then read as FP64; the FP32 path keeps the
 * integrand in FP64 up to its final rounding).  A particle whose offsets
 * decrease is a data error (recorded like |beta| >= 1; it adds nothing); the
 * sample arrays are not bounds-checked. */
#define LW_BATCH_F64_ACCEL 1u
typedef struct {
  int64_t n_particles;
  const int64_t* offsets; /* [n_particles + 1] */
  const double *x, *y, *z;
  const double *bx, *by, *bz;
  const float *ax, *ay, *az;
  const double *t0, *dt;  /* [n_particles] */
  const float *charge;    /* [n_particles] q_p in units of e */
  const float *weight;    /* [n_particles] w_p (macro-particle weight) */
  const int32_t* species; /* [n_particles] or NULL */
  uint32_t flags;         /* 0 or LW_BATCH_F64_ACCEL */
} lw_batch;

typedef struct lw_ctx lw_ctx;

/* Create a context on HIP device `device`, ordered on `stream` (hipStream_t,
 * borrowed; NULL = default stream).  *out receives the context. */
lw_status lw_create(lw_ctx** out, int device, void* stream);
/* Free the context and everything it owns (synchronises its stream).  Networks
 * (lw_mlp) and graphs (lw_graph) made on it refer to it: destroy them first. */
void lw_destroy(lw_ctx* ctx);
/* Text of the last error on this context; valid until the next call on it. */
const char* lw_last_error(const lw_ctx* ctx);
/* Change the stream later calls are ordered on. */
lw_status lw_set_stream(lw_ctx* ctx, void* stream);

/* Observer directions (Section 2.2: several far-field observers at
 * arbitrary orientation).  host_n_xyz is [nd][3], copied and normalised;
 * a zero or non-finite vector is LW_EINVAL.  Resets S. */
lw_status lw_set_directions(lw_ctx* ctx, const double* host_n_xyz, int32_t nd);
/* Frequency points (Section 2.2: logarithmic or linear binning), host [nw],
 * finite and > 0; copied.  Resets S. */
lw_status lw_set_frequencies(lw_ctx* ctx, const double* host_omega, int32_t nw);
/* w_j = wmin (wmax/wmin)^(j/(nw-1)), j = 0..nw-1, endpoints exact. Resets S. */
lw_status lw_set_log_frequencies(lw_ctx* ctx, double wmin, double wmax, int32_t nw);
/* Copy the current frequency points to host_omega [nw]. */
lw_status lw_get_frequencies(const lw_ctx* ctx, double* host_omega);
/* Number of species accumulated separately (>= 1, <= 8).  Resets S. */
lw_status lw_set_species(lw_ctx* ctx, int32_t n_species);

/* Matrix-core path options.  bands: number of frequency bands (contiguous runs
 * of the frequency list, 1..16; default 1), each with its own retarded-time
 * grid.  More bands shrink the contraction (its rows per band) but every band
 * spreads every sample again.  products_f16 / products_bf16: 1 = operands rounded once to FP16/BF16;
 * 3 = each operand split into hi + lo parts and hi*hi + hi*lo + lo*hi summed;
 * 2 (FP16 only) = the phase table rounded once and F split, E_hi*F_hi +
 * E_hi*F_lo summed.  Defaults: 3 for both.  One or two products keep 11 (FP16)
 * or 8 (BF16) mantissa bits in at least one operand and are measured, not
 * guaranteed, against the 1e-3 band target; they spread with the (W = 8,
 * sigma = 2) kernel, three products with (W = 10, sigma = 1.6).  LW_EINVAL for
 * other counts. */
lw_status lw_set_mfma_options(lw_ctx* ctx, int32_t bands, int32_t products_f16,
                              int32_t products_bf16);
/* Cap on the spread grids F (all directions and bands, FP32) held per chunk of particles,
 * in bytes; 0 restores the default of 24 GiB.  The matrix-core path walks a batch in chunks
 * of at least 64 particles that keep F under the cap (a smaller cap: a smaller workspace,
 * more launches).  Query lw_workspace_size again after changing it. */
lw_status lw_set_mfma_chunk_bytes(lw_ctx* ctx, int64_t bytes);
/* Plans the batch for a matrix-core path as lw_workspace_size does (synchronises) and
 * reports host_out[4] = {particles per chunk, chunks, frequency bands, workspace bytes}.
 * LW_EINVAL for the FP32 path. */
lw_status lw_mfma_plan_info(lw_ctx* ctx, const lw_batch* batch, lw_path path, int64_t* host_out);

/* Device workspace (bytes) lw_accumulate needs for this batch and path.  For
 * the matrix-core paths this call plans the batch: it reads the batch on the
 * device to size the retarded-time grids (it synchronises the stream),
 * prepares the phase tables (with 25 % headroom in span) and remembers the
 * batch (its offsets pointer and particle count) as planned, as
 * lw_plan_batch does.  LW_PATH_AUTO sizes the path lw_accumulate would pick. */
lw_status lw_workspace_size(lw_ctx* ctx, const lw_batch* batch, lw_path path, size_t* bytes);

/* Add the batch's spectrum into S.  Asynchronous and stream-ordered: the FP32
 * path never synchronises; the matrix-core paths do not for a planned batch
 * (the last batch lw_workspace_size or lw_plan_batch saw, identified by its
 * offsets pointer and particle count, on the same grids and options), whose
 * samples are checked against the plan on the device instead: a particle whose
 * retarded-time span outgrew the plan is recorded, and the next lw_read_spectra
 * (or lw_read_amplitudes) returns LW_ESTATE naming it -- plan the batch again and
 * redo the call.  Any other batch is planned first, which synchronises once.
 * workspace: device memory of at least lw_workspace_size bytes, 256-byte aligned.
 * per_particle: NULL or device float [n_particles][nd][nw] receiving each
 * particle's own w_p q_p^2 |A_p|^2 / (4 pi^2) (FP32 path only; LW_EUNSUPPORTED
 * otherwise).  Host-side checks (sizes, NULL pointers, flags, workspace size and
 * alignment) fail before any launch. */
lw_status lw_accumulate(lw_ctx* ctx, const lw_batch* batch, lw_path path, void* workspace,
                        size_t workspace_bytes, float* per_particle);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): lw_accumulate on the FP32 path, plain
 * grid launch, with its per-block partial sums in a library-owned static device array of
 * LW_NOALLOC_SCRATCH_MB MiB instead of a caller workspace.  The call itself allocates
 * nothing (no hipMalloc, no events; profiling and per-particle output are not offered).
 * Each GPU holds its own copy of the array from the first lw_create on it until the process
 * ends; every call on that GPU shares it, so calls that overlap on one GPU (several contexts
 * or streams) race -- order them on one stream.  The partial sums need n_blocks x
 * n_species x nd x nw (x 4 in coherent mode) doubles, n_blocks as lw_workspace_size of the
 * FP32 path counts them; a batch that needs more than the array is refused with LW_ENOMEM
 * before any launch.  Results equal lw_accumulate's plain-grid FP32 results bit for bit. */
#define LW_NOALLOC_SCRATCH_MB 64
lw_status lw_accumulate_noalloc(lw_ctx* ctx, const lw_batch* batch);

/* Synchronise the stream and copy S to host_out [n_species][nd][nw] (FP64).
 * Returns LW_ERANGE (with the particle index in lw_last_error) if a device
 * data error was recorded since the last reset; S is copied regardless. */
lw_status lw_read_spectra(lw_ctx* ctx, double* host_out);
/* Zero S and the device error record (asynchronous). */
lw_status lw_reset(lw_ctx* ctx);
/* Replace S with host_in [n_species][nd][nw] (resume from a saved state). */
lw_status lw_load_accumulator(lw_ctx* ctx, const double* host_in);
/* Periodic recording (Section 2.2 records the accumulated spectra as the run
 * goes): write the accumulator to the file at `path` -- a 64-byte header
 * ("LWACC001", species, directions, frequencies, coherent flag, payload length,
 * FNV-1a 64 checksum of everything after the header), the directions [nd][3]
 * and frequencies [nw] (FP64), then S [n_species][nd][nw] (incoherent) or A_s
 * [n_species][nd][nw][4] (coherent), little-endian FP64.  Synchronises; does
 * not report device data errors (lw_read_spectra does). */
lw_status lw_save_accumulator(lw_ctx* ctx, const char* path);
/* Resume from such a file: the context's species count, directions,
 * frequencies and mode must equal the file's (bitwise for the grids), else
 * LW_EINVAL; a short or corrupted file (checksum) is LW_EINVAL and leaves the
 * accumulator unchanged.  Synchronises. */
lw_status lw_load_accumulator_file(lw_ctx* ctx, const char* path);

/* ---- coherent synthesis and in-situ recording (Section 2.2, recording scheme) ----
 * The observed power is the squared modulus of the time integral of the summed
 * retarded fields: amplitudes add before squaring.  Summed over the particles of
 * a species (coherent synthesis) that is
 *   A_s(n, w) = sum_{p in s} w_p q_p A_p(n, w),  S = |A_s|^2 / (4 pi^2),
 * and squared per particle (incoherent synthesis, the default) it is
 * S = sum_p w_p q_p^2 |A_p|^2 / (4 pi^2).  Because the integral runs from the
 * start of recording to the current step, a spectrum taken over a later stretch
 * of time is the difference of two recorded spectra, P(t1) - P(t0).  Species
 * slots double as collection regions: the caller assigns each particle to one.
 *
 * Amplitudes are stored as four FP64 numbers per (direction, frequency): the real
 * and imaginary part of the component on e1, then those on e2, where (e1, e2, n)
 * is the orthonormal right-handed basis of lw_get_basis (A is perpendicular to n).
 *
 * lw_set_coherent: 1 = coherent, 0 = incoherent synthesis.  Resets S (and A).
 * In coherent mode lw_accumulate (every path; the matrix-core paths restore each
 * column's phase e^{i w tau_0} in the contraction's epilogue) and
 * lw_accumulate_subset add w_p q_p A_p into A_s; time windows of a run passed as
 * successive batches (each particle's t0 is the window's first sample time)
 * therefore build the integral over the whole run; lw_read_spectra returns
 * |A_s|^2 / (4 pi^2), and lw_reset zeroes A.  The surrogate is incoherent only. */
lw_status lw_set_coherent(lw_ctx* ctx, int32_t coherent);
/* host_out [nd][9]: per direction n, e1, e2 (unit vectors, FP64). */
lw_status lw_get_basis(const lw_ctx* ctx, double* host_out);
/* Coherent mode only (LW_ESTATE otherwise).  Synchronise and copy A_s to
 * host_out [n_species][nd][nw][4]; LW_ERANGE as for lw_read_spectra. */
lw_status lw_read_amplitudes(lw_ctx* ctx, double* host_out);
/* Coherent mode only: replace A_s with host_in [n_species][nd][nw][4] (resume). */
lw_status lw_load_amplitudes(lw_ctx* ctx, const double* host_in);
/* Per-particle amplitude state for incoherent in-situ recording.  amp: device
 * FP64 [n_particles][nd][nw][4], 16-byte aligned, owned by the caller, zeroed
 * by the caller before the first window; each call adds the batch's raw
 * amplitude A_p (without w_p q_p) of every particle into its own row, so
 * windows of one run must list the particles in the same order.  Leaves S and
 * A_s alone; samples with |beta| >= 1 or non-finite values are recorded for the
 * next read as in lw_accumulate.  Any path: the FP32 path needs no workspace
 * (workspace may be NULL), the matrix-core paths the lw_workspace_size bytes of
 * the same batch and path.  Asynchronous on the FP32 path. */
lw_status lw_accumulate_amplitudes(lw_ctx* ctx, const lw_batch* batch, lw_path path, void* workspace,
                                   size_t workspace_bytes, double* amp);
/* Device workspace (bytes) of lw_spectrum_from_amplitudes for n_particles. */
lw_status lw_amplitude_workspace_size(lw_ctx* ctx, int64_t n_particles, size_t* bytes);
/* Add the spectrum of a per-particle amplitude state into the accumulator:
 * S += sum_p w_p q_p^2 |amp_p|^2 / (4 pi^2) (incoherent) or A_s += sum_p w_p q_p
 * amp_p (coherent).  Only batch.n_particles, charge, weight and species are
 * read.  Call lw_reset first for the spectrum P(t) of the state alone.
 * Asynchronous; deterministic (fixed summation order). */
lw_status lw_spectrum_from_amplitudes(lw_ctx* ctx, const lw_batch* batch, const double* amp,
                                      void* workspace, size_t workspace_bytes);

/* ---- spectral diagnostics (Section 3.3; observers as in Section 2.2) ----
 * Observer-averaged spectrum and, per (species, observer) and for the average,
 * the peak and the low/high-frequency power-law indices:
 *   avg[s][j] = sum_d a_d S[s][d][j] / sum_d a_d  (a: host_weights [nd], a_d >= 0,
 *               NULL = equal weights);
 *   k = first index of the largest S over the frequency list; omega_peak = the
 *   vertex of the parabola through (ln w, ln S) at k-1, k, k+1 when it opens
 *   downwards (kept within [w_{k-1}, w_{k+1}]), else w_k;
 *   alpha, beta = least-squares slopes of ln S on ln w over the bins with S > 0
 *   and lo w_k <= w <= hi w_k; ranges = host {alpha_lo, alpha_hi, beta_lo,
 *   beta_hi} (NULL = {0.01, 0.3, 3, 30}); NaN with fewer than two bins.
 * S: device FP64 [n_species][nd][nw] (e.g. a snapshot difference), or NULL for the
 * context's current spectrum (|A_s|^2 / (4 pi^2) in coherent mode).
 * avg_out: host [n_species][nw] or NULL.  diag_out: host [n_species][nd + 1][8],
 * each row {k, w_k, omega_peak, S_k, alpha, n_alpha, beta, n_beta}, row nd being
 * the average's.  Synchronous; device errors of earlier calls are not reported here. */
lw_status lw_spectral_diagnostics(lw_ctx* ctx, const double* S, const double* host_weights,
                                  const double* ranges, double* avg_out, double* diag_out);

/* ---- pitch-cone selection (Section 3.2) ----
 * Particles whose momentum lies in narrow cones about inclinations theta_c[m] from the
 * streaming axis, against the whole ensemble, in gamma^2 bins:
 *   cos theta = |u . a| / |u| (u = gamma beta, a = host_axis normalised; the pitch angle
 *   folded to [0, pi/2], so both beams count; a particle at rest counts as on-axis);
 *   in cone m when cos(min(pi/2, theta_c[m] + dtheta)) <= cos theta <= cos(max(0,
 *   theta_c[m] - dtheta)); gamma^2 = 1 + |u|^2 in bin b when edges[b] <= gamma^2 <
 *   edges[b + 1] (outside the edges: not counted).
 * ux, uy, uz: device FP64 [n_particles].  host_theta_c [n_cones] (1..16 cones), dtheta > 0,
 * host_edges [n_bins + 1] increasing (1..256 bins).  Outputs (host): counts_out int64
 * [n_cones + 1][n_bins] (row n_cones: all particles); dev_out [n_cones][n_bins], the
 * relative deviation from isotropy (count share / isotropic share cos theta_lo -
 * cos theta_hi; NaN for an empty bin); member: NULL or device int32 [n_particles], the
 * first cone holding each particle or -1 (e.g. to synthesise one cone with
 * lw_accumulate_subset).  Counts are exact.  Synchronous. */
lw_status lw_pitch_cones(lw_ctx* ctx, int64_t n_particles, const double* ux, const double* uy,
                         const double* uz, const double* host_axis, const double* host_theta_c,
                         int32_t n_cones, double dtheta, const double* host_edges, int32_t n_bins,
                         int64_t* counts_out, double* dev_out, int32_t* member);

/* ---- batched launches (uneven lengths, several species) ----
 * Plan a batch for the persistent launch (synchronous; reads the batch offsets).
 * FP32 path: particles are ordered by decreasing trajectory length and grouped
 * into work items (particle block x direction x frequency tile) that a fixed
 * set of work-groups takes, heaviest first, from an atomic ticket queue.  Later
 * lw_accumulate calls with the same batch (same offsets pointer and size) and
 * the same grids use the plan; other batches use the plain grid launch.
 * Matrix-core paths: sizes the retarded-time grids and phase tables, so that
 * the following lw_accumulate / lw_graph_capture need no synchronisation. */
lw_status lw_plan_batch(lw_ctx* ctx, const lw_batch* batch, lw_path path);

/* Launch shape: wpt = frequencies per thread of the FP32 kernel (0 automatic,
 * 1, 2, 4, 8); pb = particles per work item (0 automatic); persistent = use a
 * matching lw_plan_batch plan (1) or always the plain grid (0); bands and the
 * contraction tile (rows x columns per work-group: LW_TILE_128x128,
 * LW_TILE_256x128, LW_TILE_128x256, LW_TILE_256x256, the default) for the
 * matrix-core path; 0 = unchanged.  A 256-row tile needs every band's row count
 * (2 x its frequencies, rounded up to 128) to be a multiple of 256; otherwise
 * the launch takes the 128-row tile of the same width.  LW_TILE_256x128 has no
 * coherent or amplitude-state epilogue: those launches take LW_TILE_128x256. */
enum { LW_TILE_128x128 = 1, LW_TILE_256x128 = 2, LW_TILE_128x256 = 3, LW_TILE_256x256 = 4 };
lw_status lw_set_tuning(lw_ctx* ctx, int32_t wpt, int32_t pb, int32_t persistent, int32_t bands,
                        int32_t tile);

/* Autotuner: time the candidate launch shapes of `path` on `batch` (repeats
 * timed runs each, HIP events on the context's stream), keep the fastest (as
 * with lw_set_tuning, plus lw_plan_batch when it is persistent) and restore S.
 * report (may be NULL): JSON text of every candidate's time and the choice,
 * truncated to report_len.  cache_json (may be NULL): file receiving the
 * same JSON.  Allocates and frees its own workspace. */
lw_status lw_tune(lw_ctx* ctx, const lw_batch* batch, lw_path path, int32_t repeats,
                  const char* cache_json, char* report, size_t report_len);

/* HIP graph of one lw_accumulate(batch, path, workspace): captured on a
 * private stream (so it also works when the context uses the null stream),
 * replayed on the context's stream by lw_graph_launch; each replay adds the
 * batch's spectrum into S like lw_accumulate.  The batch and workspace must
 * stay unchanged while the graph is in use.  The graph clears its counters with
 * kernels, not memset nodes.  lw_graph_launch returns LW_ESTATE (and launches
 * nothing) once the context's device buffers the graph refers to have been
 * freed or refilled since the capture: new grids or species (lw_set_directions,
 * lw_set_frequencies, lw_set_species, lw_set_coherent), a new lw_plan_batch
 * (also run by lw_tune), or rebuilt matrix-core tables (a batch with a longer
 * retarded-time span, other bands or products); capture again then. */
typedef struct lw_graph lw_graph;
lw_status lw_graph_capture(lw_ctx* ctx, const lw_batch* batch, lw_path path, void* workspace,
                           size_t workspace_bytes, lw_graph** out);
lw_status lw_graph_launch(lw_graph* graph);
void lw_graph_destroy(lw_graph* graph);

/* Particle subsets as batches of their own, so that any path (the matrix-core one
 * included) can sum a list of particles, e.g. the ones a surrogate defers to the exact
 * method (Section 2.2: the spectrum is a sum over particles, so any subset's sum is a
 * partial sum of the whole).
 * lw_subset_offsets: dst_offsets (device int64 [n + 1]) gets 0 and the running sums of the
 * lengths of the particles listed in `indices` (device int64 [n], each in [0, n_particles)
 * of `batch`); *host_total receives dst_offsets[n], the gathered batch's sample count.  An
 * index outside the batch (or a particle of negative length) is LW_EINVAL.  Synchronous;
 * LW_ESTATE inside graph capture.
 * lw_gather_particles: copies the listed particles' samples and per-particle values into
 * `dst`, a batch of n particles whose offsets hold lw_subset_offsets' result and whose
 * arrays (caller-owned, written here) hold that many samples; d(beta)/dt in the same
 * precision as `batch` (LW_BATCH_F64_ACCEL on both or neither); dst.species, when given,
 * gets the source's species (0 when the source has none).  Stream-ordered, no allocation;
 * n <= 2^31 - 1. */
lw_status lw_subset_offsets(lw_ctx* ctx, const lw_batch* batch, const int64_t* indices, int64_t n,
                            int64_t* dst_offsets, int64_t* host_total);
lw_status lw_gather_particles(lw_ctx* ctx, const lw_batch* batch, const int64_t* indices, int64_t n,
                              const lw_batch* dst);

/* Exact FP32 accumulation of the particles listed in `indices` (device int64
 * [n_indices], each in [0, n_particles)) of `batch`: as lw_accumulate on the
 * FP32 path restricted to those particles; per_particle (optional) keeps the
 * [n_particles][nd][nw] layout of the whole batch and is written only for the
 * listed particles.  Workspace: lw_workspace_size of a batch of n_indices
 * particles.  Used to judge and to stand in for the surrogate. */
lw_status lw_accumulate_subset(lw_ctx* ctx, const lw_batch* batch, const int64_t* indices,
                               int64_t n_indices, void* workspace, size_t workspace_bytes,
                               float* per_particle);

/* ---- learned surrogate (not part of the paper's method) ----
 * Features of every (particle, direction) pair: device float [n_particles][nd][16]
 * (log Lorentz factor and spread; transverse-acceleration mean, rms, max and
 * kurtosis; deflection in units of 1/gamma, rms and max; force reversals per
 * unit time and the jitter frequency scale; log duration; log of the energy
 * per unit solid angle radiated towards n, the Riemann sum of
 * |n x ((n - beta) x betadot)|^2 / kappa^5 dt / (4 pi) (Jackson eq. 14.38, equal
 * by Parseval to the frequency integral of the spectrum), plus 1e-30;
 * observer angle to the mean velocity times gamma; log mean and min kappa;
 * fraction of samples with the observer inside the 1/gamma cone). */
lw_status lw_features(lw_ctx* ctx, const lw_batch* batch, float* feats);

/* Add the surrogate's predicted spectra to S: ylog = device [n_particles][nd][nw]
 * log10 of each particle's own spectrum (without w q^2); calib (may be NULL) =
 * device [nd][nw] log10 correction added to every particle's ylog; err = device
 * [n_particles][nd] predicted error or NULL.  Particles whose error exceeds
 * `threshold` in any direction (or is NaN) get flags[p] = 1 (device int32
 * [n_particles]) and are left out, for lw_accumulate_subset to add exactly; the
 * others add w_p q_p^2 10^(ylog + calib) to their species.  Fixed-order reduction.
 * flagged, n_flagged (device int64 [n_particles] and [1], both or neither): the
 * flagged particle indices in increasing order and their count.  Workspace:
 * ceil(n_particles / 128) x n_species x nd x nw doubles; at most 65535 x 256
 * (direction, frequency) columns per call (LW_ERANGE beyond). */
lw_status lw_surrogate_accumulate(lw_ctx* ctx, const lw_batch* batch, const float* ylog,
                                  const float* calib, const float* err, float threshold, int32_t* flags,
                                  int64_t* flagged, int64_t* n_flagged, void* workspace,
                                  size_t workspace_bytes);

/* Training targets from the exact kernel's per-particle output (lw_accumulate's
 * per_particle array, device [n_particles][nd][nw]): out = log10(pp / (w q^2) +
 * floor_value), device float of the same shape; floor_value > 0. */
lw_status lw_surrogate_targets(lw_ctx* ctx, const lw_batch* batch, const float* per_particle,
                               double floor_value, float* out);

/* Calibration statistics of the surrogate, on the device (the training set-up of the
 * learned surrogate: input normalisation, the per-direction mean spectrum, the error-head
 * targets, the fallback threshold and the per-bin calibration).
 *
 * lw_column_stats: x = device FP32 [rows][cols], row r = p groups + g of particle p and
 * group g (rows a multiple of groups, groups <= 65535, rows / groups <= 65535 x 256).  For
 * each group and column, out (device double [groups][cols][2]) = mean and mean square of
 * v = x[r][j] + row_add_coeff row_add[r row_add_stride] (row_add may be NULL), or of 10^v
 * when exp10 != 0, over the kept particles: all of them when err is NULL, else those whose
 * largest err[p][g'] (device FP32 [rows]) is <= threshold (zeros when none is kept).  FP64
 * sums in a fixed order.  Workspace: ceil(P / 256) x groups x cols x 3 doubles
 * (LW_ENOMEM if smaller; the needed size is in the error text). */
lw_status lw_column_stats(lw_ctx* ctx, const float* x, int64_t rows, int32_t cols, int32_t groups,
                          const float* row_add, int64_t row_add_stride, double row_add_coeff, int32_t exp10,
                          const float* err, float threshold, double* out, void* workspace,
                          size_t workspace_bytes);

/* Error-head target of each row (surrogate pair): share[r] = log10(mean_j |10^pred[r][j] -
 * 10^y[r][j]| / smean[((r mod groups) cols + j) smean_stride] + floor_value), the pair's
 * share in the error of the summed spectrum.  pred, y = device FP32 [rows][cols]; smean =
 * device double (e.g. the means of lw_column_stats with stride 2); share = device FP32 [rows]. */
lw_status lw_error_share(lw_ctx* ctx, const float* pred, const float* y, int64_t rows, int32_t cols,
                         int32_t groups, const double* smean, int64_t smean_stride, double floor_value,
                         float* share);

/* q-quantile (0 <= q <= 1; linear interpolation between the order statistics around
 * q (n - 1)) of the per-particle maxima max_g v[p][g] of v = device FP32 [n][groups]; NaN
 * counts as the largest value.  Exact: the order statistics are selected by four byte-wise
 * histogram passes over order-preserving keys (each pass synchronises the stream).  Result
 * in *host_out.  Workspace: ceil(4 n / 256) x 256 + 1280 bytes. */
lw_status lw_quantile_of_maxima(lw_ctx* ctx, const float* v, int64_t n, int32_t groups, double q,
                                double* host_out, void* workspace, size_t workspace_bytes);

/* out[i] = log10(num[i num_stride] / den[i den_stride]) in FP32 where both are positive,
 * else 0, for i < n (device arrays): the per-bin calibration from two means. */
lw_status lw_log_ratio(lw_ctx* ctx, const double* num, int64_t num_stride, const double* den,
                       int64_t den_stride, int64_t n, float* out);

/* MLP n_in -> [Linear, GELU] x n_hidden -> Linear -> n_out, FP32 master weights,
 * products in BF16 on the matrix cores with FP32 accumulation, AdamW updates,
 * plus an error head (Linear on the last hidden layer -> 1).  Parameter layout:
 * per layer W [out][in] row-major then b [out].  x, t, y, err are device
 * [rows][width] FP32; the network allocates its activation workspace on first use
 * of a row count (and keeps it).  Loss: mean squared error over rows and outputs. */
typedef struct lw_mlp lw_mlp;
lw_status lw_mlp_create(lw_ctx* ctx, int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out,
                        uint64_t seed, lw_mlp** out);
void lw_mlp_destroy(lw_mlp* net);
lw_status lw_mlp_num_params(const lw_mlp* net, int64_t* count);
/* host_head (may be NULL): the error head's hidden + 1 parameters. */
lw_status lw_mlp_get_params(lw_mlp* net, float* host, int64_t count, float* host_head);
lw_status lw_mlp_set_params(lw_mlp* net, const float* host, int64_t count, const float* host_head);
/* Input normalisation applied in FP32 before the first product (so that
 * features with a large offset keep their resolution in BF16): the network
 * reads (x[k] - shift[k]) * scale[k].  shift, scale: host float [n_in], both
 * NULL to remove it.  Used by every later forward, gradient and training call. */
lw_status lw_mlp_set_input_norm(lw_mlp* net, const float* shift, const float* scale);
/* Output skip: every output gets coeff * x[input_index] (the raw input, before
 * the normalisation) added, in forward, gradient and training calls alike, so
 * the network learns the outputs relative to that input; input_index = -1
 * removes it. */
lw_status lw_mlp_set_output_skip(lw_mlp* net, int32_t input_index, float coeff);
/* y: device [rows][n_out]; err_head (may be NULL): device [rows], the error head's output.
 * Networks with a hidden width that is a multiple of 64, an output width a multiple of 32
 * (both at most 256), an input width a multiple of 8 (at most 256), 1 to 8 hidden layers and
 * 16-byte aligned x and y run as one kernel per tile of 128 rows: activations stay on chip, the
 * weights are rounded to BF16 once per call, and GELU's erf is a rational form within 1.5e-7
 * of erf.  Other shapes run layer by layer, as the training calls do.  Both keep the
 * roundings of the products (BF16 operands, FP32 accumulation). */
lw_status lw_mlp_forward(lw_mlp* net, const float* x, int64_t rows, float* y, float* err_head);
/* Loss and its gradient (copied to grad_host when not NULL), no update. */
lw_status lw_mlp_loss_grad(lw_mlp* net, const float* x, const float* t, int64_t rows, float* grad_host,
                           double* loss);
lw_status lw_mlp_train_step(lw_mlp* net, const float* x, const float* t, int64_t rows, float lr,
                            float weight_decay, double* loss);
/* One AdamW step of the error head towards err_target [rows] (main net frozen). */
lw_status lw_mlp_train_head_step(lw_mlp* net, const float* x, const float* err_target, int64_t rows,
                                 float lr, double* loss);
/* Write the network to `path`: a header ("LWMLP001", n_in, hidden, n_hidden, n_out,
 * parameter count, FNV-1a 64 checksum of what follows), then FP32 master
 * parameters, error-head parameters, AdamW first and second moments of both and
 * their step counts, the input normalisation (flag, shift, scale) and the output
 * skip (index, coefficient): everything a later process needs to infer or to
 * continue training.  Synchronises. */
lw_status lw_mlp_save(lw_mlp* net, const char* path);
/* Restore such a file into a network of the same shape (LW_EINVAL otherwise, or on
 * a short or corrupted file, leaving the network unchanged). */
lw_status lw_mlp_load(lw_mlp* net, const char* path);

/* Kernel timing with HIP events recorded on the context's stream around each
 * accumulation kernel launch (enable != 0 turns it on; off by default). */
lw_status lw_set_profiling(lw_ctx* ctx, int32_t enable);
/* Synchronise, then report and clear the timings gathered since the last read:
 * host_out[7] = {FP32 accumulation kernel ms, spreading kernel ms, matrix-core
 * contraction kernel ms, useful contraction FLOPs (2 x rows x columns x inner
 * length per particle, direction and band, times the number of products),
 * FP32 kernel launches, contraction kernel launches, spreading kernel launches}. */
lw_status lw_profile_read(lw_ctx* ctx, double* host_out);

/* Load balance of the last persistent FP32 launch made with profiling on (lw_plan_batch
 * plan in use): each work-group records the compute unit it ran on (XCC and hardware ids)
 * and its start and end on the device's real-time counter; a compute unit's busy time is
 * the sum over its work-groups of (end - start).  Several work-groups are resident on one
 * compute unit at once, so a busy time is about that residency times the launch's duration;
 * the spread of busy times across units is the load-balance figure.  Synchronises.
 * host_out[4] = {compute units seen, min, mean, max busy ms}.  LW_ESTATE if no such launch
 * was made. */
lw_status lw_profile_cu_busy(lw_ctx* ctx, double* host_out);

/* Number of successful lw_accumulate calls since creation. */
lw_status lw_stats(const lw_ctx* ctx, int64_t* calls);

#ifdef __cplusplus
}
#endif
#endif /* LW_H */
