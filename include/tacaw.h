/* tacaw.h - C ABI of the time auto-correlation (TACAW) hot-path library for gfx950 (MI355X).
 *
 * The method (Castellanos-Reyes, Zeiger, Rusz, arXiv 2401.15599): the electron beam is propagated by
 * multislice through every snapshot tau(t) of a time-ordered atomic trajectory; the exit waves
 * phi(q, t) are stacked into a (qx, qy, t) dataset, Fourier transformed from time to energy, squared,
 * multiplied by the detailed-balance factor and normalised to a fractional intensity I(q, E).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: lengths in Angstrom, energies of the beam in eV, potentials in V*Angstrom (projected per
 *   slice), times in fs, temperatures in K.
 * Complex data: tacaw_c64 (interleaved float re, im).  Real data: float.  Positions: float x, y, z.
 * Grids: nx, ny are powers of two in [16, 1024], or 560 or 1000 (each axis independently; the
 * grids of the paper's Si/hBN and Fe runs); images are row-major [ny][nx] (x fastest).
 *   Reciprocal-space images use DFT storage order: index m holds kx = m/Lx for m < nx/2 and
 *   (m - nx)/Lx otherwise (likewise for y).
 * Memory: "dev" pointers are device memory on the context's GPU, owned by the caller (for instance
 *   torch tensors).  "host" pointers are read during the call only.  The library owns only its
 *   workspace inside the context.
 * Execution: every call is asynchronous on `stream` (a hipStream_t; NULL = the null stream) unless
 *   stated otherwise; results are ready when the stream reaches the call.
 * Errors: every call returns a tacaw_status.  Arguments are validated before any launch, so an
 *   error other than TACAW_E_HIP leaves outputs unwritten.  tacaw_last_error() returns a message for
 *   the calling thread's last failure.  No C++ exception crosses this interface.
 * Threading: a context is not thread-safe; use one context per host thread.
 * Determinism: reductions use a fixed order (no floating-point atomics); repeated calls with the
 *   same inputs and the same tuning give bit-identical results.
 */
#ifndef TACAW_H
#define TACAW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } tacaw_c64;

typedef enum {
  TACAW_OK = 0,
  TACAW_E_ARG = -1,   /* null pointer, negative count, inconsistent sizes, unknown option */
  TACAW_E_SIZE = -2,  /* a size outside what the kernels support (grid, segment length, species) */
  TACAW_E_HIP = -3,   /* a HIP runtime call failed; message from tacaw_last_error() */
  TACAW_E_NOMEM = -4, /* workspace allocation failed */
  TACAW_E_STATE = -5  /* an object is unusable (wrong device, destroyed, or a finished stream) */
} tacaw_status;

typedef struct tacaw_ctx tacaw_ctx;

/* Library version (major*10000 + minor*100 + patch). */
int tacaw_version(void);

/* Create a context bound to HIP device `hip_device`; *out receives it.  The context owns a growing
 * workspace, the propagator/band-limit tables, cached launch plans and hipGraphs, and the FFT
 * schedule choices (see tacaw_autotune).  Errors: TACAW_E_ARG (out NULL), TACAW_E_HIP. */
int tacaw_create(int hip_device, tacaw_ctx** out);

/* Free the context and everything it owns.  Waits for the device to finish work that uses the
 * workspace.  NULL is accepted. */
void tacaw_destroy(tacaw_ctx* ctx);

/* Message of the calling thread's last failed call (empty string if none). */
const char* tacaw_last_error(void);

/* ----------------------------------------------------------------------------------------------
 * Problem description (the paper's statement of the problem: positions of all nuclei per
 * configuration, slices through the specimen on a numerical grid, beam energy and illumination,
 * time step and the (q, E) output grid).
 */
typedef struct {
  int32_t nx, ny;          /* grid: powers of two in [16, 1024], 560 or 1000 */
  double lx, ly;           /* orthorhombic cell, periodic in x and y (Angstrom) */
  int32_t n_slices;        /* S >= 1 */
  const double* dz;        /* host [S] slice thicknesses (Angstrom), > 0 */
  double z0;               /* entrance plane; slice s is [z_s, z_{s+1}), z_{s+1} = z_s + dz[s] */
  double bandlimit;        /* band limit as a fraction of min(nx/(2lx), ny/(2ly)); <= 0: none */
} tacaw_specimen;

typedef struct {
  double energy_ev;        /* beam energy (eV), > 0 */
  int32_t kind;            /* TACAW_PLANE_WAVE or TACAW_PROBE */
  double alpha_rad;        /* probe: convergence semi-angle (rad) */
  double defocus_a;        /* probe: defocus (Angstrom), chi = pi lambda df k^2 + pi Cs lambda^3 k^4 / 2 */
  double cs_a;             /* probe: spherical aberration (Angstrom) */
  int32_t n_pos;           /* number of probe positions P (1 for a plane wave) */
  const double* pos_xy;    /* host [P][2] probe positions (Angstrom); ignored for a plane wave */
} tacaw_beam;

enum { TACAW_PLANE_WAVE = 0, TACAW_PROBE = 1 };

/* Scalar relations used by the library (host, synchronous).
 * wavelength: lambda = hc / sqrt(E (2 m0c^2 + E)) (Angstrom);
 * interaction parameter: sigma = (2 pi / (lambda E)) (m0c^2 + E) / (2 m0c^2 + E) (rad / (V Angstrom));
 * energy axis: E_j = 2 pi hbar (j - n_e/2) / (n_e dt) (eV), j = 0..n_e-1 ascending, positive = loss
 * (first step of the paper's two-step procedure: E_min = 2 pi hbar / t_tot, E_max = pi hbar / dt). */
double tacaw_wavelength(double energy_ev);
double tacaw_interaction_parameter(double energy_ev);
int tacaw_energy_axis(int32_t n_e, double dt_fs, double* e_ev /* host [n_e] */);

/* ----------------------------------------------------------------------------------------------
 * Slice binning (textbook multislice slicing; the paper slices its specimens into hundreds of
 * slices in its multislice runs).
 * Atom j of snapshot t belongs to slice s when z_s <= z < z_{s+1}, decided in float64 with
 * z_0 = z0 and z_{s+1} = z_s + dz[s] accumulated in slice order.  Atoms outside [z_0, z_S) belong to
 * no slice and are dropped (counted in *n_outside).
 *   xyz       dev [n_snap][n_atoms][3] float positions
 *   species   dev [n_atoms] int32 in [0, n_species) (an atom with any other value is not binned
 *             and counts as outside the slab)
 *   offsets   dev out [n_snap][S*n_species + 1] int32: atoms of (t, s, Z) are
 *             order[t][offsets[t][s*n_species+Z] .. offsets[t][s*n_species+Z+1])
 *   order     dev out [n_snap][n_atoms] int32 atom indices, sorted by (slice, species, index)
 *   n_outside dev out [n_snap] int32 dropped atoms per snapshot, or NULL
 * Integer results; identical to any correct stable binning.  Errors: TACAW_E_ARG, TACAW_E_SIZE
 * (S * n_species > 16384). */
int tacaw_bin_atoms(tacaw_ctx* ctx, const tacaw_specimen* spec, int32_t n_snap, int32_t n_atoms,
                    const float* xyz, const int32_t* species, int32_t n_species, int32_t* offsets,
                    int32_t* order, int32_t* n_outside, void* stream);

/* Projected slice potentials of every snapshot.
 *   V_s(k) = (2 pi a0 e / (Lx Ly)) M(k) sum_{j in s} f_{Z_j}(|k|) exp(-2 pi i k.r_j),
 *   V_s(r) = Re sum_k V_s(k) exp(+2 pi i k.r) on the grid r = (x Lx/nx, y Ly/ny),
 *   f_Z(q) = sum_i a_i/(q^2 + b_i) + sum_i c_i exp(-d_i q^2),  2 pi a0 e = 47.8777 V Angstrom^2,
 *   M(k) = 1 when kx^2 + ky^2 < (bandlimit * kN)^2 (float64), else 0 (M = 1 if bandlimit <= 0).
 * The paper obtains the exit waves with ordinary multislice; this is that method's textbook potential.
 * The contraction over atoms runs on the matrix cores, by default with every phase factor split
 * into fp16 high and low parts (three f16 products per term, fp32 accumulation, error below
 * 2^-22 per unit phase product); tacaw_set_potential_precision selects plain fp32 operands.
 *   ff        host [n_species][12]: a1,b1,a2,b2,a3,b3,c1,d1,c2,d2,c3,d3 (q in 1/Angstrom)
 *   V         dev out [n_snap][S][ny][nx] float (V Angstrom)
 *   n_outside dev out [n_snap] int32 or NULL (as in tacaw_bin_atoms)
 * Errors: TACAW_E_ARG, TACAW_E_SIZE (grid, n_species > 8), TACAW_E_NOMEM, TACAW_E_HIP. */
int tacaw_build_potentials(tacaw_ctx* ctx, const tacaw_specimen* spec, int32_t n_snap,
                           int32_t n_atoms, const float* xyz, const int32_t* species,
                           int32_t n_species, const double* ff, float* V, int32_t* n_outside,
                           void* stream);

/* Gradient of a loss with respect to the atoms' lateral positions, given dL/dV (the adjoint of
 * tacaw_build_potentials at fixed slice membership):
 *   dL/dx_j = Re sum_k conj(G_s(k)) C M(k) f_Zj(|k|) (-2 pi i kx) exp(-2 pi i k.r_j),  G_s = DFT[dL/dV_s]
 * and likewise for y_j (dL/dz_j = 0: slice membership is piecewise constant in z).
 *   grad_V   dev [n_snap][S][ny][nx] float
 *   grad_xy  dev out [n_snap][n_atoms][2] float (atoms outside the slab get 0)
 * Errors as tacaw_build_potentials. */
int tacaw_build_potentials_backward(tacaw_ctx* ctx, const tacaw_specimen* spec, int32_t n_snap,
                                    int32_t n_atoms, const float* xyz, const int32_t* species,
                                    int32_t n_species, const double* ff, const float* grad_V,
                                    float* grad_xy, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Batched multislice: the second step of the paper's procedure - the beam is propagated through
 * every snapshot and the exit waves are accumulated into the dataset phi(qx, qy, t).
 *   psi_{s+1} = F^-1[ M P_s F[ exp(i sigma V_s) psi_s ] ],  P_s(k) = exp(-i pi lambda dz_s |k|^2)
 *   phi(q)    = M P_{S-1} F[ exp(i sigma V_{S-1}) psi_{S-1} ] / sqrt(nx ny)   (orthonormal)
 * with F the unnormalised DFT exp(-2 pi i k.r).  psi_0 is a plane wave 1/sqrt(nx ny), or a probe
 *   psi_0(k) ~ A(k) exp(-i chi(k)) exp(-2 pi i k.r_p),  A(k) = 1 iff lambda^2 (kx^2 + ky^2) <= alpha^2
 * (float64), normalised to sum_r |psi_0|^2 = 1.
 *
 * One call runs a batch of jobs; job j has its own specimen, beam, trajectory length and buffers.
 * Waves of the same snapshot (probe positions) share one read of V per slice.
 */
typedef struct {
  const tacaw_specimen* spec;
  const tacaw_beam* beam;
  int32_t n_snap;          /* T_j */
  const float* V;          /* dev [T_j][S][ny][nx] from tacaw_build_potentials */
  tacaw_c64* exit;         /* dev out [T_j][P][ny][nx]: phi(q, t) in DFT order (also the working buffer) */
  tacaw_c64* ckpt;         /* dev out [T_j][P][ceil(S/ckpt_stride)][ny][nx] checkpoints, or NULL */
} tacaw_ms_job;

enum {
  TACAW_MODE_PLAIN = 0,    /* one snapshot per launch sequence: 2 launches per slice per snapshot */
  TACAW_MODE_BATCHED = 1,  /* the waves of a grid class in blocks of consecutive snapshots (by
                              default about 192 MiB of band-limited wave data each, sized to stay
                              in the memory-side cache between the passes): each block runs all
                              of its slices, one launch per slice and pass over the block's waves,
                              successive blocks alternating between two streams forked from and
                              joined back into `stream` (tacaw_set_slice_blocking); the slice loop
                              is captured into a hipGraph once per call structure (shapes, slice
                              counts, band, schedule, blocking: not buffer addresses) and
                              replayed; at most 32 graphs are kept per context (least recently
                              used first out); a probe job's entrance waves are built once into
                              library workspace (P x ny x nx complex64 per probe job) and read by
                              the first slice of every snapshot */
  TACAW_MODE_PERSISTENT = 2 /* as BATCHED, with the grid classes of a call as concurrent branches of
                              the captured graph, and square classes of at most 128 points per
                              axis run by one launch of persistent workgroups: each keeps a whole
                              wave on its CU (registers and LDS) through all of that wave's
                              slices, reading only V and writing the checkpoints and the exit
                              wave, then takes the next wave of the class (any slice count) */
};

/* ckpt_stride: 0 = no checkpoints; k > 0 stores the wave entering slices 0, k, 2k, ... (the state
 * needed by tacaw_multislice_adjoint; k = ceil(sqrt(S)) bounds memory by 2 sqrt(S) images per wave).
 * Errors: TACAW_E_ARG, TACAW_E_SIZE, TACAW_E_NOMEM, TACAW_E_HIP. */
int tacaw_multislice(tacaw_ctx* ctx, int32_t n_jobs, const tacaw_ms_job* jobs,
                     int32_t ckpt_stride, int32_t mode, void* stream);

/* Adjoint multislice: given G_phi = dL/dRe(phi) + i dL/dIm(phi) (the PyTorch convention, i.e.
 * 2 dL/d conj(phi)) for every exit wave, accumulate dL/dV for every slice:
 *   chi_{S-1} = F^-1[conj(M P_{S-1}) G_phi] sqrt(nx ny),  dL/dV_s = -sigma Im(conj(chi_s) t_s psi_s),
 *   G_psi_s = conj(t_s) chi_s,  chi_{s-1} = F^-1[conj(M P_{s-1}) F[G_psi_s]],
 * summed over probe positions.  psi_s is recomputed segment by segment from the checkpoints written
 * by tacaw_multislice with the same ckpt_stride (so memory stays O(sqrt S) waves).
 *   jobs[j].V, .ckpt as in the forward call; .exit is not used.
 *   grad_exit  per job: dev [T_j][P][ny][nx] (read only)
 *   grad_V     per job: dev out [T_j][S][ny][nx] float (overwritten)
 * Errors as tacaw_multislice. */
int tacaw_multislice_adjoint(tacaw_ctx* ctx, int32_t n_jobs, const tacaw_ms_job* jobs,
                             int32_t ckpt_stride, const tacaw_c64* const* grad_exit,
                             float* const* grad_V, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Time auto-correlation spectrum (spectral decomposition, Kubo correction, convolution theorem and
 * fractional normalisation of the paper).
 *   Segment g covers snapshots g*hop .. g*hop+n_e-1, G = floor((T - n_e)/hop) + 1 (tail dropped).
 *   Phi_g(q, k) = sum_t phi(q, g hop + t) exp(-2 pi i k t / n_e)   (rectangular window, no padding)
 *   P(q, k) = (1/G) sum_g sum_p |Phi_g(q, k)|^2  (= DFT of the circular auto-correlation)
 *   E_k = 2 pi hbar k' / (n_e dt), k' = k - n_e for k >= n_e/2 (the Nyquist bin is a gain)
 *   K(E) = beta E / (1 - exp(-beta E)), K(0) = 1,  beta = 1/(k_B T)
 *   I(q, E) = K P / Z,  Z = sum over the full q grid and all n_e bins of K P
 * Output S[e][iy][ix] (float): energies ascending (bin e has k' = e - n_e/2), q centred (index i holds
 * the signed frequency i - nq/2) and cropped to nqy_out x nqx_out.
 */
typedef struct {
  double dt_fs;            /* snapshot spacing (fs) */
  double temperature_k;    /* > 0 */
  int32_t n_e;             /* segment length = energy bins, power of two in [16, 1024] */
  int32_t hop;             /* segment offset >= 1 */
  int32_t nqx_out, nqy_out;/* centred crop, 1..nx and 1..ny */
} tacaw_spectrum_opts;

/* Periodogram accumulation: P_acc[k][q] (+)= (1/G) sum_g sum_p |Phi_g(q, k)|^2 (DFT order, float).
 *   exit   dev [n_snap][n_pos][ny][nx]
 *   P_acc  dev [n_e][ny][nx] float; overwritten when accumulate == 0, added to otherwise (use this
 *          to sum probe positions processed in chunks).
 * Errors: TACAW_E_ARG, TACAW_E_SIZE (n_e; or nx * ny not a multiple of the q tile of the time
 * kernels: 128 for n_e = 16, 64 for 32, 32 for 64, 16 above), TACAW_E_HIP. */
int tacaw_periodogram(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap, int32_t n_pos,
                      const tacaw_c64* exit, int32_t n_e, int32_t hop, float* P_acc,
                      int32_t accumulate, void* stream);

/* The same periodogram over a sub-range of probe positions, pos0 .. pos0 + n_pos_used - 1, of an
 * exit stack [n_snap][n_pos][ny][nx]: one spectrum per probe position of a scan (n_pos_used = 1),
 * or positions accumulated chunk by chunk from one resident stack (accumulate = 1).
 * Errors: as tacaw_periodogram, TACAW_E_ARG for a position range outside the stack. */
int tacaw_periodogram_positions(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap,
                                int32_t n_pos, const tacaw_c64* exit, int32_t pos0,
                                int32_t n_pos_used, int32_t n_e, int32_t hop, float* P_acc,
                                int32_t accumulate, void* stream);

/* Streamed segment periodograms for trajectories too long to keep every exit wave (the paper's
 * paragraph on averaging over segments of one long trajectory, after the two-step procedure,
 * and the segment counts of its Si and Fe footnotes): exit waves arrive chunk by chunk in snapshot
 * order; the object keeps only the snapshots a not-yet-complete segment still needs (a window
 * of at most n_e + the largest chunk snapshots, in library-owned device memory), and adds each
 * segment's |Phi_g|^2 to P_acc as soon as its last snapshot has arrived.  Segments start at
 * multiples of hop (hop > n_e leaves gaps, like tacaw_periodogram).  finish scales P_acc by 1/G,
 * so that it equals tacaw_periodogram of the whole stack with G complete segments.
 *   create   P_acc dev [n_e][ny][nx] float, owned by the caller, written by push and finish
 *   push     exit dev [n_snap][n_pos][ny][nx], the next n_snap snapshots (copied; the caller may
 *            reuse its buffer once the stream has passed the copy)
 *   finish   n_segments (host out, may be NULL): G; no further push
 *   window   capacity and held snapshots of the window (host out, may be NULL)
 * Errors: TACAW_E_ARG, TACAW_E_SIZE (grid, n_e, q tile as tacaw_periodogram), TACAW_E_NOMEM,
 * TACAW_E_STATE (push or finish after finish; finish before a complete segment), TACAW_E_HIP. */
typedef struct tacaw_segstream tacaw_segstream;
int tacaw_segstream_create(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_pos, int32_t n_e,
                           int32_t hop, float* P_acc, tacaw_segstream** out);
int tacaw_segstream_push(tacaw_segstream* s, int32_t n_snap, const tacaw_c64* exit, void* stream);
int tacaw_segstream_finish(tacaw_segstream* s, int32_t* n_segments, void* stream);
int tacaw_segstream_window(const tacaw_segstream* s, int32_t* capacity, int32_t* held);
void tacaw_segstream_destroy(tacaw_segstream* s);

/* Kubo correction, normalisation, energy shift and q crop of an accumulated periodogram.
 *   S     dev out [n_e][nqy_out][nqx_out] float
 *   norm  dev out [1] double: Z, or NULL */
int tacaw_spectrum_finalize(tacaw_ctx* ctx, int32_t nx, int32_t ny, const float* P_acc,
                            const tacaw_spectrum_opts* opts, float* S, double* norm, void* stream);

/* tacaw_spectrum_finalize without any allocation, for callers that cannot allocate device memory
 * (code under hipGraph capture, tight serving loops): the same kernels, with the partial sums of
 * Z and the Kubo table (computed on the device) in a fixed 16 KiB scratch array that the library
 * holds once per GPU for the life of the process.  Supports every n_e of tacaw_spectrum_finalize
 * (<= 1024).  Calls no hipMalloc/hipFree, uploads no table and never trims the context caches.
 * Every call on one GPU uses that GPU's one scratch array: calls that overlap on one GPU (other
 * streams, other threads, other contexts) race and must be serialised by the caller.
 * Arguments, outputs and errors as tacaw_spectrum_finalize (TACAW_E_SIZE if n_e would not fit). */
int tacaw_spectrum_finalize_noalloc(tacaw_ctx* ctx, int32_t nx, int32_t ny, const float* P_acc,
                                    const tacaw_spectrum_opts* opts, float* S, double* norm,
                                    void* stream);

/* tacaw_periodogram (accumulate = 0) followed by tacaw_spectrum_finalize; P_acc lives in the
 * workspace. */
int tacaw_autocorr_spectrum(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap, int32_t n_pos,
                            const tacaw_c64* exit, const tacaw_spectrum_opts* opts, float* S,
                            double* norm, void* stream);

/* Adjoint of tacaw_autocorr_spectrum: from g = dL/dS (output grid) to G_phi (PyTorch convention):
 *   dL/dP = (K/Z)(g - sum(g S)),  G_phi(g hop + t) += (2/G) sum_k dL/dP(k) Phi_g(k) exp(+2 pi i k t/n_e)
 *   S, norm    the forward outputs (dev)
 *   grad_S     dev [n_e][nqy_out][nqx_out] float
 *   grad_exit  dev out [n_snap][n_pos][ny][nx] (snapshots in no segment get 0) */
int tacaw_autocorr_spectrum_backward(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap,
                                     int32_t n_pos, const tacaw_c64* exit,
                                     const tacaw_spectrum_opts* opts, const float* S,
                                     const double* norm, const float* grad_S,
                                     tacaw_c64* grad_exit, void* stream);

/* ----------------------------------------------------------------------------------------------
 * Analysis outputs of the spectra (the Si and hBN results paragraphs, Figs. 1 and 2).  Every sum runs in a fixed order
 * (float64, no atomics); maps are centred and cropped like the spectrum (index i holds the signed
 * frequency i - nq/2).  Asynchronous on `stream`; the library's workspace holds the per-q sums.
 * Errors: TACAW_E_ARG, TACAW_E_SIZE (n_e), TACAW_E_NOMEM, TACAW_E_HIP.
 *
 * Energy-integrated diffraction patterns of an accumulated periodogram (the method's patterns of
 * Fig. 1): c_tilde(q) = sum_k P(q, k) before the Kubo correction and c(q) = sum_k K(E_k) P(q, k)
 * after it, each divided by its total over the full nx x ny grid.  By Parseval's theorem the first
 * equals the QEP pattern of the same snapshots when the segments do not overlap.
 *   P_acc         dev [n_e][ny][nx] float, DFT order (tacaw_periodogram)
 *   opts          n_e, dt_fs, temperature_k and the crop nqx_out x nqy_out are used
 *   c_tilde, c    dev out [nqy_out][nqx_out] float; either may be NULL */
int tacaw_energy_integrals(tacaw_ctx* ctx, int32_t nx, int32_t ny, const float* P_acc,
                           const tacaw_spectrum_opts* opts, float* c_tilde, float* c,
                           void* stream);

/* QEP (quantum excitation of phonons) pattern: |phi(q)|^2 summed over the snapshots t0 + j t_stride
 * (j < t_count) and all probe positions, divided by its total over the full grid (the standard
 * frozen-snapshot average the paper compares against, e.g. 100 evenly spaced snapshots or all).
 *   exit  dev [n_snap][n_pos][ny][nx];  out dev [nqy_out][nqx_out] float */
int tacaw_qep_pattern(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap, int32_t n_pos,
                      const tacaw_c64* exit, int32_t t0, int32_t t_stride, int32_t t_count,
                      int32_t nqx_out, int32_t nqy_out, float* out, void* stream);

/* Line profile of Fig. 1: out[i] = (A - B) / (A + B) along the q_y = 0 row (index nqy / 2) of two
 * centred maps of the same crop; 0 where A + B = 0.
 *   A, B  dev [nqy][nqx] float;  out_row dev [nqx] float */
int tacaw_relative_difference(tacaw_ctx* ctx, int32_t nqx, int32_t nqy, const float* A,
                              const float* B, float* out_row, void* stream);

/* Dispersion cut of Fig. 2: S(q, E) along the polyline through `vertices` (host [n_vert][2],
 * (qx, qy) in 1/Angstrom, n_vert >= 2): n_per_seg points per segment starting at its first vertex,
 * then the last vertex, so n_pts = (n_vert - 1) n_per_seg + 1.  Each point is sampled bilinearly at
 * the fractional pixel (qx lx + nqx/2, qy ly + nqy/2) of the centred map; pixels outside the map
 * count as zero.
 *   S    dev [n_e][nqy][nqx] float (tacaw_spectrum_finalize output)
 *   out  dev [n_e][n_pts] float */
int tacaw_path_cut(tacaw_ctx* ctx, double lx, double ly, int32_t nqx, int32_t nqy, int32_t n_e,
                   const float* S, int32_t n_vert, const double* vertices, int32_t n_per_seg,
                   float* out, void* stream);

/* ----------------------------------------------------------------------------------------------
 * FFT schedule autotuning (the kernels' radix plan, lanes per line and columns per LDS tile).
 * Times every compiled variant of the slice-step kernels for grid n (nx = ny = n) on a scratch batch
 * of `n_waves` waves with HIP events, keeps the fastest per (n, pass) in the context and, when
 * cache_path is not NULL, merges the choice into that JSON file (read back by tacaw_load_tuning).
 * Synchronous (waits for the device).  Errors: TACAW_E_SIZE, TACAW_E_NOMEM, TACAW_E_HIP. */
int tacaw_autotune(tacaw_ctx* ctx, int32_t n, int32_t n_waves, const char* cache_path,
                   void* stream);
/* Load tuning choices previously written by tacaw_autotune (host, synchronous).  One JSON object
 * per line: {"n": grid, "row": x-pass plan, "col": y-pass plan, "C": columns per tile (power of
 * two <= 64 dividing n), "kind": y-pass kernel (0 staged, 1 workgroup-exchange block, 2
 * wave-per-column; 2 only for plans whose lines fill a wavefront, i.e. not for 560 and 1000),
 * "pp": ping-pong exchange buffers of kind 1 (0/1; 2: ping-pong and the split-layout transforms,
 * one workgroup barrier per transform, only for the 512-point plan 8x8x8 with C a multiple of 8)}.
 * C is reduced at launch to what divides the image width and fits the workgroup and the LDS (a
 * split request whose reduced C is no longer a multiple of 8 runs pp 1); a wave-per-column
 * request that no width can serve runs the staged kind.  A missing file is not an error.
 * Errors: TACAW_E_ARG (malformed file). */
int tacaw_load_tuning(tacaw_ctx* ctx, const char* cache_path);
/* Number of compiled FFT plans (radix chains and lanes per line) for grid size n, 0 if none. */
int tacaw_plan_count(int32_t n);
/* Current schedule for grid n as text ("row=<plan> col=<plan> C=<cols>"), for logging. */
const char* tacaw_describe_schedule(tacaw_ctx* ctx, int32_t n);

/* ----------------------------------------------------------------------------------------------
 * Kernel timing instrumentation (for benchmarks and roofline reports).
 * With timing enabled, every slice-step launch (kinds "row", "col", "row_adj", "col_adj"), every
 * structure-factor launch ("sf"), potential inverse FFT ("pot_ifft"), periodogram ("pgram") and
 * position-gradient contraction of tacaw_build_potentials_backward ("pos_grad", no byte model) is
 * bracketed by HIP events recorded on the stream it runs on, and its algorithmic HBM bytes are
 * recorded: x pass 8 (wave in) + 8 (wave out) [+ 8 checkpoint] [+ 8 stash] per image element and
 * wave, plus 4 per element of each V row read once for all probe positions (8 with dL/dV); y pass
 * 16 per element and wave.  Batched multislice calls then launch eagerly instead of replaying
 * their hipGraph (the same kernels and grids).
 * tacaw_get_timing waits for the recorded events, sums launches, milliseconds and bytes of one kind
 * (all kinds for NULL or ""), and forgets them.  The library folds recorded pairs into per-kind sums
 * every 2048 launches (waiting for them), so that a call with many launches keeps few events alive;
 * timing is meant for eager calls, not for a stream the caller is capturing. */
typedef struct {
  int64_t launches;
  double total_ms;
  double algo_bytes;
} tacaw_kernel_stats;
int tacaw_set_timing(tacaw_ctx* ctx, int32_t enable);
/* Structure-factor operand precision for tacaw_build_potentials on this context:
 * 1 (default) fp16 hi/lo split on v_mfma_f32_32x32x16_f16, 0 fp32 v_mfma_f32_32x32x2f32.
 * Errors: TACAW_E_ARG (other values). */
int tacaw_set_potential_precision(tacaw_ctx* ctx, int32_t split16);
/* Blocking of the batched slice loop on this context (TACAW_MODE_BATCHED, and the classes of
 * TACAW_MODE_PERSISTENT that are not run by the resident kernel): block_bytes = band-limited wave
 * bytes (8 ny n_band per wave) per block of consecutive snapshots, 0 = one block per grid class;
 * streams = 1..3 streams that successive blocks alternate over (1 = the caller's stream only).
 * Blocking changes the launch order only, never the arithmetic: exit waves are bit-identical for
 * every setting.  Defaults 192 MiB and 2.  Errors: TACAW_E_ARG. */
int tacaw_set_slice_blocking(tacaw_ctx* ctx, int64_t block_bytes, int32_t streams);
int tacaw_get_timing(tacaw_ctx* ctx, const char* kind, tacaw_kernel_stats* out);

/* ----------------------------------------------------------------------------------------------
 * Context caches.  A context keeps device copies of the small host tables its calls derive
 * (propagator factors, band-limit and aperture tables, job tables, wave lists) keyed by content,
 * and the captured graphs of batched multislice calls.  When a call starts while the tables exceed
 * max_entries or max_bytes, the context waits for the device and drops every table and graph
 * (they are rebuilt on demand); tables are never dropped during a call.  Graphs beyond max_graphs
 * are dropped least recently used first, after their last replay has finished.
 * Defaults: 4096 tables, 256 MiB, 32 graphs.  Values < 1 are rejected (TACAW_E_ARG).
 * tacaw_cache_stats reports the current number of tables, their bytes and the number of graphs
 * (host out pointers, each may be NULL). */
int tacaw_set_cache_limits(tacaw_ctx* ctx, int64_t max_entries, int64_t max_bytes,
                           int32_t max_graphs);
int tacaw_cache_stats(tacaw_ctx* ctx, int64_t* n_tables, int64_t* table_bytes, int32_t* n_graphs);

#ifdef __cplusplus
}
#endif
#endif /* TACAW_H */
