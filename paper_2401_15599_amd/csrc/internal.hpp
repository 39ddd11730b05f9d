// Internal declarations shared by the kernels and the host library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plans.hpp"

namespace tacaw {

constexpr int kWaves = 4;              // wavefronts per workgroup in every FFT kernel
constexpr int kThreads = 64 * kWaves;
constexpr int kMaxSpecies = 8;

// Per-job view used by the multislice kernels (device memory; built by the host per call).
struct MsJobDev {
  const float* V;          // [T][S][ny][nx]
  float2* W;               // [T][P][ny][nx]   forward working buffer / exit waves
  float2* ckpt;            // [T][P][nck][ny][nx] or null
  const float2* px;        // [S][nx] exp(-i pi lambda dz_s kx^2)
  const float2* py;        // [S][ny] exp(-i pi lambda dz_s ky^2)
  const int* nmax;         // [nx] band limit: column m keeps signed ky index n with |n| <= nmax[m]
  const int* nap;          // [nx] probe aperture, same convention
  const double* pxy;       // [P][2] probe positions
  float2* adj;             // [T][P][ny][nx] adjoint state
  float2* rec;             // [T][P][ny][nx] forward recompute buffer
  float2* stash;           // [T][P][K][ny][nx] pre-transmission real-space waves of one segment
  const float2* gexit;     // [T][P][ny][nx]
  float* gV;               // [T][S][ny][nx]
  float2* entr;            // [P][ny][nx] probe entrance waves shared by all snapshots (batched
                           // forward), or null
  int T, P, S, nx, ny;
  int kxb;                 // band-limited columns: kx index m is kept by some ky iff
                           // m <= kxb or m >= nx - kxb (nx/2 without a band limit)
  int ck_stride, n_ck, stash_k;
  float sigma;
  float scale_mid, scale_last, scale_probe;
  double lx, ly, lambda, defocus, cs;
};

// BUF_ENTR: a probe job's entrance wave of position (wave mod P) when the job has them, else BUF_W
enum Buf : int { BUF_W = 0, BUF_REC = 1, BUF_ADJ = 2, BUF_GEXIT = 3, BUF_CKPT = 4, BUF_ENTR = 5 };

__host__ __device__ inline size_t img_off(int wave, int nx, int ny) {
  return (size_t)wave * (size_t)nx * (size_t)ny;
}

struct RowArgs {
  const MsJobDev* jobs;
  const int2* groups;      // (job, t), sorted by S descending
  int n_groups;            // active prefix
  int s;                   // slice
  int in_buf, out_buf;     // Buf codes; BUF_CKPT as input reads checkpoint s / ck_stride
  int store_ckpt;          // forward: store the input row to the checkpoint of slice s
  int stash_slot;          // >= 0: store psi_s (real space) into stash slot
  int write_out;           // 0: skip the forward x-transform and the store
  int ny;                  // rows per image (all jobs of a launch share nx, ny)
  int band_in;             // the input is zero in the columns outside the band: not read
  int band_out;            // the consumer ignores columns outside the band: not written
  int prune;               // band_in and band_out hold and the band leaves out the two middle
                           // registers of the plan (kx index N/2 - L .. N/2 + L - 1) in every job:
                           // the transforms skip them (forward kernel, plans with E >= 8)
  int single_pos;          // every job of the launch has one wave per snapshot (P = 1): the
                           // forward kernel evaluates the transmission where it applies it
};

struct ColArgs {
  const MsJobDev* jobs;
  const int4* waves;       // (job, t, p, -), sorted by S descending
  int n_waves;             // active prefix
  int s;                   // slice whose propagator is applied
  int in_buf, out_buf;
  int conj_prop;           // apply conj(M P_s) (adjoint) instead of M P_s
  int C;                   // columns per tile
  float scale;             // 1/(nx ny), 1/sqrt(nx ny), ...
  int nx;                  // columns per image (all jobs of a launch share nx, ny)
  int pingpong;            // block kernel: two LDS exchange regions (one barrier per exchange);
                           // 2: also the split-layout transforms where the plan has them
  // Column tiles visited per wave: the first tiles_lo and the last tiles_hi of nx / C (both 0: all).
  // Tiles left out hold only columns outside every job's band; they are neither read nor written.
  // Inside visited tiles, a column outside its job's band is taken as zero (its output is zero
  // whatever the input, since M vanishes on the whole column).
  int tiles_lo, tiles_hi;
  int prune;               // M vanishes for ky index N/2 - L .. N/2 + L - 1 in every column of
                           // every job: the y transforms skip those two middle registers
                           // (block and wave-per-column kernels, plans with E >= 8)
};

// plain batched 2-D transforms of contiguous images (potential build, position gradient)
struct PlainArgs {
  const void* in;
  void* out;
  int n_img, nx, ny, C;
  // inverse transform of band-limited maps: columns kxb < m < nx - kxb and rows kyb < n < ny - kyb
  // are zero on input and are neither read nor transformed (-1: no band)
  int kxb = -1, kyb = -1;
  // inverse transform to real maps, two at a time: maps 2p and 2p + 1 (Hermitian spectra A, B)
  // are transformed as A + iB, whose real and imaginary parts are the two real maps (only for
  // spectra without Nyquist terms, whose missing partners would leak into the other map)
  int pair = 0;
  // slice maps without atoms (CSR offsets [t][S * nsp + 1]; map m is slice m % S of snapshot
  // t0 + m / S) are written as exact zeros instead of their partner's rounding residue
  const int* csr = nullptr;
  int csr_t0 = 0, csr_S = 1, csr_nsp = 1;
  // forward transform of real maps: rows of the result written (0: all); the column band kxb then
  // selects the column tiles that are transformed and written
  int rows_out = 0;
  // forward transform: per-map maximum of |Re| and |Im| over the written part of the result
  // (raised with atomic maxima on the float bits; the caller zeroes it first), or null
  float* absmax = nullptr;
};

// -------- launchers (defined in the .hip files) --------
int n_plans(int n);
const char* plan_name(int n, int idx);
hipError_t launch_row(int n, int plan, bool adj, const RowArgs& a, int grid, hipStream_t st);
// kind 0: LDS-staged tile, whole columns per wavefront; kind 1: block kernel, lanes of a column
// spread over the workgroup (C * L threads), tile loaded straight into registers
hipError_t launch_col(int n, int plan, int kind, bool dofwd, bool doinv, const ColArgs& a, int grid,
                      hipStream_t st);
int col_block_lds_bytes(int n, int plan, int C, int pingpong);
int col_block_max_threads(int n, int plan);   // launch bound of the block kind (C * L threads)
bool plan_prunable(int n, int plan, int kb);
// kind 2: LDS-staged tile, one line per wavefront lane group, C * 64 / LINES threads
int col_wave_lds_bytes(int n, int plan, int C);
int col_wave_threads(int n, int plan, int C);
int plan_lanes(int n, int plan);
hipError_t launch_probe_init(int n, int plan, const ColArgs& a, int grid, hipStream_t st);
hipError_t launch_plane_init(const ColArgs& a, int grid, hipStream_t st);
// waves (job, t, p) := wave (job, 0, p) of the same buffer (entrance waves of probe jobs)
hipError_t launch_wave_copy(const ColArgs& a, int grid, hipStream_t st);
// resident slice loop of small square grids (whole wave per workgroup, every slice on the CU):
// available grids, workgroups per CU, launch over a class's S-sorted wave list (a.scale = 1/(n n))
bool resident_ok(int nx, int ny);
int resident_workgroups_per_cu(int n, int max_lds);
hipError_t launch_resident(int n, const ColArgs& a, int grid, hipStream_t st);
int row_lines_per_wave(int n, int plan);
int col_lds_bytes(int n, int plan, int C);
// grid lengths with FFT plans; the root-table LDS of a plan; y-pass kinds a plan supports
bool grid_size_ok(int n);
int plan_static_lds(int n, int plan);
bool plan_kind_ok(int n, int plan, int kind);
int col_block_lx_cols(int n, int plan);   // 0: no split-layout transforms

// potentials
hipError_t launch_bin_atoms(const float* xyz, const int* species, int n_snap, int n_atoms,
                            int n_species, const double* bounds, int S, int* offsets, int* order,
                            int* n_out, hipStream_t st);
struct SfArgs {
  const float* xyz; const int* order; const int* offsets; const float* ff;  // ff: [nsp][12] f32
  float2* vk;              // [maps][ny][nx]
  int t0, s_count, n_atoms, n_species, nx, ny;  // maps = (t0 + i / S, i % S)
  double lx, ly;
  float pref;              // 2 pi a0 e / (Lx Ly)
  float kmax2;             // band limit in (1/A)^2 for |k|^2 (float comparison only for tile skip)
  const int* nmax;         // [nx] exact band-limit table
  int n_maps;
  void* arec;              // workspace: 24-byte phase record per (snapshot of the pass, atom)
  int hermitian;           // compute ky >= 0 only and write the conjugate reflection
  int split16;             // fp16 hi/lo split operands on the f16 matrix cores (else fp32 MFMA)
  // quarter-plane kernel: tiles of a map in launch order, those with kept k first (n_live of
  // them), so that consecutive workgroups (dealt round-robin to the XCDs) share the live work
  const int* tile_order;
  int n_live;
};
hipError_t launch_structure_factor(const SfArgs& a, hipStream_t st);
hipError_t launch_ifft2_real(int nx, int ny, float2* vk, float* V, int n_img, int kxb, int kyb,
                             int pair, const int* csr, int t0, int S, int nsp, hipStream_t st);
// forward 2-D DFT of real maps where only the band |kx index| <= kxb (kxb >= nx / 2: all columns)
// and the rows n < rows_out are wanted: columns of width-C tiles without a kept column are left
// unwritten, the other columns outside the band hold zeros, rows from rows_out on are unwritten.
// absmax (n_img floats, zeroed by the caller, or null) receives each map's maximum of |Re| and
// |Im| over the band and the written rows.
hipError_t launch_fft2_real(int nx, int ny, const float* g, float2* gk, int n_img, int kxb,
                            int rows_out, float* absmax, hipStream_t st);
struct PgArgs {
  const float* xyz; const int* order; const int* offsets; const float* ff;
  const float2* gk;        // [maps][ny][nx] DFT of dL/dV
  float* gxy;              // [T][N][2]
  int t0, s_count, n_atoms, n_species, nx, ny, n_maps;
  double lx, ly;
  float pref;
  const int* nmax;
  void* arec;              // per-atom phase records of the pass (CSR order)
  int hermitian;           // visit ky >= 0 only (band limit on)
  const float* vtab;       // [n_species][ny_h][nx] pref M(k) f_Z(|k|) w(k) (ny_h = ny/2 or ny)
  float hbound;            // max over vtab of |v| max(1, |ky|)
  const float* absmax;     // [n_maps] max |Re G|, |Im G| over the band and the visited rows
  // [kx tile][ky fill of 32 rows]: 1 when some k of it passes the band limit (64-wide kx tiles,
  // fills of the visited rows), from the exact band table on the host
  const int* fill_live;
};
hipError_t launch_atom_phase(const float* xyz, const int* order, int t0, int nt, int n_atoms,
                             double lx, double ly, void* rec, hipStream_t st);
hipError_t launch_position_grad(const PgArgs& a, hipStream_t st);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t st);

// spectrum
struct SpecArgs {
  const float2* exit;      // [T][Ps][nq]; positions p0 .. p0 + Pn - 1 are used
  float* P;                // [n_e][nq]
  int T, Pn, nq, n_e, hop, G, accumulate, Qt;
  int Ps, p0;              // positions per snapshot in memory, first position used
};
hipError_t launch_periodogram(const SpecArgs& a, hipStream_t st);
struct FinArgs {
  const float* P; const float* K;   // K: [n_e] DFT order
  float* S; double* partial; double* norm;
  int n_e, nx, ny, nqx, nqy, n_part;
};
hipError_t launch_finalize(const FinArgs& a, hipStream_t st);
hipError_t launch_kubo_fill(float* K, int n_e, double dt_fs, double beta, hipStream_t st);

// analysis outputs (patterns, line profiles, dispersion cuts)
hipError_t launch_energy_sums(const float* P, const float* K, int n_e, long nq, double* sp,
                              double* skp, hipStream_t st);
hipError_t launch_snapshot_sums(const float2* exit, int n_pos, long nq, int t0, int ts, int count,
                                double* s, hipStream_t st);
// x / (fixed-order total of x over nq), centred and cropped; partial: n_part + 1 doubles
hipError_t launch_norm_crop(const double* x, long nq, int nx, int ny, int nqx, int nqy,
                            double* partial, int n_part, float* out, hipStream_t st);
hipError_t launch_rel_diff_row(const float* A, const float* B, int nqx, int nqy, float* out,
                               hipStream_t st);
hipError_t launch_scale(float* x, long n, float s, hipStream_t st);
hipError_t launch_path_cut(const float* S, int n_e, int nqx, int nqy, const double2* uv, int n_pts,
                           float* out, hipStream_t st);
struct SpecBwdArgs {
  const float2* exit; const float* S; const double* norm; const float* gS; const float* K;
  float2* gexit; double* partial;
  int T, Pn, nx, ny, nq, n_e, hop, G, nqx, nqy, Qt, n_part;
};
hipError_t launch_spectrum_backward(const SpecBwdArgs& a, hipStream_t st);

}  // namespace tacaw
