// Slice binning, projected slice potentials and their adjoint with respect to atom positions.
//
// V_s(k) = pref M(k) sum_Z f_Z(|k|) sum_{j in (s, Z)} exp(-2 pi i kx x_j) exp(-2 pi i ky y_j)
// The phase factorises into an x table and a y table per atom, so each 64 x 64 tile of k-space is a
// small complex outer-product accumulation over the atoms of a slice (a GEMM-like contraction done
// on the vector ALUs from LDS-staged phase tables).  Phases use exact argument reduction: the
// fractional coordinate x/Lx is rounded to a 32-bit fixed-point number U, and the phase of index m
// is the wrapped integer product m*U (units of 2^-32 turns), so no large float argument ever
// reaches the sine/cosine.  Tiles outside the band limit are written as zeros without any work.
#include "internal.hpp"

namespace tacaw {

// ---------------------------------------------------------------------------------------------
// binning: one workgroup per snapshot, stable counting sort by key = slice * n_species + species.
// The NW wavefronts of a workgroup own contiguous atom ranges (wave w: [w R, (w + 1) R)) and a
// counter row each: counts per (wave, key), then a scan in (key, wave) order gives every wave its
// start position per key, then each wave scatters its range in order, 64 atoms at a time, ranking
// a lane among the lanes of equal key by matching the key bits with ballots.  The result is the
// stable order (ascending atom index within each key).
__device__ __forceinline__ int slice_of(float zf, const double* b, int S) {
  const double z = (double)zf;
  if (!(z >= b[0]) || !(z < b[S])) return -1;
  int lo = 0, hi = S;            // b[lo] <= z < b[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (b[mid] <= z) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(1024) void k_bin(const float* xyz, const int* species, int n_atoms,
                                              int nsp, const double* bounds, int S, int* offsets,
                                              int* order, int* n_out) {
  extern __shared__ int sh[];
  const int K = S * nsp, NW = (int)blockDim.x >> 6;
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int* cur = sh;                       // [NW][K] counts, then start positions
  int* part = sh + NW * K;             // [blockDim] scan partials and outside counts
  const float* X = xyz + (size_t)t * n_atoms * 3;
  const int R = (n_atoms + NW - 1) / NW;
  const int j0 = min(n_atoms, w * R), j1 = min(n_atoms, j0 + R);
  // key of atom j, or -1 outside the slab (or, for memory safety, with a species outside
  // [0, nsp))
  auto key_of = [&](int j) {
    const int sl = slice_of(X[3 * j + 2], bounds, S);
    const int z = species[j];
    return (sl < 0 || (unsigned)z >= (unsigned)nsp) ? -1 : sl * nsp + z;
  };
  for (int i = tid; i < NW * K; i += blockDim.x) cur[i] = 0;
  __syncthreads();
  int outside = 0;
  for (int j = j0 + lane; j < j1; j += 64) {
    const int key = key_of(j);
    if (key < 0) ++outside;
    else atomicAdd(&cur[w * K + key], 1);
  }
  part[tid] = outside;
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) tot += part[i];
    if (n_out) n_out[t] = tot;
  }
  __syncthreads();
  // exclusive scan over (key, wave): each thread owns a contiguous key range
  const int per = (K + blockDim.x - 1) / blockDim.x;
  const int a0 = min(K, tid * per), a1 = min(K, a0 + per);
  int local = 0;
  for (int k = a0; k < a1; ++k)
    for (int v = 0; v < NW; ++v) local += cur[v * K + k];
  part[tid] = local;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < (int)blockDim.x; ++i) { const int v = part[i]; part[i] = run; run += v; }
  }
  __syncthreads();
  int run = part[tid];
  int* off = offsets + (size_t)t * (K + 1);
  for (int k = a0; k < a1; ++k) {
    off[k] = run;
    for (int v = 0; v < NW; ++v) { const int c = cur[v * K + k]; cur[v * K + k] = run; run += c; }
  }
  if (tid == (int)blockDim.x - 1) off[K] = part[tid] + local;
  __syncthreads();
  // ordered scatter of each wave's range
  const int nbits = K > 1 ? 32 - __builtin_clz((unsigned)(K - 1)) : 0;
  const unsigned long long below = (1ull << lane) - 1ull;
  int* ord = order + (size_t)t * n_atoms;
  int* mycur = cur + w * K;
  for (int base = j0; base < j1; base += 64) {
    const int j = base + lane;
    const int key = j < j1 ? key_of(j) : -1;
    unsigned long long match = __ballot(key >= 0);
    for (int b = 0; b < nbits; ++b) {
      const unsigned long long bal = __ballot(key >= 0 && ((key >> b) & 1));
      match &= ((key >> b) & 1) ? bal : ~bal;
    }
    if (key >= 0) {
      const int rank = __popcll(match & below);
      ord[mycur[key] + rank] = j;
      // the highest lane of the group advances the cursor after every lane has read it
      if ((match >> lane) == 1ull) mycur[key] += rank + 1;
    }
  }
}

hipError_t launch_bin_atoms(const float* xyz, const int* species, int n_snap, int n_atoms,
                            int n_species, const double* bounds, int S, int* offsets, int* order,
                            int* n_out, hipStream_t st) {
  const int K = S * n_species;
  // as many wavefronts as keep their counter rows within 64 KB of LDS (K <= 16384 allows one)
  int nw = 16;
  while (nw > 1 && (long)nw * K * (int)sizeof(int) > 65536) nw /= 4;
  const int threads = 64 * nw;
  const int lds = (nw * K + threads) * (int)sizeof(int);
  hipFuncSetAttribute((const void*)k_bin, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  hipLaunchKernelGGL(k_bin, dim3(n_snap), dim3(threads), lds, st, xyz, species, n_atoms,
                     n_species, bounds, S, offsets, order, n_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// phase tables
__device__ __forceinline__ unsigned frac_fixed(float x, double len) {
  double u = (double)x / len;
  u -= floor(u);
  long long q = llrint(u * 4294967296.0);
  return (unsigned)(q & 0xffffffffLL);
}

__device__ __forceinline__ float form_factor(const float* f, float q2) {
  return f[0] / (q2 + f[1]) + f[2] / (q2 + f[3]) + f[4] / (q2 + f[5]) +
         f[6] * __expf(-f[7] * q2) + f[8] * __expf(-f[9] * q2) + f[10] * __expf(-f[11] * q2);
}

constexpr int kTile = 64;     // k-space tile edge (clamped to the grid)
constexpr int kChunk = 64;    // atoms staged per LDS fill

// Per-atom phase records in CSR order: fixed-point fractional coordinates and the exact phase
// factors of index 1 (the unit steps used to extend a block of phase factors).
struct AtomPhase {   // 24 bytes: fixed-point fractional x, y and unit phase steps
  unsigned ux, uy;
  float2 sx, sy;
};
static_assert(sizeof(AtomPhase) == 24 && alignof(AtomPhase) == 8, "phase record layout");

__global__ __launch_bounds__(256) void k_atom_phase(const float* xyz, const int* order, int t0,
                                                    int nt, int n_atoms, double lx, double ly,
                                                    AtomPhase* rec) {
  const long total = (long)nt * n_atoms;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < total; i += (long)gridDim.x * 256) {
    const int tl = (int)(i / n_atoms), p = (int)(i % n_atoms);
    const int aj = order[(size_t)(t0 + tl) * n_atoms + p];
    AtomPhase r;
    if (aj >= 0 && aj < n_atoms) {
      const float* X = xyz + ((size_t)(t0 + tl) * n_atoms + aj) * 3;
      r.ux = frac_fixed(X[0], lx);
      r.uy = frac_fixed(X[1], ly);
    } else {
      r.ux = r.uy = 0u;   // positions past the binned atoms of this snapshot (never read)
    }
    r.sx = phase_factor(1, r.ux);
    r.sy = phase_factor(1, r.uy);
    rec[i] = r;
  }
}

// One workgroup per (map, 64 x 64 k-tile), four wavefronts each owning a 32 x 32 quadrant.  The
// complex outer-product sum over the atoms of a slice is a GEMM with K = atoms (A = y phases down
// the quadrant's 32 ky, B = x phases across its 32 kx).  Phase tables for a chunk of atoms are
// generated once per workgroup in LDS.
//   SPLIT = false: fp32 operands, four v_mfma_f32_32x32x2f32 per atom pair.
//   SPLIT = true:  every phase component p is split as p = hi + lo with hi = fp16(p) (rounded
//                  toward zero) and lo = fp16(p - hi) (nearest); hi*hi + hi*lo + lo*hi accumulate in fp32
//                  by v_mfma_f32_32x32x16_f16 (the dropped lo*lo term is below 2^-22 for unit
//                  phases), twelve MFMAs per 16 atoms.
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __fp16 h2 __attribute__((ext_vector_type(2)));   // the packing builtin's type
typedef unsigned v4u __attribute__((ext_vector_type(4)));
// the fp16 pair (x0 - hi[0], x1 - hi[1]) rounded to nearest, hi being the packed fp16 high parts
// of x0 and x1: one mixed-precision fused multiply-add per half (x - hi is exact in fp32)
__device__ __forceinline__ h2 split_lo(float x0, float x1, h2 hi) {
  unsigned d;
  asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(d) : "v"(x0), "v"(hi));
  asm("v_fma_mixhi_f16 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "+v"(d) : "v"(x1), "v"(hi));
  return __builtin_bit_cast(h2, d);
}
constexpr int kSfChunk = 32;   // atoms per phase-table fill
// atom records staged per LDS batch (the next batch is in flight in registers)
template <bool SPLIT> constexpr int sf_batch() { return SPLIT ? 96 : 256; }
// Split tables: a (component, k) row holds the 32 atoms of a chunk in four 16-byte granules (8 atoms
// each).  Row r starts at 64 r bytes plus 64 bytes per preceding group of 8 rows, and its granules
// are permuted by XOR with h(r).  With 64 banks of 4 bytes (16 lanes per 16-byte read) or 32 banks
// (8 lanes per read), the operand reads (16 consecutive rows, one granule each) and the generator's
// stores (16 atom pairs x 4 rows 8 apart) both fill distinct banks.
__device__ __forceinline__ int row_h(int r) { return ((r >> 1) & 3) ^ ((r >> 3) & ~r & 1); }
__device__ __forceinline__ int split_at(int r, int granule) {   // halves from the table start
  return 32 * r + 32 * (r >> 3) + 8 * (granule ^ row_h(r));
}
constexpr int kTabH = 32 * kTile + 32 * (kTile / 8);   // halves per (axis, component) table

template <bool SPLIT>
__global__ __launch_bounds__(256) void k_structure_factor(SfArgs a) {
  // fp32 tables ex/ey [atom][k] (float2) or split tables [axis][component][k][atom] (fp16)
  constexpr int kBytesF32 = 2 * kSfChunk * (kTile + 1) * (int)sizeof(float2);
  constexpr int kBytesF16 = 2 * 4 * kTabH * (int)sizeof(_Float16);
  __shared__ __attribute__((aligned(16))) char tables[SPLIT ? kBytesF16 : kBytesF32];
  float2 (*ex)[kTile + 1] = reinterpret_cast<float2 (*)[kTile + 1]>(tables);
  float2 (*ey)[kTile + 1] = reinterpret_cast<float2 (*)[kTile + 1]>(tables) + kSfChunk;
  _Float16* tb = reinterpret_cast<_Float16*>(tables);   // [axis][component][split_at(k, atom / 8)]
  constexpr int kSfBatch = sf_batch<SPLIT>();
  __shared__ AtomPhase batch[kSfBatch];   // phase records of up to kSfBatch atoms of one species
  __shared__ float ffs[kMaxSpecies * 12];
  // Hermitian mode (band limit on, ny >= 128): only storage rows [0, ny/2) are computed; row
  // n > 0 is also written, conjugated, at (-n, -m); the Nyquist row is zero.
  const int herm = a.hermitian;
  const int tx_n = (a.nx + kTile - 1) / kTile;
  const int ty_n = herm ? (a.ny / 2 + kTile - 1) / kTile : (a.ny + kTile - 1) / kTile;
  const int tiles = tx_n * ty_n;
  const int map = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  if (map >= a.n_maps) return;
  const int TW = min(kTile, a.nx), TH = min(kTile, a.ny);
  const int m0 = (tile % tx_n) * TW, n0 = (tile / tx_n) * TH;
  // the last tile of an axis whose length is not a multiple of 64 is partial: kx < TWe, ky < THe
  // (rows below ny/2 only in Hermitian mode)
  const int TWe = min(TW, a.nx - m0), THe = min(TH, (herm ? a.ny / 2 : a.ny) - n0);
  const int t = a.t0 + map / a.s_count, s = map % a.s_count;
  const int tid = threadIdx.x;
  for (int i = tid; i < a.n_species * 12; i += 256) ffs[i] = a.ff[i];
  float2* out = a.vk + (size_t)map * a.nx * a.ny;
  auto put = [&](int n, int m, float2 v) {
    out[(size_t)n * a.nx + m] = v;
    if (herm && n > 0)
      out[(size_t)(a.ny - n) * a.nx + (a.nx - m) % a.nx] = make_float2(v.x, -v.y);
  };
  if (herm && n0 == 0)
    for (int m = m0 + tid; m < m0 + TWe; m += 256)
      out[(size_t)(a.ny / 2) * a.nx + m] = make_float2(0.f, 0.f);

  // does any k of this tile pass the band limit?  (exact integer table)
  int any = 0;
  {
    int minabs_n = 1 << 30;
    for (int n = n0; n < n0 + THe; ++n) {
      int ns = n < a.ny / 2 ? n : n - a.ny;
      minabs_n = min(minabs_n, ns < 0 ? -ns : ns);
    }
    for (int m = m0 + tid; m < m0 + TWe; m += 256) any |= (a.nmax[m] >= minabs_n);
  }
  any = __syncthreads_or(any);
  if (!any) {
    for (int i = tid; i < TWe * THe; i += 256) put(n0 + i / TWe, m0 + i % TWe, make_float2(0.f, 0.f));
    return;
  }

  const int lane = tid & 63, w = tid >> 6, wy = w >> 1, wx = w & 1;
  const int li = lane & 31, lk = lane >> 5;
  const int* off = a.offsets + (size_t)t * (a.s_count * a.n_species + 1);
  const AtomPhase* R = (const AtomPhase*)a.arec + (size_t)(t - a.t0) * a.n_atoms;
  // the species present in this slice; the sums of all but the last one pass through the output
  // (no per-species accumulators in registers)
  int zfirst = -1, zlast = -1;
  for (int z = 0; z < a.n_species; ++z)
    if (off[s * a.n_species + z + 1] > off[s * a.n_species + z]) {
      if (zfirst < 0) zfirst = z;
      zlast = z;
    }
  if (zlast < 0) {
    for (int i = tid; i < TWe * THe; i += 256) put(n0 + i / TWe, m0 + i % TWe, make_float2(0.f, 0.f));
    return;
  }
  const int tj = 32 * wx + li;
  // does any k of this wavefront's 32 x 32 quadrant pass the band limit?  A quadrant that does not
  // skips its matrix-core products (its outputs are all zero); the tables are still generated
  bool quad_live;
  {
    int minabs_q = 1 << 30;
    for (int n = n0 + 32 * wy; n < min(n0 + THe, n0 + 32 * wy + 32); ++n) {
      const int ns = n < a.ny / 2 ? n : n - a.ny;
      minabs_q = min(minabs_q, ns < 0 ? -ns : ns);
    }
    quad_live = __ballot(tj < TWe && a.nmax[m0 + min(tj, TWe - 1)] >= minabs_q) != 0ull;
  }
  for (int z = 0; z < a.n_species; ++z) {
    const int j0 = off[s * a.n_species + z], j1 = off[s * a.n_species + z + 1];
    if (j1 <= j0) continue;
    v16f cr = {0}, ci = {0};
    // the next batch's records travel in registers as three 8-byte words (a struct held in a
    // local variable would go through scratch memory and wait for the load at once)
    const uint2* Rw = reinterpret_cast<const uint2*>(R);
    uint2* bw = reinterpret_cast<uint2*>(batch);
    uint2 nr0 = make_uint2(0u, 0u), nr1 = nr0, nr2 = nr0;
    if (tid < kSfBatch && j0 + tid < j1) {
      nr0 = Rw[3 * (j0 + tid)];
      nr1 = Rw[3 * (j0 + tid) + 1];
      nr2 = Rw[3 * (j0 + tid) + 2];
    }
    for (int c0 = j0; c0 < j1; c0 += kSfChunk) {
      const int na = min(kSfChunk, j1 - c0);
      const int bi = (c0 - j0) % kSfBatch;    // chunk offset in the staged batch
      __syncthreads();                        // previous chunk's tables (and batch) are consumed
      if (bi == 0) {
        if (tid < kSfBatch) {
          bw[3 * tid] = nr0;                  // this batch (loaded one batch ahead)
          bw[3 * tid + 1] = nr1;
          bw[3 * tid + 2] = nr2;
          const int nb = c0 + kSfBatch + tid; // prefetch the next batch of this species
          if (nb < j1) {
            nr0 = Rw[3 * nb];
            nr1 = Rw[3 * nb + 1];
            nr2 = Rw[3 * nb + 2];
          }
        }
        __syncthreads();
      }
      const AtomPhase* arec = batch + bi;
      // blocks of 8 consecutive indices: exact factor at the block start, then 7 steps of the
      // atom's unit phase (aligned blocks never cross the +-N/2 wrap of the signed index)
      if constexpr (!SPLIT) {
        for (int i = tid; i < 2 * kSfChunk * (kTile / 8); i += 256) {
          const int axis = i / (kSfChunk * (kTile / 8));
          const int rem = i % (kSfChunk * (kTile / 8));
          const int at = rem / (kTile / 8), k0 = (rem % (kTile / 8)) * 8;
          float2* dst = axis == 0 ? &ex[at][k0] : &ey[at][k0];
          const int lim = axis == 0 ? TWe : THe;
          if (at >= na || k0 >= lim) {
#pragma unroll
            for (int q = 0; q < 8; ++q) dst[q] = make_float2(0.f, 0.f);
            continue;
          }
          const int nn = axis == 0 ? a.nx : a.ny;
          const int idx = (axis == 0 ? m0 : n0) + k0;
          const int sidx = idx < nn / 2 ? idx : idx - nn;
          const int qw = nn / 2 - idx;      // the signed index jumps to -nn/2 at step qw
          const AtomPhase& ap = arec[at];
          const unsigned U = axis == 0 ? ap.ux : ap.uy;
          float2 f = phase_factor(sidx, U);
          const float2 st = axis == 0 ? ap.sx : ap.sy;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            if (q == qw) f = phase_factor(idx + q - nn, U);
            dst[q] = f;
            f = cmul(f, st);
          }
        }
      } else {
        // one item per thread: (axis, block of 8 k, atom pair); components stored as packed
        // (atom 2p, atom 2p+1) half pairs
        const int axis = tid >> 7, k0 = ((tid >> 4) & 7) * 8, pair = tid & 15;
        const int lim = axis == 0 ? TWe : THe;
        const int nn = axis == 0 ? a.nx : a.ny;
        const int idx = (axis == 0 ? m0 : n0) + k0;
        const int sidx = idx < nn / 2 ? idx : idx - nn;
        // the signed index jumps to -nn/2 at step qw; only a length with nn/2 not a multiple of 8
        // has a block that straddles the jump (then the factor is restarted exactly there)
        const int qw = nn / 2 - idx;
        const bool wraps = qw > 0 && qw < 8;
        float2 f[2], st[2];
        unsigned Ua[2];
        bool live[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int at = 2 * pair + u;
          live[u] = at < na && k0 < lim;
          Ua[u] = 0u;
          if (live[u]) {
            const AtomPhase& ap = arec[at];
            Ua[u] = axis == 0 ? ap.ux : ap.uy;
            f[u] = phase_factor(sidx, Ua[u]);
            st[u] = axis == 0 ? ap.sx : ap.sy;
          } else {
            f[u] = make_float2(0.f, 0.f);
            st[u] = make_float2(0.f, 0.f);
          }
        }
        // hi = fp16 of p rounded toward zero (packed for the atom pair), lo = fp16(p - hi); p - hi
        // is exact in fp32 and |lo| < one fp16 ulp of p
        _Float16* row = tb + axis * 4 * kTabH + 2 * (pair & 3);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (wraps && q == qw) {
#pragma unroll
            for (int u = 0; u < 2; ++u)
              if (live[u]) f[u] = phase_factor(idx + q - nn, Ua[u]);
          }
          const h2 rh = __builtin_amdgcn_cvt_pkrtz(f[0].x, f[1].x);
          const h2 ih = __builtin_amdgcn_cvt_pkrtz(f[0].y, f[1].y);
          const h2 rl = split_lo(f[0].x, f[1].x, rh);
          const h2 il = split_lo(f[0].y, f[1].y, ih);
          _Float16* dst = row + split_at(k0 + q, pair >> 2);
          *reinterpret_cast<h2*>(dst) = rh;
          *reinterpret_cast<h2*>(dst + kTabH) = ih;
          *reinterpret_cast<h2*>(dst + 2 * kTabH) = rl;
          *reinterpret_cast<h2*>(dst + 3 * kTabH) = il;
          f[0] = cmul(f[0], st[0]);
          f[1] = cmul(f[1], st[1]);
        }
      }
      __syncthreads();
      if (!quad_live) {
        // no kept k in this quadrant
      } else if constexpr (!SPLIT) {
        const int npair = (na + 1) >> 1;
        for (int p = 0; p < npair; ++p) {
          const float2 yv = ey[2 * p + lk][32 * wy + li];
          const float2 xv = ex[2 * p + lk][32 * wx + li];
          cr = __builtin_amdgcn_mfma_f32_32x32x2f32(yv.x, xv.x, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x2f32(yv.x, xv.y, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x2f32(-yv.y, xv.y, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x2f32(yv.y, xv.x, ci, 0, 0, 0);
        }
      } else {
        for (int b = 0; 16 * b < na; ++b) {
          // atoms 16 b + 8 lk .. + 7 of rows 32 wy + li (y) and 32 wx + li (x)
          const _Float16* ty = tb + 4 * kTabH + split_at(32 * wy + li, 2 * b + lk);
          const _Float16* tx = tb + split_at(32 * wx + li, 2 * b + lk);
          const v8h yrh = *reinterpret_cast<const v8h*>(ty);
          const v8h yih = *reinterpret_cast<const v8h*>(ty + kTabH);
          const v8h yrl = *reinterpret_cast<const v8h*>(ty + 2 * kTabH);
          const v8h yil = *reinterpret_cast<const v8h*>(ty + 3 * kTabH);
          const v8h xrh = *reinterpret_cast<const v8h*>(tx);
          const v8h xih = *reinterpret_cast<const v8h*>(tx + kTabH);
          const v8h xrl = *reinterpret_cast<const v8h*>(tx + 2 * kTabH);
          const v8h xil = *reinterpret_cast<const v8h*>(tx + 3 * kTabH);
          // -yi by flipping the two sign bits of each packed word (one XOR per 32 bits)
          const v8h nyih = __builtin_bit_cast(v8h, __builtin_bit_cast(v4u, yih) ^ 0x80008000u);
          const v8h nyil = __builtin_bit_cast(v8h, __builtin_bit_cast(v4u, yil) ^ 0x80008000u);
          // Re += yr xr - yi xi,  Im += yr xi + yi xr  (each as hi*hi + hi*lo + lo*hi)
          cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xrh, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xih, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xrl, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xil, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrl, xrh, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrl, xih, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(nyih, xih, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(yih, xrh, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(nyih, xil, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(yih, xrl, ci, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(nyil, xih, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(yil, xrh, ci, 0, 0, 0);
        }
      }
    }
    // accumulator element r of this lane is (row (r&3) + 4 lk + 8 (r>>2), column li) of the
    // quadrant: V += f_z(|k|) S_z, the running sum kept in the output until the last species,
    // which applies the prefactor and the band limit
    if (tj < TWe) {
      const float* f = ffs + 12 * z;
      // the element coordinates are recomputed here on every species rather than held in
      // registers across the contraction loop (the opaque copy stops their hoisting)
      int tib = 32 * wy + 4 * lk;
      asm volatile("" : "+v"(tib));
      const int m = m0 + tj, ms = m < a.nx / 2 ? m : m - a.nx;
      const float kx = (float)ms / (float)a.lx;
      const int nm = a.nmax[m];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ti = tib + (r & 3) + 8 * (r >> 2);
        if (ti >= THe) continue;
        const int n = n0 + ti, ns = n < a.ny / 2 ? n : n - a.ny, an = ns < 0 ? -ns : ns;
        const float ky = (float)ns / (float)a.ly;
        const float fz = form_factor(f, kx * kx + ky * ky);
        float2 v = z == zfirst ? make_float2(0.f, 0.f) : out[(size_t)n * a.nx + m];
        v.x = fmaf(fz, cr[r], v.x);
        v.y = fmaf(fz, ci[r], v.y);
        if (z == zlast)
          put(n, m, an <= nm ? make_float2(v.x * a.pref, v.y * a.pref) : make_float2(0.f, 0.f));
        else
          out[(size_t)n * a.nx + m] = v;
      }
    }
  }
}

// Split structure factor over a quarter of k-space (Hermitian mode: band limit on, so the Nyquist
// row and column are zero).  An atom's x phase at -kx is the conjugate of the one at +kx, so with
//   P1 = sum yr xr,  P2 = sum yi xi,  P3 = sum yr xi,  P4 = sum yi xr   (kx >= 0, ky >= 0)
// the sums at (ky, kx) and (ky, -kx) are (P1 - P2) + i (P3 + P4) and (P1 + P2) + i (P4 - P3); the
// rows ky < 0 follow by conjugation (real V).  Each 32 x 32 block of four real products (twelve
// split-fp16 MFMAs per 16 atoms, as above) thus yields two output blocks, and phase tables are
// generated for kx >= 0 only: half the matrix-core work and half the table generation of the
// half-plane kernel.  One workgroup per (map, 64 x 64 tile of 0 <= kx < nx/2, 0 <= ky < ny/2).
__global__ __launch_bounds__(256, 4) void k_structure_factor_quarter(SfArgs a) {
  constexpr int kBytes = 2 * 4 * kTabH * (int)sizeof(_Float16);
  __shared__ __attribute__((aligned(16))) char tables[kBytes];
  _Float16* tb = reinterpret_cast<_Float16*>(tables);   // [axis][component][split_at(k, atom / 8)]
  constexpr int kSfBatch = sf_batch<true>();
  __shared__ AtomPhase batch[kSfBatch];
  __shared__ float ffs[kMaxSpecies * 12];
  const int nx = a.nx, ny = a.ny, hx = nx / 2, hy = ny / 2;
  const int tx_n = (hx + kTile - 1) / kTile, ty_n = (hy + kTile - 1) / kTile;
  const int tiles = tx_n * ty_n;
  // workgroups 0 .. n_maps n_live - 1 take the tiles with kept k, map by map; the rest the others
  const int nl = a.n_live, nlive_wg = a.n_maps * nl;
  const int bid = blockIdx.x;
  int map, tile;
  if (bid < nlive_wg) {
    map = bid / nl;
    tile = a.tile_order[bid % nl];
  } else {
    const int nd = tiles - nl, r = bid - nlive_wg;
    map = r / nd;
    tile = a.tile_order[nl + r % nd];
  }
  if (map >= a.n_maps) return;
  const int m0 = (tile % tx_n) * kTile, n0 = (tile / tx_n) * kTile;
  const int TWe = min(kTile, hx - m0), THe = min(kTile, hy - n0);
  const int t = a.t0 + map / a.s_count, s = map % a.s_count;
  const int tid = threadIdx.x;
  for (int i = tid; i < a.n_species * 12; i += 256) ffs[i] = a.ff[i];
  float2* out = a.vk + (size_t)map * nx * ny;
  // (n, m) with 0 <= n < ny/2, 0 <= m < nx/2: vp at (n, m), vm at (n, -m), and for n > 0 their
  // conjugates at (-n, -m) and (-n, m)
  auto put = [&](int n, int m, float2 vp, float2 vm) {
    const int mm = m == 0 ? 0 : nx - m;
    out[(size_t)n * nx + m] = vp;
    if (m > 0) out[(size_t)n * nx + mm] = vm;
    if (n > 0) {
      const size_t rr = (size_t)(ny - n) * nx;
      out[rr + mm] = make_float2(vp.x, -vp.y);
      if (m > 0) out[rr + m] = make_float2(vm.x, -vm.y);
    }
  };
  // the Nyquist row and column (zero under the band limit)
  if (n0 == 0)
    for (int m = m0 + tid; m < m0 + TWe; m += 256) {
      out[(size_t)hy * nx + m] = make_float2(0.f, 0.f);
      if (m > 0) out[(size_t)hy * nx + nx - m] = make_float2(0.f, 0.f);
    }
  if (m0 == 0) {
    for (int n = n0 + tid; n < n0 + THe; n += 256) {
      out[(size_t)n * nx + hx] = make_float2(0.f, 0.f);
      if (n > 0) out[(size_t)(ny - n) * nx + hx] = make_float2(0.f, 0.f);
    }
    if (n0 == 0 && tid == 0) out[(size_t)hy * nx + hx] = make_float2(0.f, 0.f);
  }
  auto zero_tile = [&]() {
    for (int i = tid; i < TWe * THe; i += 256)
      put(n0 + i / TWe, m0 + i % TWe, make_float2(0.f, 0.f), make_float2(0.f, 0.f));
  };
  // does any k of this tile pass the band limit?  (exact integer table, symmetric in kx)
  int any = 0;
  for (int m = m0 + tid; m < m0 + TWe; m += 256) any |= (a.nmax[m] >= n0);
  if (!__syncthreads_or(any)) {
    zero_tile();
    return;
  }
  const int lane = tid & 63, w = tid >> 6, wy = w >> 1, wx = w & 1;
  const int li = lane & 31, lk = lane >> 5;
  const int* off = a.offsets + (size_t)t * (a.s_count * a.n_species + 1);
  const AtomPhase* R = (const AtomPhase*)a.arec + (size_t)(t - a.t0) * a.n_atoms;
  int zfirst = -1, zlast = -1;
  for (int z = 0; z < a.n_species; ++z)
    if (off[s * a.n_species + z + 1] > off[s * a.n_species + z]) {
      if (zfirst < 0) zfirst = z;
      zlast = z;
    }
  if (zlast < 0) {
    zero_tile();
    return;
  }
  const int tj = 32 * wx + li;
  // a 32 x 32 block with no kept k skips its matrix-core products (the tables are still generated)
  const int qn = 32 * wy < THe ? n0 + 32 * wy : (1 << 30);
  const bool quad_live = __ballot(tj < TWe && a.nmax[m0 + min(tj, TWe - 1)] >= qn) != 0ull;
  for (int z = 0; z < a.n_species; ++z) {
    const int j0 = off[s * a.n_species + z], j1 = off[s * a.n_species + z + 1];
    if (j1 <= j0) continue;
    v16f p1 = {0}, p2 = {0}, p3 = {0}, p4 = {0};
    const uint2* Rw = reinterpret_cast<const uint2*>(R);
    uint2* bw = reinterpret_cast<uint2*>(batch);
    uint2 nr0 = make_uint2(0u, 0u), nr1 = nr0, nr2 = nr0;
    if (tid < kSfBatch && j0 + tid < j1) {
      nr0 = Rw[3 * (j0 + tid)];
      nr1 = Rw[3 * (j0 + tid) + 1];
      nr2 = Rw[3 * (j0 + tid) + 2];
    }
    for (int c0 = j0; c0 < j1; c0 += kSfChunk) {
      const int na = min(kSfChunk, j1 - c0);
      const int bi = (c0 - j0) % kSfBatch;
      __syncthreads();                        // previous chunk's tables (and batch) are consumed
      if (bi == 0) {
        if (tid < kSfBatch) {
          bw[3 * tid] = nr0;
          bw[3 * tid + 1] = nr1;
          bw[3 * tid + 2] = nr2;
          const int nb = c0 + kSfBatch + tid;
          if (nb < j1) {
            nr0 = Rw[3 * nb];
            nr1 = Rw[3 * nb + 1];
            nr2 = Rw[3 * nb + 2];
          }
        }
        __syncthreads();
      }
      const AtomPhase* arec = batch + bi;
      {
        // one item per thread: (axis, block of 8 k, atom pair); every index is below n/2, so the
        // signed index equals the storage index and a block never wraps
        const int axis = tid >> 7, k0 = ((tid >> 4) & 7) * 8, pair = tid & 15;
        const int lim = axis == 0 ? TWe : THe;
        const int idx = (axis == 0 ? m0 : n0) + k0;
        float2 f[2], st[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int at = 2 * pair + u;
          if (at < na && k0 < lim) {
            const AtomPhase& ap = arec[at];
            f[u] = phase_factor(idx, axis == 0 ? ap.ux : ap.uy);
            st[u] = axis == 0 ? ap.sx : ap.sy;
          } else {
            f[u] = make_float2(0.f, 0.f);
            st[u] = make_float2(0.f, 0.f);
          }
        }
        _Float16* row = tb + axis * 4 * kTabH + 2 * (pair & 3);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const h2 rh = __builtin_amdgcn_cvt_pkrtz(f[0].x, f[1].x);
          const h2 ih = __builtin_amdgcn_cvt_pkrtz(f[0].y, f[1].y);
          const h2 rl = split_lo(f[0].x, f[1].x, rh);
          const h2 il = split_lo(f[0].y, f[1].y, ih);
          _Float16* dst = row + split_at(k0 + q, pair >> 2);
          *reinterpret_cast<h2*>(dst) = rh;
          *reinterpret_cast<h2*>(dst + kTabH) = ih;
          *reinterpret_cast<h2*>(dst + 2 * kTabH) = rl;
          *reinterpret_cast<h2*>(dst + 3 * kTabH) = il;
          f[0] = cmul(f[0], st[0]);
          f[1] = cmul(f[1], st[1]);
        }
      }
      __syncthreads();
      if (quad_live) {
        for (int b = 0; 16 * b < na; ++b) {
          const _Float16* ty = tb + 4 * kTabH + split_at(32 * wy + li, 2 * b + lk);
          const _Float16* tx = tb + split_at(32 * wx + li, 2 * b + lk);
          const v8h yrh = *reinterpret_cast<const v8h*>(ty);
          const v8h yih = *reinterpret_cast<const v8h*>(ty + kTabH);
          const v8h yrl = *reinterpret_cast<const v8h*>(ty + 2 * kTabH);
          const v8h yil = *reinterpret_cast<const v8h*>(ty + 3 * kTabH);
          const v8h xrh = *reinterpret_cast<const v8h*>(tx);
          const v8h xih = *reinterpret_cast<const v8h*>(tx + kTabH);
          const v8h xrl = *reinterpret_cast<const v8h*>(tx + 2 * kTabH);
          const v8h xil = *reinterpret_cast<const v8h*>(tx + 3 * kTabH);
          // each real product as hi*hi + hi*lo + lo*hi, the four sums interleaved
          p1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xrh, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yih, xih, p2, 0, 0, 0);
          p3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xih, p3, 0, 0, 0);
          p4 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yih, xrh, p4, 0, 0, 0);
          p1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xrl, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yih, xil, p2, 0, 0, 0);
          p3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrh, xil, p3, 0, 0, 0);
          p4 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yih, xrl, p4, 0, 0, 0);
          p1 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrl, xrh, p1, 0, 0, 0);
          p2 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yil, xih, p2, 0, 0, 0);
          p3 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yrl, xih, p3, 0, 0, 0);
          p4 = __builtin_amdgcn_mfma_f32_32x32x16_f16(yil, xrh, p4, 0, 0, 0);
        }
      }
    }
    // accumulator element r of this lane is (row (r&3) + 4 lk + 8 (r>>2), column li) of the
    // block; V += f_z(|k|) S_z at (ky, kx) and (ky, -kx), the running sums kept in the output
    // until the last species, which applies the prefactor and the band limit
    if (tj < TWe) {
      const float* f = ffs + 12 * z;
      int tib = 32 * wy + 4 * lk;
      asm volatile("" : "+v"(tib));
      const int m = m0 + tj, mm = m == 0 ? 0 : nx - m;
      const float kx = (float)m / (float)a.lx;
      const int nmp = a.nmax[m], nmm = a.nmax[mm];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ti = tib + (r & 3) + 8 * (r >> 2);
        if (ti >= THe) continue;
        const int n = n0 + ti;
        const float ky = (float)n / (float)a.ly;
        const float fz = form_factor(f, kx * kx + ky * ky);
        float2 vp = make_float2(0.f, 0.f), vm = vp;
        if (z != zfirst) {
          vp = out[(size_t)n * nx + m];
          vm = out[(size_t)n * nx + mm];
        }
        vp.x = fmaf(fz, p1[r] - p2[r], vp.x);
        vp.y = fmaf(fz, p3[r] + p4[r], vp.y);
        vm.x = fmaf(fz, p1[r] + p2[r], vm.x);
        vm.y = fmaf(fz, p4[r] - p3[r], vm.y);
        if (z == zlast) {
          put(n, m, n <= nmp ? make_float2(vp.x * a.pref, vp.y * a.pref) : make_float2(0.f, 0.f),
              n <= nmm ? make_float2(vm.x * a.pref, vm.y * a.pref) : make_float2(0.f, 0.f));
        } else {
          out[(size_t)n * nx + m] = vp;
          if (m > 0) out[(size_t)n * nx + mm] = vm;
        }
      }
    }
  }
}

hipError_t launch_atom_phase(const float* xyz, const int* order, int t0, int nt, int n_atoms,
                             double lx, double ly, void* rec, hipStream_t st) {
  const long total = (long)nt * n_atoms;
  long blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_atom_phase, dim3((unsigned)blocks), dim3(256), 0, st, xyz, order, t0, nt,
                     n_atoms, lx, ly, (AtomPhase*)rec);
  return hipGetLastError();
}

hipError_t launch_structure_factor(const SfArgs& a, hipStream_t st) {
  {
    hipError_t e = launch_atom_phase(a.xyz, a.order, a.t0, a.n_maps / a.s_count, a.n_atoms, a.lx,
                                     a.ly, a.arec, st);
    if (e != hipSuccess) return e;
  }
  const int tx_n = (a.nx + kTile - 1) / kTile;
  const int ty_n = a.hermitian ? (a.ny / 2 + kTile - 1) / kTile : (a.ny + kTile - 1) / kTile;
  const long blocks = (long)a.n_maps * tx_n * ty_n;
  if (blocks <= 0) return hipSuccess;
  if (a.split16 && a.hermitian) {
    const long qb = (long)a.n_maps * ((a.nx / 2 + kTile - 1) / kTile) * ((a.ny / 2 + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_structure_factor_quarter, dim3((unsigned)qb), dim3(256), 0, st, a);
  } else if (a.split16)
    hipLaunchKernelGGL(k_structure_factor<true>, dim3((unsigned)blocks), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_structure_factor<false>, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// dL/d(x, y): one workgroup per (map, species-pure chunk of at most 64 atoms).
// With H(k) = conj(G(k)) pref M(k) f_Z(|k|) w(k), G = DFT[dL/dV_s] (w = 2 for ky > 0 rows when
// only the ky >= 0 half is visited, else 1; the factors other than G come from vtab):
//   T[a][m]  = sum_n ey_a(n) H(n, m),   T'[a][m] = sum_n ey_a(n) ky_n H(n, m)      (MFMA, K = ky)
//   dx_a = 2 pi Im sum_m T[a][m] kx_m ex_a(m),   dy_a = 2 pi Im sum_m T'[a][m] ex_a(m)
// G is Hermitian (dL/dV is real), so the summand at -k is minus the conjugate of the one at k and
// the imaginary parts agree: with the band limit on, rows ky > 0 are visited with weight 2 and the
// row ky = 0 with weight 1.  Both operands are split into fp16 high and low parts (as in the
// structure factor) for v_mfma_f32_32x32x16_f16: the phases are unit numbers, and H is scaled by a
// power of two per map (from max |G| and a host bound on the other factors) so that its split
// parts are normal fp16 numbers; the scale is removed when T is folded with the x phases.
// Four wavefronts: (atom half) x (kx half) quadrants of 32 x 32; ky in fills of 32.
constexpr int kPgKy = 32;     // ky per LDS fill
constexpr int kPgRow = 40;    // halves per table row (32 + pad: rows 80 bytes apart)

__global__ __launch_bounds__(256) void k_position_grad(PgArgs a, const int4* chunks,
                                                      const int* n_chunks) {
  __shared__ __attribute__((aligned(16))) _Float16 Et[4][kChunk][kPgRow];      // y phases (split)
  __shared__ __attribute__((aligned(16))) char hraw[8 * kTile * kPgRow * 2];   // H, ky H (split)
  __shared__ AtomPhase rec[kChunk];
  __shared__ float red[4][32][2];
  _Float16 (*Ht)[kTile][kPgRow] = reinterpret_cast<_Float16 (*)[kTile][kPgRow]>(hraw);
  float2 (*Ex)[kTile + 1] = reinterpret_cast<float2 (*)[kTile + 1]>(hraw);     // x phases (fold)
  static_assert(sizeof(float2) * kChunk * (kTile + 1) <= sizeof(hraw), "x-phase table fits");
  if ((int)blockIdx.x >= *n_chunks) return;
  const int4 ch = chunks[blockIdx.x];          // (map, first CSR index, count, species)
  const int map = ch.x, c0 = ch.y, na = ch.z, z = ch.w;
  const int tl = map / a.s_count, t = a.t0 + tl;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 31, lk = lane >> 5, wa = w >> 1, wk = w & 1;
  const AtomPhase* R = (const AtomPhase*)a.arec + (size_t)tl * a.n_atoms;
  if (tid < kChunk) {
    AtomPhase r{0u, 0u, make_float2(1.f, 0.f), make_float2(1.f, 0.f)};
    if (tid < na) r = R[c0 + tid];
    rec[tid] = r;
  }
  const float2* G = a.gk + (size_t)map * a.nx * a.ny;
  const int herm = a.hermitian;
  const int ny_h = herm ? a.ny / 2 : a.ny;
  const float* vt = a.vtab + (size_t)z * ny_h * a.nx;
  const int TW = min(kTile, a.nx);
  const int tx_n = (a.nx + TW - 1) / TW;
  // power-of-two scale of H for this map
  float hs = 1.f;
  {
    const float b = a.absmax[map] * a.hbound;
    if (b > 0.f && b < 3.0e38f) {
      int e;
      (void)frexpf(b, &e);                      // b <= 2^e
      hs = ldexpf(1.f, 14 - e);
    }
  }
  const float inv_hs = 1.f / hs;
  const float inv_ly = (float)(1.0 / (double)a.ly);
  float sx[16], sy[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) { sx[r] = 0.f; sy[r] = 0.f; }

  for (int tx = 0; tx < tx_n; ++tx) {
    const int m0 = tx * TW;
    const int TWe = min(TW, a.nx - m0);   // the last kx tile of a length not a multiple of 64
    v16f cr = {0}, ci = {0}, tr = {0}, ti = {0};
    int used = 0;
    const int n_fills = (ny_h + kPgKy - 1) / kPgKy;
    for (int n0 = 0; n0 < ny_h; n0 += kPgKy) {
      const int kh = min(kPgKy, ny_h - n0);
      // fills without a kept k are skipped (the table is uniform across the workgroup)
      if (!a.fill_live[tx * n_fills + n0 / kPgKy]) continue;
      __syncthreads();                          // the previous fill's readers are done
      used = 1;
      // H and ky H for (kx = m0 + c, ky rows n0 + 8 kb + q): 8 consecutive ky per thread, each
      // component split as hi = fp16 (round toward zero) and lo = fp16(x - hi) for the pairs of
      // consecutive rows that share a packed word
      {
        const int c = tid & 63, kb = tid >> 6;
        const int m = m0 + c;
        // the eight rows' G and factor-table values are loaded together (one wait); a position
        // outside the tile reads element 0 and is then taken as zero
        float vq[8];
        float2 gq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int n = n0 + 8 * kb + q;
          const size_t idx = (c < TWe && n < n0 + kh) ? (size_t)n * a.nx + m : 0;
          vq[q] = vt[idx];
          gq[q] = G[idx];
        }
        float comps[4][8];   // Re H, Im H, Re ky H, Im ky H
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int n = n0 + 8 * kb + q;
          const bool in = c < TWe && n < n0 + kh;
          const int ns = n < a.ny / 2 ? n : n - a.ny;
          const float ky = in ? (float)ns * inv_ly : 0.f;
          const float v = in ? vq[q] * hs : 0.f;
          // G is set only inside the band (where the table is not zero): outside it, take zero
          const float2 h = v != 0.f ? make_float2(gq[q].x * v, -gq[q].y * v) : make_float2(0.f, 0.f);
          comps[0][q] = h.x;
          comps[1][q] = h.y;
          comps[2][q] = ky * h.x;
          comps[3][q] = ky * h.y;
        }
        // table order: 0 Re H hi, 1 Im H hi, 2 Re H lo, 3 Im H lo, 4..7 the same for ky H
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v4u hi, lo;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const h2 hh = __builtin_amdgcn_cvt_pkrtz(comps[u][2 * j], comps[u][2 * j + 1]);
            hi[j] = __builtin_bit_cast(unsigned, hh);
            lo[j] = __builtin_bit_cast(unsigned, split_lo(comps[u][2 * j], comps[u][2 * j + 1], hh));
          }
          const int th = (u >> 1) * 4 + (u & 1);
          *reinterpret_cast<v4u*>(&Ht[th][c][8 * kb]) = hi;
          *reinterpret_cast<v4u*>(&Ht[th + 2][c][8 * kb]) = lo;
        }
      }
      // y phases of the 64 atoms at ky rows n0 + 8 kb .. + 7 (exact start, unit steps), split as
      // above
      {
        const int at = tid & 63, kb = tid >> 6;
        const int n = n0 + 8 * kb;
        const int sidx = n < a.ny / 2 ? n : n - a.ny;
        const int qw = a.ny / 2 - n;            // the signed index jumps to -ny/2 at step qw
        const bool live = at < na && 8 * kb < kh;
        float2 f = make_float2(0.f, 0.f), st = make_float2(0.f, 0.f);
        if (live) {
          f = phase_factor(sidx, rec[at].uy);
          st = rec[at].sy;
        }
        float2 fq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (q == qw && live) f = phase_factor(n + q - a.ny, rec[at].uy);
          fq[q] = f;
          f = cmul(f, st);
        }
        v4u rh, ih, rl, il;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const h2 a_hi = __builtin_amdgcn_cvt_pkrtz(fq[2 * j].x, fq[2 * j + 1].x);
          const h2 b_hi = __builtin_amdgcn_cvt_pkrtz(fq[2 * j].y, fq[2 * j + 1].y);
          rh[j] = __builtin_bit_cast(unsigned, a_hi);
          ih[j] = __builtin_bit_cast(unsigned, b_hi);
          rl[j] = __builtin_bit_cast(unsigned, split_lo(fq[2 * j].x, fq[2 * j + 1].x, a_hi));
          il[j] = __builtin_bit_cast(unsigned, split_lo(fq[2 * j].y, fq[2 * j + 1].y, b_hi));
        }
        *reinterpret_cast<v4u*>(&Et[0][at][8 * kb]) = rh;
        *reinterpret_cast<v4u*>(&Et[1][at][8 * kb]) = ih;
        *reinterpret_cast<v4u*>(&Et[2][at][8 * kb]) = rl;
        *reinterpret_cast<v4u*>(&Et[3][at][8 * kb]) = il;
      }
      __syncthreads();
      const int ar = 32 * wa + li, hc = 32 * wk + li;
#pragma unroll
      for (int b = 0; b < kPgKy / 16; ++b) {
        const int kb = 16 * b + 8 * lk;
        const v8h erh = *reinterpret_cast<const v8h*>(&Et[0][ar][kb]);
        const v8h eih = *reinterpret_cast<const v8h*>(&Et[1][ar][kb]);
        const v8h erl = *reinterpret_cast<const v8h*>(&Et[2][ar][kb]);
        const v8h eil = *reinterpret_cast<const v8h*>(&Et[3][ar][kb]);
        const v8h neih = __builtin_bit_cast(v8h, __builtin_bit_cast(v4u, eih) ^ 0x80008000u);
        const v8h neil = __builtin_bit_cast(v8h, __builtin_bit_cast(v4u, eil) ^ 0x80008000u);
        const v8h hrh = *reinterpret_cast<const v8h*>(&Ht[0][hc][kb]);
        const v8h hih = *reinterpret_cast<const v8h*>(&Ht[1][hc][kb]);
        const v8h hrl = *reinterpret_cast<const v8h*>(&Ht[2][hc][kb]);
        const v8h hil = *reinterpret_cast<const v8h*>(&Ht[3][hc][kb]);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, hrh, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, hih, ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, hrl, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, hil, ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(erl, hrh, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(erl, hih, ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(neih, hih, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(eih, hrh, ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(neih, hil, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(eih, hrl, ci, 0, 0, 0);
        cr = __builtin_amdgcn_mfma_f32_32x32x16_f16(neil, hih, cr, 0, 0, 0);
        ci = __builtin_amdgcn_mfma_f32_32x32x16_f16(eil, hrh, ci, 0, 0, 0);
        const v8h prh = *reinterpret_cast<const v8h*>(&Ht[4][hc][kb]);
        const v8h pih = *reinterpret_cast<const v8h*>(&Ht[5][hc][kb]);
        const v8h prl = *reinterpret_cast<const v8h*>(&Ht[6][hc][kb]);
        const v8h pil = *reinterpret_cast<const v8h*>(&Ht[7][hc][kb]);
        tr = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, prh, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, pih, ti, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, prl, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_32x32x16_f16(erh, pil, ti, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_32x32x16_f16(erl, prh, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_32x32x16_f16(erl, pih, ti, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_32x32x16_f16(neih, pih, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_32x32x16_f16(eih, prh, ti, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_32x32x16_f16(neih, pil, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_32x32x16_f16(eih, prl, ti, 0, 0, 0);
        tr = __builtin_amdgcn_mfma_f32_32x32x16_f16(neil, pih, tr, 0, 0, 0);
        ti = __builtin_amdgcn_mfma_f32_32x32x16_f16(eil, prh, ti, 0, 0, 0);
      }
    }
    if (!used) continue;
    // fold with the x phases of this kx tile (table aliases H: wait for the last MFMA readers)
    __syncthreads();
    for (int i = tid; i < kChunk * (kTile / 8); i += 256) {
      const int at = i / (kTile / 8), kb = (i % (kTile / 8)) * 8;
      float2* dst = &Ex[at][kb];
      if (at >= na || kb >= TWe) {
#pragma unroll
        for (int q = 0; q < 8; ++q) dst[q] = make_float2(0.f, 0.f);
        continue;
      }
      const int idx = m0 + kb, sidx = idx < a.nx / 2 ? idx : idx - a.nx;
      const int qw = a.nx / 2 - idx;           // the signed index jumps to -nx/2 at step qw
      float2 ph = phase_factor(sidx, rec[at].ux);
      const float2 st = rec[at].sx;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (q == qw) ph = phase_factor(idx + q - a.nx, rec[at].ux);
        dst[q] = ph;
        ph = cmul(ph, st);
      }
    }
    __syncthreads();
    const int col = 32 * wk + li, m = m0 + col, ms = m < a.nx / 2 ? m : m - a.nx;
    const float kx = (float)ms / (float)a.lx;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * wa + (r & 3) + 4 * lk + 8 * (r >> 2);
      const float2 e = Ex[row][col];
      sx[r] += inv_hs * kx * (cr[r] * e.y + ci[r] * e.x);
      sy[r] += inv_hs * (tr[r] * e.y + ti[r] * e.x);
    }
  }
  // sum over the 32 columns held by the lanes li of each half-wave
#pragma unroll
  for (int r = 0; r < 16; ++r) {
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) {
      sx[r] += __shfl_xor(sx[r], o, 32);
      sy[r] += __shfl_xor(sy[r], o, 32);
    }
  }
  if (li == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = (r & 3) + 4 * lk + 8 * (r >> 2);
      red[w][row][0] = sx[r];
      red[w][row][1] = sy[r];
    }
  }
  __syncthreads();
  if (tid < na) {
    const int h = tid >> 5, row = tid & 31;
    const float dx = red[2 * h][row][0] + red[2 * h + 1][row][0];
    const float dy = red[2 * h][row][1] + red[2 * h + 1][row][1];
    const int aj = a.order[(size_t)t * a.n_atoms + c0 + tid];
    float* out = a.gxy + ((size_t)t * a.n_atoms + aj) * 2;
    const float two_pi = 6.283185307179586f;
    out[0] = two_pi * dx;
    out[1] = two_pi * dy;
  }
}

}  // namespace tacaw

namespace tacaw {
// Work list for the position gradient: species-pure chunks of at most 64 atoms per map, in map
// order, built on the device from the CSR offsets (one workgroup, fixed order, no host sync).
__global__ __launch_bounds__(256) void k_chunk_list(const int* offsets, int t0, int nt, int S,
                                                   int nsp, int4* chunks, int cap, int* count) {
  __shared__ int sc[256];
  const int tid = threadIdx.x;
  const int K = S * nsp, total = nt * K;
  int running = 0;
  for (int base = 0; base < total; base += 256) {
    const int i = base + tid;
    int nch = 0, start = 0, cnt = 0, map = 0, z = 0;
    if (i < total) {
      const int tl = i / K, key = i % K;
      const int* off = offsets + (size_t)(t0 + tl) * (K + 1);
      start = off[key];
      cnt = off[key + 1] - start;
      nch = (cnt + kChunk - 1) / kChunk;
      map = tl * S + key / nsp;
      z = key % nsp;
    }
    sc[tid] = nch;
    __syncthreads();
    for (int w = 1; w < 256; w <<= 1) {      // inclusive scan (Hillis-Steele)
      int v = tid >= w ? sc[tid - w] : 0;
      __syncthreads();
      sc[tid] += v;
      __syncthreads();
    }
    const int pos = running + sc[tid] - nch;
    for (int k = 0; k < nch; ++k)
      if (pos + k < cap)
        chunks[pos + k] = make_int4(map, start + k * kChunk, min(kChunk, cnt - k * kChunk), z);
    running += sc[255];
    __syncthreads();
  }
  if (tid == 0) *count = running < cap ? running : cap;
}

hipError_t launch_chunk_list(const int* offsets, int t0, int nt, int S, int nsp, int4* chunks,
                             int cap, int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_chunk_list, dim3(1), dim3(256), 0, st, offsets, t0, nt, S, nsp, chunks, cap,
                     count);
  return hipGetLastError();
}

hipError_t launch_position_grad_chunks(const PgArgs& a, const int4* chunks, int cap,
                                       const int* count, hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_position_grad, dim3(cap), dim3(256), 0, st, a, chunks, count);
  return hipGetLastError();
}

__global__ void k_zero(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = i; k < n16; k += stride) p[k] = make_uint4(0, 0, 0, 0);
  if (i < ntail) tail[i] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  size_t n16 = bytes / 16, ntail = bytes % 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint4*)p, n16,
                     (unsigned char*)p + n16 * 16, ntail);
  return hipGetLastError();
}
}  // namespace tacaw
