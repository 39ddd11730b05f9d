// Multislice slice-step kernels: the x pass (row kernel) and the y pass (column kernel).
//
// A slice step psi <- F^-1[M P_s F[t_s psi]] is split at the 2-D transform's two axes.  Between
// launches a wave is stored in the (kx, y) representation W = F_x[psi] / nx:
//   row kernel, slice s:  psi = G_x W (x inverse transform), u = t_s psi, W' = F_x u
//   column kernel, s:     W = G_y[ M P_s F_y W' ] / (nx ny)   (or, after the last slice, the exit
//                         wave phi = M P_s F_y W' / sqrt(nx ny) stored in (kx, ky))
// with F/G the unnormalised forward/inverse DFTs.  Each pass reads and writes the wave once (plus V
// in the row pass, shared by the probe positions of a snapshot): 32 N^2 bytes per slice step and
// wave plus 4 N^2 per snapshot, less where the band limit leaves columns out.
//
// Row kernel: one line = one image row, held by L lanes of a wave; lines never share LDS, so the
// transform needs no workgroup barrier.  All probe positions of a snapshot share one load of the V
// row and one evaluation of exp(i sigma V).  Column kernel: a workgroup stages C columns x N rows
// through LDS with coalesced row segments, each wave transforms whole columns in place in that
// tile, and the tile is written back with coalesced stores.
#include <type_traits>

#include "internal.hpp"

namespace tacaw {

template <class F> static bool with_plan(int n, int idx, F&& f) {
  switch (n) {
    case 16: if (idx == 1) f(P16b{}); else f(P16a{}); return true;
    case 32: if (idx == 1) f(P32b{}); else f(P32a{}); return true;
    case 64: if (idx == 1) f(P64b{}); else f(P64a{}); return true;
    case 128: if (idx == 1) f(P128b{}); else f(P128a{}); return true;
    case 256: if (idx == 1) f(P256b{}); else if (idx == 2) f(P256c{}); else f(P256a{}); return true;
    case 512: if (idx == 1) f(P512b{}); else f(P512a{}); return true;
    case 1024: if (idx == 1) f(P1024b{}); else f(P1024a{}); return true;
    case 560:
      if (idx == 1) f(P560b{}); else if (idx == 2) f(P560c{}); else if (idx == 3) f(P560d{}); else f(P560a{});
      return true;
    case 1000: if (idx == 1) f(P1000b{}); else f(P1000a{}); return true;
    default: return false;
  }
}

int n_plans(int n) {
  switch (n) {
    case 16: case 32: case 64: case 128: case 512: case 1024: return 2;
    case 256: return 3;
    case 560: return 4;
    case 1000: return 2;
    default: return 0;
  }
}

const char* plan_name(int n, int idx) {
  static const char* names[] = {"16:L2:8x2", "16:L4:4x4", "32:L4:8x4", "32:L2:16x2", "64:L8:8x8",
                                "64:L4:16x4", "128:L16:8x4x4", "128:L8:16x8", "256:L32:8x8x4",
                                "256:L16:16x16", "256:L64:4x4x4x4", "512:L64:8x8x8",
                                "512:L32:16x8x4", "1024:L64:16x16x4", "1024:L64:16x4x16",
                                "560:L28:4x5x4x7", "560:L56:2x5x2x2x14", "560:L28:20x4x7",
                                "560:L28:20x28", "1000:L50:4x5x5x10", "1000:L50:10x10x10"};
  int base = 0;
  switch (n) {
    case 16: base = 0; break; case 32: base = 2; break; case 64: base = 4; break;
    case 128: base = 6; break; case 256: base = 8; break; case 512: base = 11; break;
    case 1024: base = 13; break; case 560: base = 15; break; case 1000: base = 19; break;
    default: return "?";
  }
  if (idx < 0 || idx >= n_plans(n)) return "?";
  return names[base + idx];
}

// Address spaces.  Wave data is accessed through global-address-space pointers: flat (generic)
// accesses share the LDS completion counter, so every LDS wait inside a transform would also wait
// for the prefetch of the next tile.  Job descriptors and task lists are read-only during a launch
// and indexed uniformly, so they are read through the constant address space (scalar loads).
// (The host compilation pass only type-checks kernel bodies; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL_AS __attribute__((address_space(1)))
#define CONST_AS __attribute__((address_space(4)))
#else
#define GLOBAL_AS
#define CONST_AS
#endif
typedef const CONST_AS MsJobDev CJob;

template <class T> __device__ __forceinline__ GLOBAL_AS T* gp(T* p) { return (GLOBAL_AS T*)p; }
__device__ __forceinline__ CJob& job_at(const MsJobDev* jobs, int i) { return ((CJob*)jobs)[i]; }
template <class T> __device__ __forceinline__ T const_at(const T* base, int i) {
  return ((const CONST_AS T*)base)[i];
}

__device__ __forceinline__ GLOBAL_AS float2* pick_buf(CJob& J, int code, int wave, int s) {
  size_t o = img_off(wave, J.nx, J.ny);
  switch (code) {
    case BUF_W: return gp(J.W) + o;
    case BUF_REC: return gp(J.rec) + o;
    case BUF_ADJ: return gp(J.adj) + o;
    case BUF_GEXIT: return gp(const_cast<float2*>(J.gexit)) + o;
    case BUF_ENTR: return J.entr ? gp(J.entr) + img_off(wave % J.P, J.nx, J.ny) : gp(J.W) + o;
    default: return gp(J.ckpt) + img_off(wave * J.n_ck + s / J.ck_stride, J.nx, J.ny);
  }
}

// elements from one probe position's image to the next in a buffer kind (for per-position bases
// derived from the first one)
__device__ __forceinline__ size_t buf_pos_stride(CJob& J, int code) {
  const size_t img = (size_t)J.nx * J.ny;
  return code == BUF_CKPT ? img * J.n_ck : img;
}

// The x pass streams its rows through HBM once (read once, written once, far larger than the
// caches): its wave loads and stores carry the non-temporal hint (measured: 3.5 % faster there,
// 7 % slower in the y pass, whose column tiles keep plain accesses).
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 load_nt(const GLOBAL_AS float2* p) {
  const f2v x = __builtin_nontemporal_load(reinterpret_cast<const GLOBAL_AS f2v*>(p));
  return make_float2(x.x, x.y);
}
__device__ __forceinline__ void store_nt(GLOBAL_AS float2* p, float2 v) {
  const f2v x = {v.x, v.y};
  __builtin_nontemporal_store(x, reinterpret_cast<GLOBAL_AS f2v*>(p));
}

// *p when c holds, else zero (the load is not issued for lanes where c fails)
__device__ __forceinline__ float2 load_if(const GLOBAL_AS float2* p, bool c) {
  float2 x = make_float2(0.f, 0.f);
  if (c) x = *p;
  return x;
}
__device__ __forceinline__ float2 load_if_nt(const GLOBAL_AS float2* p, bool c) {
  float2 x = make_float2(0.f, 0.f);
  if (c) x = load_nt(p);
  return x;
}

// Branch-free masked access to one wave image: a raw buffer resource over the image (uniform base,
// size in bytes) and per-lane byte offsets; a lane whose element is not wanted passes an offset
// beyond the resource, which the hardware answers with zeros (loads) or drops (stores) without a
// memory access.  Images are at most 1024 x 1024 complex values (8 MiB), far below the offset used.
constexpr unsigned kNoElem = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t image_rsrc(const GLOBAL_AS float2* base, int n_elem) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, n_elem * 8, 0x00020000);
}
// aux 2: non-temporal (streamed once).  The offset passes through an empty asm operand so that
// the optimiser keeps the lane select as a select instead of splitting the access into branches.
__device__ __forceinline__ unsigned opaque(unsigned x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm("" : "+v"(x));
#endif
  return x;
}
template <int AUX> __device__ __forceinline__ float2 bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const f2v x = __builtin_amdgcn_raw_buffer_load_b64(r, opaque(off), 0, AUX);
  return make_float2(x.x, x.y);
}
template <int AUX> __device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, float2 v) {
  const f2v x = {v.x, v.y};
  __builtin_amdgcn_raw_buffer_store_b64(x, r, opaque(off), 0, AUX);
}

// a if R, else b (both lvalues; only the chosen branch is instantiated)
template <bool R, class A, class B> __device__ __forceinline__ decltype(auto) pick_if(A& a, B& b) {
  if constexpr (R) return (a);
  else return (b);
}

// wait for every outstanding memory access of this wavefront
__device__ __forceinline__ void vmem_drain() { __builtin_amdgcn_s_waitcnt(0); }

// column (or row element) index m of an n-point axis inside the job's band
__device__ __forceinline__ bool in_band(int m, int kxb, int n) { return (m <= kxb) | (m >= n - kxb); }

// y-pass task -> (wave index, first column): tiles_lo tiles from the start of each wave's columns,
// then tiles_hi from the end (all tiles when both are 0)
__device__ __forceinline__ int col_tiles_per_wave(const ColArgs& a, int tpi) {
  return (a.tiles_lo + a.tiles_hi) > 0 ? a.tiles_lo + a.tiles_hi : tpi;
}
__device__ __forceinline__ void col_task(const ColArgs& a, int task, int tpw, int tpi, int& wi,
                                         int& col0) {
  wi = task / tpw;
  const int jt = task - wi * tpw;
  col0 = (jt < a.tiles_lo || a.tiles_hi == 0 ? jt : jt + tpi - a.tiles_lo - a.tiles_hi) * a.C;
}

// (wave index, tile) of the tasks a workgroup visits, advanced by gridDim.x tasks at a time
// without a division per step
struct ColCursor {
  int wi, jt;
  __device__ __forceinline__ void init(int task, int tpw) {
    wi = task / tpw;
    jt = task - wi * tpw;
  }
  __device__ __forceinline__ void step(int gdiv, int gmod, int tpw) {
    wi += gdiv;
    jt += gmod;
    if (jt >= tpw) {
      jt -= tpw;
      ++wi;
    }
  }
};
// first column of tile jt of a wave
__device__ __forceinline__ int col_first(const ColArgs& a, int jt, int tpi) {
  return (jt < a.tiles_lo || a.tiles_hi == 0 ? jt : jt + tpi - a.tiles_lo - a.tiles_hi) * a.C;
}

// The y pass's propagator rows py of the job of wave wi (conjugated for the adjoint) into LDS;
// returns that job.  The caller separates the writes from their readers with a barrier.
template <int N>
__device__ __forceinline__ int load_py_rows_w(const ColArgs& a, int wi, float2* pyl) {
  const int job = const_at(a.waves, wi).x;
  const GLOBAL_AS float2* pys = gp(job_at(a.jobs, job).py) + a.s * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    float2 q = pys[i];
    if (a.conj_prop) q.y = -q.y;
    pyl[i] = q;
  }
  return job;
}
template <int N>
__device__ __forceinline__ int load_py_rows(const ColArgs& a, int task, int tpw, int tpi, float2* pyl) {
  int wi, col0;
  col_task(a, task, tpw, tpi, wi, col0);
  const int job = const_at(a.waves, wi).x;
  const GLOBAL_AS float2* pys = gp(job_at(a.jobs, job).py) + a.s * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    float2 q = pys[i];
    if (a.conj_prop) q.y = -q.y;
    pyl[i] = q;
  }
  return job;
}

// Lengths that are not powers of two ask the compiler for at least 3 wavefronts per SIMD (2 for
// the adjoint x pass, which holds three line-sized arrays); their transforms would otherwise take
// every register for instruction-level parallelism.
template <class P, bool ADJ = false> constexpr int min_waves() { return P::POW2 ? 1 : (ADJ ? 2 : 3); }
// x pass: E = 16 power-of-two plans (1024 points) are held to 3 wavefronts per SIMD (their LDS
// allows 3 workgroups per CU; measured 3.4 -> 4.0 TB/s at 1024^2 against the unconstrained
// allocation at 2 per SIMD); forcing more than the natural 4 on E = 8 plans spills and is slower.
template <class P, bool ADJ = false> constexpr int row_min_waves() {
  return P::POW2 ? (ADJ ? 1 : (P::E <= 8 ? 1 : 3)) : (ADJ ? 2 : 3);
}

// ------------------------------------------------------------------------------------------------
// x pass
// Power-of-two plans read their per-lane twiddles from one LDS table per workgroup, laid out
// [k][L] (a line's lanes read consecutive words), instead of holding them in registers.  ONE: every
// job of the launch has a single wave per snapshot (plane waves, single probe positions), so the
// transmission is not shared; the V row is held as floats through the inverse transform and
// exp(i sigma V) is evaluated where it is applied (fewer live registers).
template <class P, bool ADJ, bool PR = false, bool ONE = false>
__global__ __launch_bounds__(kThreads, (row_min_waves<P, ADJ>())) void k_row(RowArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES;
  static_assert(!(ADJ && ONE), "the adjoint x pass evaluates the transmission once per row");
  __shared__ float2 lds_all[kWaves * LINES * P::LDS_LINE];
  __shared__ float2 twl[P::POW2 ? P::NTW * L : 1];
  // the wavefront index is uniform: the tasks, groups and job descriptors below are then read
  // with scalar loads
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int line = lane / L, l = lane % L;
  float2* lds = lds_all + (wave * LINES + line) * P::LDS_LINE;
  if constexpr (P::POW2) {
    if ((int)threadIdx.x < L) {
      float2 t[P::NTW] = {};
      PlanOps<P>::twiddles(t, threadIdx.x);
#pragma unroll
      for (int k = 0; k < P::NTW; ++k) twl[k * L + threadIdx.x] = t[k];
    }
    __syncthreads();
  }
  // E <= 8 plans of the forward pass copy their lane's twiddles to registers (room is left)
  constexpr bool TWREG = P::POW2 && P::E <= 8 && !ADJ;
  const TwStrided tws{twl + l, L};
  float2 twr[TWREG ? P::NTW : 1];
  if constexpr (TWREG) {
#pragma unroll
    for (int k = 0; k < P::NTW; ++k) twr[k] = tws[k];
  }
  const auto& tw = pick_if<TWREG>(twr, tws);
  const float2* tab = fft_table_init<P>();

  // rows per image rounded up to whole wavefronts of lines (the LINES lines of a wavefront then
  // always belong to one image: uniform group index); the rounding rows are skipped
  const int ny = a.ny, nyp = (ny + LINES - 1) / LINES * LINES, ysh = __builtin_ctz(nyp);
  const bool ypow2 = (nyp & (nyp - 1)) == 0;
  const int n_tasks = a.n_groups * nyp;
  const int stride = (int)gridDim.x * kWaves * LINES;
  for (int base = ((int)blockIdx.x * kWaves + wave) * LINES; base < n_tasks; base += stride) {
    const int g = ypow2 ? base >> ysh : base / nyp, y = base - g * nyp + line;
    if ((!P::FULL && line >= LINES) || y >= ny) continue;
    const int2 gr = const_at(a.groups, g);
    CJob& J = job_at(a.jobs, gr.x);
    const int t = gr.y, s = a.s;
    const size_t row = (size_t)y * N;
    const GLOBAL_AS float* vrow = gp(J.V) + ((size_t)(t * J.S + s) * ny) * N + row;
    const float sigma = J.sigma;
    // the row's V values are loaded together (one wait), then turned into exp(i sigma V)
    float vv[E];
#pragma unroll
    for (int j = 0; j < E; ++j) vv[j] = vrow[l + L * j];
    float2 tr[ONE ? 1 : E];
    if constexpr (!ONE) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        float sn, cs;
        sincos_phase(sigma * vv[j], &sn, &cs);
        tr[j] = make_float2(cs, sn);
      }
    }
    float gacc[ADJ ? E : 1];
    if constexpr (ADJ) {
#pragma unroll
      for (int j = 0; j < E; ++j) gacc[j] = 0.f;
    }
    const int P_ = ONE ? 1 : J.P;
    // band: element x of a row (a kx column of W) outside the job's band is zero on input (not
    // read) and of no use on output (not written) when band_in / band_out say so
    const int kxb = J.kxb;
    // bit j: element l + L j is inside the band
    typedef std::conditional_t<(E > 32), unsigned long long, unsigned> Mask;
    Mask inb = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) inb |= (in_band(l + L * j, kxb, N) ? Mask(1) : Mask(0)) << j;
    const Mask rmask = a.band_in ? inb : ~Mask(0), wmask = a.band_out ? inb : ~Mask(0);
    // forward, several positions: the row's wave buffers of position 0, the other positions at
    // fixed strides (one position per snapshot and the adjoint look each up directly, which keeps
    // registers free for their longer live state)
    constexpr bool STRIDED = !ONE && !ADJ;
    const GLOBAL_AS float2* in_p0 = STRIDED ? pick_buf(J, a.in_buf, t * J.P, s) : nullptr;
    GLOBAL_AS float2* out_p0 = STRIDED ? pick_buf(J, a.out_buf, t * J.P, s) : nullptr;
    const size_t in_ps = STRIDED ? buf_pos_stride(J, a.in_buf) : 0;
    const size_t out_ps = STRIDED ? buf_pos_stride(J, a.out_buf) : 0;
    for (int p = 0; p < P_; ++p) {
      const int w = t * J.P + p;
      float2 v[E];
      {
        const __amdgpu_buffer_rsrc_t in =
            image_rsrc(STRIDED ? in_p0 + p * in_ps : pick_buf(J, a.in_buf, w, s), N * ny);
#pragma unroll
        for (int j = 0; j < E; ++j)
          v[j] = (PR && (j == E / 2 - 1 || j == E / 2))
                     ? make_float2(0.f, 0.f)
                     : bload<2>(in, ((rmask >> j) & 1) ? (unsigned)(row + l + L * j) * 8u : kNoElem);
      }
      if (!ADJ && a.store_ckpt) {
        GLOBAL_AS float2* ck = gp(J.ckpt) + img_off(w * J.n_ck + s / J.ck_stride, N, ny) + row;
#pragma unroll
        for (int j = 0; j < E; ++j) ck[l + L * j] = v[j];
      }
      FFT<P>::template run<true, PR ? 1 : 0>(v, tw, lds, l, tab);     // psi_s (real space)
      if constexpr (!ADJ) {
        if (a.stash_slot >= 0) {
          GLOBAL_AS float2* st = gp(J.stash) + img_off(w * J.stash_k + a.stash_slot, N, ny) + row;
#pragma unroll
          for (int j = 0; j < E; ++j) st[l + L * j] = v[j];
        }
        if constexpr (ONE) {
#pragma unroll
          for (int j = 0; j < E; ++j) {
            float sn, cs;
            sincos_phase(sigma * vv[j], &sn, &cs);
            v[j] = cmul(v[j], make_float2(cs, sn));
          }
        } else {
#pragma unroll
          for (int j = 0; j < E; ++j) v[j] = cmul(v[j], tr[j]);
        }
      } else {
        // v = chi_s (adjoint at the post-transmission point); psi_s from the stash
        const GLOBAL_AS float2* st = gp(J.stash) + img_off(w * J.stash_k + a.stash_slot, N, ny) + row;
#pragma unroll
        for (int j = 0; j < E; ++j) {
          float2 tp = cmul(tr[j], st[l + L * j]);
          gacc[j] -= sigma * (v[j].x * tp.y - v[j].y * tp.x);   // -sigma Im(conj(chi) t psi)
          v[j] = cmulc(v[j], tr[j]);                             // conj(t) chi
        }
      }
      if (a.write_out) {
        FFT<P>::template run<false, PR ? 2 : 0>(v, tw, lds, l, tab);
        const __amdgpu_buffer_rsrc_t out =
            image_rsrc(STRIDED ? out_p0 + p * out_ps : pick_buf(J, a.out_buf, w, s), N * ny);
#pragma unroll
        for (int j = 0; j < E; ++j)
          if (!(PR && (j == E / 2 - 1 || j == E / 2)))
            bstore<2>(out, ((wmask >> j) & 1) ? (unsigned)(row + l + L * j) * 8u : kNoElem, v[j]);
      }
    }
    if constexpr (ADJ) {
      GLOBAL_AS float* grow = gp(J.gV) + ((size_t)(t * J.S + s) * ny) * N + row;
#pragma unroll
      for (int j = 0; j < E; ++j) grow[l + L * j] = gacc[j];
    }
  }
}

// ------------------------------------------------------------------------------------------------
// y pass: optional forward y transform, propagator, optional inverse y transform
template <class P, bool DOFWD, bool DOINV>
__global__ __launch_bounds__(kThreads, min_waves<P>()) void k_col(ColArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES, CS = P::LDS_LINE;
  extern __shared__ float2 tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  float2 tw[P::NTW];
  PlanOps<P>::twiddles(tw, l);
  const float2* tab = fft_table_init<P>();
  const int C = a.C, nx = a.nx;
  const int tpi = nx / C, tpw = col_tiles_per_wave(a, tpi);
  const int n_tasks = a.n_waves * tpw;
  for (int task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    int wi, col0;
    col_task(a, task, tpw, tpi, wi, col0);
    const int4 wv = const_at(a.waves, wi);
    CJob& J = job_at(a.jobs, wv.x);
    const int w = wv.y * J.P + wv.z, s = a.s;
    const int kxb = J.kxb;
    const GLOBAL_AS float2* in = pick_buf(J, a.in_buf, w, s);
    GLOBAL_AS float2* out = pick_buf(J, a.out_buf, w, s);
    __syncthreads();
    for (int idx = threadIdx.x; idx < C * N; idx += kThreads) {
      int c = idx % C, r = idx / C;
      tile[c * CS + P::pad(r)] =
          load_if(in + (size_t)r * nx + col0 + c, in_band(col0 + c, kxb, nx));
    }
    __syncthreads();
    for (int cb = wave * LINES; cb < C; cb += kWaves * LINES) {
      const int c = cb + line;
      if ((P::FULL || line < LINES) && c < C) {
        float2* lds = tile + c * CS;
        float2 v[E];
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = lds[P::pad(l + L * j)];
        if constexpr (DOFWD) FFT<P>::template run<false>(v, tw, lds, l, tab);
        const int m = col0 + c;
        const int nm = gp(J.nmax)[m];
        const float2 pxm = gp(J.px)[(size_t)s * nx + m];
        const GLOBAL_AS float2* pys = gp(J.py) + (size_t)s * N;
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int n = l + L * j;
          const int ns = n < N / 2 ? n : n - N;
          float2 d = make_float2(0.f, 0.f);
          if ((ns < 0 ? -ns : ns) <= nm) d = cmul(pxm, pys[n]);
          if (a.conj_prop) d.y = -d.y;
          v[j] = cscale(cmul(v[j], d), a.scale);
        }
        if constexpr (DOINV) FFT<P>::template run<true>(v, tw, lds, l, tab);
#pragma unroll
        for (int j = 0; j < E; ++j) lds[P::pad(l + L * j)] = v[j];
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < C * N; idx += kThreads) {
      int c = idx % C, r = idx / C;
      out[(size_t)r * nx + col0 + c] = tile[c * CS + P::pad(r)];
    }
  }
}

// y pass, block variant: a workgroup of C * L threads owns C adjacent columns; thread (c, l) holds
// rows l + L j of column c (striped for the column transform), loaded and stored with C-wide row
// segments.  The next tile is prefetched into registers while the current one is transformed.
// Twiddles stay in registers; the per-row propagator factors py of the current job sit in LDS.
// (lengths that are not powers of two and E = 16 plans: at most 512 threads, which leaves their
// longer lines enough registers; the odd lengths also ask for 2 wavefronts per SIMD)
template <class P> constexpr int colb_max_threads() { return P::POW2 && P::E <= 8 ? 1024 : 512; }

// LX: the split-layout transforms (SplitFFT; 512 = 8 x 8 x 8) with one workgroup barrier per
// transform instead of two.  Loads, the first forward stage, the last inverse stage and the stores
// keep the numbering (c, l) of the row-segment tiles; the stages in between run on (cx, lx), under
// which wavefront (d, g) holds the 64 / R2 columns g CW ... and every lane lx = R1 h + d of them.
template <class P> constexpr bool colb_lx_ok() { return SplitFFT<P>::OK && 64 % P::radix(1) == 0; }

template <class P, bool DOFWD, bool DOINV, bool PR = false, bool LX = false>
__global__ __launch_bounds__(colb_max_threads<P>(), (P::POW2 ? 1 : 2)) void k_colb(ColArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, CS = P::LDS_LINE, NTW = P::NTW;
  static_assert(!LX || colb_lx_ok<P>(), "plan without split-layout transforms");
  using SF = SplitFFT<P>;
  extern __shared__ float2 lds_mem[];
  const int C = a.C, nx = a.nx;
  const int c = (int)threadIdx.x % C, l = (int)threadIdx.x / C;
  int cx = c, lx = l;
  if constexpr (LX) {
    constexpr int R1 = P::radix(0), R2 = P::radix(1), CW = 64 / R2;
    const int t = (int)threadIdx.x;
    cx = t % CW + CW * (t / (64 * R1));
    lx = R1 * ((t / CW) % R2) + (t / 64) % R1;
  }
  // numbering of the loads (the forward's first stage, or the inverse's input) and of the stores
  const int cl = (LX && !DOFWD) ? cx : c, ll = (LX && !DOFWD) ? lx : l;
  const int cs = (LX && !DOINV) ? cx : c, ls = (LX && !DOINV) ? lx : l;
  float2* reg0 = lds_mem + c * CS;
  float2* reg1 = a.pingpong ? lds_mem + (C + c) * CS : reg0;
  float2* xreg0 = lds_mem + cx * CS;
  float2* xreg1 = a.pingpong ? lds_mem + (C + cx) * CS : xreg0;
  float2* twl = lds_mem + (a.pingpong ? 2 : 1) * C * CS;
  float2* pyl = twl + L * NTW;                       // [N] propagator factors of the current job
  // the lane's twiddles stay in registers for the whole kernel (each transform would otherwise
  // read them from LDS, which the exchanges already keep busy); the first L threads evaluate them
  // once into LDS, every thread copies its lane's
  if ((int)threadIdx.x < L) {
    float2 t[NTW] = {};
    PlanOps<P>::twiddles(t, threadIdx.x);
#pragma unroll
    for (int k = 0; k < NTW; ++k) twl[threadIdx.x * NTW + k] = t[k];
  }
  __syncthreads();
  float2 tw[NTW];
#pragma unroll
  for (int k = 0; k < NTW; ++k) tw[k] = twl[lx * NTW + k];
  const float2* tab = fft_table_init<P>();   // (lengths that are not powers of two)
  int buf = 0;
  const int s = a.s;
  const int tpi = nx / C, tpw = col_tiles_per_wave(a, tpi);
  const int n_tasks = a.n_waves * tpw;
  float2 nxt[E];
  float2 nxt_px = make_float2(0.f, 0.f);
  int nxt_nm = -1;
  // uniform image base + per-lane 32-bit element offsets; a column outside the band reads zeros
  auto load = [&](int wi, int col0) {
    const int4 wv = const_at(a.waves, wi);
    CJob& J = job_at(a.jobs, wv.x);
    const __amdgpu_buffer_rsrc_t in = image_rsrc(pick_buf(J, a.in_buf, wv.y * J.P + wv.z, s), nx * N);
    const int m = col0 + cl;
    const bool inb = in_band(m, J.kxb, nx);
#pragma unroll
    for (int j = 0; j < E; ++j) nxt[j] = bload<0>(in, inb ? (unsigned)((ll + L * j) * nx + m) * 8u : kNoElem);
    nxt_px = gp(J.px)[s * nx + col0 + cx];
    nxt_nm = gp(J.nmax)[col0 + cx];
  };
  int py_job = -1;
  int task = blockIdx.x;
  const int gdiv = (int)gridDim.x / tpw, gmod = (int)gridDim.x - gdiv * tpw;
  ColCursor cur, nxc;
  cur.init(task, tpw);
  nxc = cur;
  nxc.step(gdiv, gmod, tpw);
  if (task < n_tasks) {
    load(cur.wi, col_first(a, cur.jt, tpi));
    py_job = load_py_rows_w<N>(a, cur.wi, pyl);   // with the first tile, one wait for both
  }
  // the first tile is waited for here, so that the loop head has no loads of its own pending:
  // otherwise the wait the compiler places there for them also drains the previous tile's stores
  // on every later iteration
  vmem_drain();
  __syncthreads();
  for (; task < n_tasks; task += gridDim.x) {
    float2 v[E];
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = nxt[j];
    const float2 pxm = nxt_px;
    const int nm = nxt_nm;
    const int wi = cur.wi, col0 = col_first(a, cur.jt, tpi);
    const int4 wv = const_at(a.waves, wi);
    // the output image is resolved here, while the tile's loads are in flight (raw buffer stores:
    // 32-bit element offsets instead of 64-bit addresses per element)
    CJob& J = job_at(a.jobs, wv.x);
    const __amdgpu_buffer_rsrc_t out = image_rsrc(pick_buf(J, a.out_buf, wv.y * J.P + wv.z, s), nx * N);
    // one-way split tiles: the previous tile's readers of the regions are done (with both ways,
    // the other transform's barrier already separates them)
    if constexpr (LX && !(DOFWD && DOINV)) __syncthreads();
    if (wv.x != py_job) {                            // uniform branch
      __syncthreads();                               // previous tile's readers are done
      const GLOBAL_AS float2* pys = gp(job_at(a.jobs, wv.x).py) + s * N;
      for (int i = threadIdx.x; i < N; i += blockDim.x) {
        float2 q = pys[i];
        if (a.conj_prop) q.y = -q.y;
        pyl[i] = q;
      }
      __syncthreads();
      py_job = wv.x;
    }
    if (task + (int)gridDim.x < n_tasks) load(nxc.wi, col_first(a, nxc.jt, tpi));
    cur = nxc;
    nxc.step(gdiv, gmod, tpw);
    if constexpr (DOFWD) {
      if constexpr (LX) {
        SF::fwd1(v, reg0, l);
        __syncthreads();
        SF::fwd2(v, tw, xreg0, xreg0, lx);
        wave_lds_sync();
        SF::fwd3(v, tw, xreg0, lx);
        prune_mid<E, PR ? 2 : 0>(v, 2);
      } else {
        FFT<P>::template run_block<false, PR ? 2 : 0>(v, tw, reg0, reg1, l, buf, tab);
      }
    }
    if constexpr (PR) prune_mid<E, 1>(v, 1);   // M is zero there (also for a raw adjoint input)
    {
      // band-limited propagator (conjugated for the adjoint; pyl is stored conjugated then); the
      // pruned middle registers stay zero
      float2 pxs = cscale(pxm, a.scale);
      if (a.conj_prop) pxs.y = -pxs.y;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if (PR && E >= 4 && (j == E / 2 - 1 || j == E / 2)) continue;
        const int n = lx + L * j;
        const int ns = n < N / 2 ? n : n - N;
        float2 d = cmul(pxs, pyl[n]);
        if ((ns < 0 ? -ns : ns) > nm) d = make_float2(0.f, 0.f);
        v[j] = cmul(v[j], d);
      }
    }
    if constexpr (DOINV) {
      if constexpr (LX) {
        prune_mid<E, PR ? 1 : 0>(v, 1);   // known zeros for the first (transposed) stage
        wave_lds_sync();
        SF::inv1(v, tw, xreg0, lx);
        wave_lds_sync();
        SF::inv2(v, tw, xreg0, xreg1, lx);
        __syncthreads();
        SF::inv3(v, reg1, l);
      } else {
        FFT<P>::template run_block<true, PR ? 1 : 0>(v, tw, reg0, reg1, l, buf, tab);
      }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) bstore<0>(out, (unsigned)((ls + L * j) * nx + col0 + cs) * 8u, v[j]);
  }
}

// y pass, wave-per-column variant: the tile of C columns is staged through LDS with coalesced row
// segments (column stride 1 mod 16: conflict-free transposes); every wavefront then transforms
// whole columns with wave-local exchanges (no barrier inside a transform).  The next tile is
// prefetched into registers while the current one is transformed.  C * 64 / LINES threads.
template <class P> constexpr int colw_max_threads() { return P::E > 8 ? 512 : 1024; }

template <class P, bool DOFWD, bool DOINV, bool PR = false>
__global__ __launch_bounds__(colw_max_threads<P>()) void k_colw(ColArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES, CS = P::LDS_LINE, NTW = P::NTW;
  extern __shared__ float2 lds_mem[];
  const int C = a.C, nx = a.nx;
  const int nthr = blockDim.x;
  float2* tile = lds_mem;
  float2* twl = lds_mem + C * CS;                 // [L][NTW]
  float2* pyl = twl + L * NTW;                    // [N]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  const int c = wave * LINES + line;              // column of the tile owned by this line
  if (threadIdx.x < L) {
    float2 t[NTW] = {};
    PlanOps<P>::twiddles(t, threadIdx.x);
#pragma unroll
    for (int k = 0; k < NTW; ++k) twl[threadIdx.x * NTW + k] = t[k];
  }
  const float2* tw = twl + l * NTW;
  const float2* tab = fft_table_init<P>();
  static_assert(P::FULL, "the staging loops assume whole lines per wavefront");
  const int s = a.s;
  const int tpi = nx / C, tpw = col_tiles_per_wave(a, tpi);
  const int n_tasks = a.n_waves * tpw;
  // staging: C * N elements per tile over C * 64 / LINES threads = E per thread; C is a power of 2
  const int csh = __builtin_ctz(C), cmask = C - 1;
  float2 nxt[E];
  auto load = [&](int wi, int col0) {
    const int4 wv = const_at(a.waves, wi);
    CJob& J = job_at(a.jobs, wv.x);
    const __amdgpu_buffer_rsrc_t in = image_rsrc(pick_buf(J, a.in_buf, wv.y * J.P + wv.z, s), nx * N);
    const int kxb = J.kxb;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int idx = (int)threadIdx.x + k * nthr;
      const int col = col0 + (idx & cmask);
      nxt[k] = bload<0>(in, in_band(col, kxb, nx) ? (unsigned)((idx >> csh) * nx + col) * 8u : kNoElem);
    }
  };
  int py_job = -1;
  int task = blockIdx.x;
  const int gdiv = (int)gridDim.x / tpw, gmod = (int)gridDim.x - gdiv * tpw;
  ColCursor cur, nxc;   // (as in k_colb)
  cur.init(task, tpw);
  nxc = cur;
  nxc.step(gdiv, gmod, tpw);
  if (task < n_tasks) {
    load(cur.wi, col_first(a, cur.jt, tpi));
    py_job = load_py_rows_w<N>(a, cur.wi, pyl);
  }
  vmem_drain();   // (as in k_colb; the rows are read after the next barrier)
  for (; task < n_tasks; task += gridDim.x) {
    const int wi = cur.wi, col0 = col_first(a, cur.jt, tpi);
    const int4 wv = const_at(a.waves, wi);
    __syncthreads();                                // previous tile fully stored from LDS
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int idx = (int)threadIdx.x + k * nthr;
      tile[(idx & cmask) * CS + P::pad(idx >> csh)] = nxt[k];
    }
    if (wv.x != py_job) {
      const GLOBAL_AS float2* pys = gp(job_at(a.jobs, wv.x).py) + s * N;
      for (int i = threadIdx.x; i < N; i += nthr) {
        float2 q = pys[i];
        if (a.conj_prop) q.y = -q.y;
        pyl[i] = q;
      }
      py_job = wv.x;
    }
    if (task + (int)gridDim.x < n_tasks) load(nxc.wi, col_first(a, nxc.jt, tpi));
    cur = nxc;
    nxc.step(gdiv, gmod, tpw);
    __syncthreads();
    CJob& J = job_at(a.jobs, wv.x);
    if (c < C) {
      const int m = col0 + c;
      const int nm = gp(J.nmax)[m];
      const float2 pxm = gp(J.px)[s * nx + m];
      float2* reg = tile + c * CS;
      float2 v[E];
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = reg[P::pad(l + L * j)];
      if constexpr (DOFWD) FFT<P>::template run<false, PR ? 2 : 0>(v, tw, reg, l, tab);
      if constexpr (PR) prune_mid<E, 1>(v, 1);   // M is zero there (also for a raw adjoint input)
      float2 pxs = cscale(pxm, a.scale);
      if (a.conj_prop) pxs.y = -pxs.y;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if (PR && E >= 4 && (j == E / 2 - 1 || j == E / 2)) continue;   // stay zero
        const int n = l + L * j;
        const int ns = n < N / 2 ? n : n - N;
        float2 d = cmul(pxs, pyl[n]);
        if ((ns < 0 ? -ns : ns) > nm) d = make_float2(0.f, 0.f);
        v[j] = cmul(v[j], d);
      }
      if constexpr (DOINV) FFT<P>::template run<true, PR ? 1 : 0>(v, tw, reg, l, tab);
#pragma unroll
      for (int j = 0; j < E; ++j) reg[P::pad(l + L * j)] = v[j];
    }
    __syncthreads();
    GLOBAL_AS float2* out = pick_buf(J, a.out_buf, wv.y * J.P + wv.z, s) + col0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int idx = (int)threadIdx.x + k * nthr;
      out[(idx >> csh) * nx + (idx & cmask)] = tile[(idx & cmask) * CS + P::pad(idx >> csh)];
    }
  }
}

// probe: psi_0 in the (kx, y) representation, W = G_y[a(k)] / (sqrt(nx ny) sqrt(n_aperture))
template <class P>
__global__ __launch_bounds__(kThreads, min_waves<P>()) void k_probe_init(ColArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES, CS = P::LDS_LINE;
  extern __shared__ float2 tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  float2 tw[P::NTW];
  PlanOps<P>::twiddles(tw, l);
  const float2* tab = fft_table_init<P>();
  const int C = a.C, nx = a.nx;
  const int tpi = nx / C;
  const long n_tasks = (long)a.n_waves * tpi;
  for (long task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    const int4 wv = a.waves[task / tpi];
    const int col0 = (int)(task % tpi) * C;
    CJob& J = job_at(a.jobs, wv.x);
    const int w = wv.y * J.P + wv.z;
    GLOBAL_AS float2* out = pick_buf(J, a.out_buf, w, 0);
    const double xp = gp(J.pxy)[2 * wv.z], yp = gp(J.pxy)[2 * wv.z + 1];
    __syncthreads();
    for (int cb = wave * LINES; cb < C; cb += kWaves * LINES) {
      const int c = cb + line;
      if ((P::FULL || line < LINES) && c < C) {
        float2* lds = tile + c * CS;
        const int m = col0 + c;
        const int ms = m < nx / 2 ? m : m - nx;
        const int na = gp(J.nap)[m];
        const double kx = (double)ms / J.lx;
        float2 v[E];
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int n = l + L * j;
          const int ns = n < N / 2 ? n : n - N;
          v[j] = make_float2(0.f, 0.f);
          if ((ns < 0 ? -ns : ns) <= na) {
            const double ky = (double)ns / J.ly;
            const double k2 = kx * kx + ky * ky;
            const double chi = M_PI * J.lambda * J.defocus * k2 +
                               0.5 * M_PI * J.cs * J.lambda * J.lambda * J.lambda * k2 * k2;
            double cyc = chi / (2.0 * M_PI) + kx * xp + ky * yp;
            cyc -= floor(cyc);
            double sn, cs;
            sincos(-2.0 * M_PI * cyc, &sn, &cs);
            v[j] = make_float2((float)cs, (float)sn);
          }
        }
        FFT<P>::template run<true>(v, tw, lds, l, tab);
#pragma unroll
        for (int j = 0; j < E; ++j) lds[P::pad(l + L * j)] = cscale(v[j], J.scale_probe);
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < C * N; idx += kThreads) {
      int c = idx % C, r = idx / C;
      out[(size_t)r * nx + col0 + c] = tile[c * CS + P::pad(r)];
    }
  }
}

// ------------------------------------------------------------------------------------------------
// Resident slice loop (small square grids).  One workgroup of N lines x L lanes keeps a whole wave
// in LDS for all of its slices, as a table T[y][x] whose rows use the padded exchange layout
// (element x of row y at y XS + pad(x)).  The x transforms run on the rows and the y transforms
// on the columns (element y of column c at y XS + pad(c)), each line exchanging in place in its
// own row or column, so no registers hold the wave between the phases and no transposes are
// needed; a workgroup barrier separates the phases.  Per slice step HBM sees the V map of the
// slice and the checkpoints; the wave is read once (entrance, written by the init kernels) and
// written once (exit).  The workgroups are persistent: each takes waves wi = blockIdx.x,
// blockIdx.x + gridDim.x, ... of the class's S-sorted wave list and runs each through its own
// job's slice count.
template <class P> constexpr int res_line_stride() {
  // padded positions 0 .. pad_of(N - 1) of a row, rounded up to an odd count
  return ((P::N - 1 + (P::N - 1) / 8 + 1) | 1);
}
template <class P> constexpr int res_lds_words() { return P::N * res_line_stride<P>() + P::NTW * P::L; }
template <class P> constexpr int max_radix() {
  int m = 0;
  for (int k = 0; k < P::NR; ++k) m = P::radix(k) > m ? P::radix(k) : m;
  return m;
}
// at most 1024 threads, each taking H = N L / threads lines in turn; at most 8 values per lane and
// radix 8 (the registers of a 1024-thread workgroup)
template <class P> constexpr int res_threads() { return P::N * P::L < 1024 ? P::N * P::L : 1024; }
template <class P> constexpr bool res_plan_ok() {
  return P::POW2 && P::FULL && P::N <= 128 && P::E <= 8 && max_radix<P>() <= 8 &&
         (P::N * P::L) % res_threads<P>() == 0 && res_lds_words<P>() * 8 <= 160 * 1024;
}

// A line of the table: position p at base[p * stride] (stride = 1 for rows; pad(c) folded into
// base and stride XS for column c, whose positions are not padded in the row direction)
struct TableLine {
  float2* base;
  int stride, padded;   // padded: rows (p + p/8); columns: p XS
  __device__ __forceinline__ float2& operator()(int p) const {
    return padded ? base[p + (p >> 3)] : base[p * stride];
  }
};

// Transform of one line held striped in v, exchanging in place through acc (register stages only:
// power-of-two plans).  Same stages and index algebra as FFT<P>::run.
template <int N, int L, bool INV, int NS, int TO, class TW, int R, int... Rest>
__device__ __forceinline__ void fft_line_rec(float2* v, const TW& tw, const TableLine& acc, int l) {
  constexpr int E = N / L, B = E / R;
  stage_compute<N, L, R, NS, INV, TO>(v, tw, (const float2*)nullptr, l);
  if constexpr (sizeof...(Rest) > 0) {
    wave_lds_sync();
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int r = 0; r < R; ++r) acc(stage_out_pos<N, L, R, NS>(l, i, r)) = v[i + B * r];
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < E; ++j) v[j] = acc(l + L * j);
    fft_line_rec<N, L, INV, NS * R, (NS > 1) ? TO + B * (R - 1) : TO, TW, Rest...>(v, tw, acc, l);
  }
}
template <class P> struct LineFFT;
template <int N, int L, int... Rs> struct LineFFT<Plan<N, L, Rs...>> {
  template <bool INV, class TW>
  __device__ __forceinline__ static void run(float2* v, const TW& tw, const TableLine& acc, int l) {
    fft_line_rec<N, L, INV, 1, 0, TW, Rs...>(v, tw, acc, l);
  }
};

template <class P>
__global__ __launch_bounds__(res_threads<P>()) void k_resident(ColArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, XS = res_line_stride<P>();
  constexpr int H = P::N * P::L / res_threads<P>(), NL = N / H;   // lines per thread, per pass
  extern __shared__ float2 lds_mem[];
  float2* twl = lds_mem + N * XS;
  const int tid = threadIdx.x, line = tid / L, l = tid % L;
  if (tid < L) {
    float2 t[P::NTW] = {};
    PlanOps<P>::twiddles(t, tid);
#pragma unroll
    for (int k = 0; k < P::NTW; ++k) twl[k * L + tid] = t[k];
  }
  const TwStrided tw{twl + l, L};
  const float inv_n = a.scale;                     // 1 / (N N)
  for (int wi = blockIdx.x; wi < a.n_waves; wi += gridDim.x) {
    const int4 wv = const_at(a.waves, wi);
    CJob& J = job_at(a.jobs, wv.x);
    const int w = wv.y * J.P + wv.z, S = J.S, t = wv.y;
    GLOBAL_AS float2* img = gp(J.W) + img_off(w, N, N);
    // the entrance wave W(kx, y), written by the init kernels, into the table (row layout)
    __syncthreads();                               // the previous wave's last readers are done
#pragma unroll 1
    for (int h = 0; h < H; ++h) {
      const int y = line + h * NL;
      const TableLine row{lds_mem + y * XS, 1, 1};
#pragma unroll
      for (int j = 0; j < E; ++j) row(l + L * j) = img[(size_t)y * N + l + L * j];
    }
    __syncthreads();
    for (int s = 0; s < S; ++s) {
      // x pass on rows y: psi = G_x W, u = exp(i sigma V_s) psi, W' = F_x u
      const bool ck = J.n_ck > 0 && s % J.ck_stride == 0;
      const float sigma = J.sigma;
#pragma unroll 1
      for (int h = 0; h < H; ++h) {
        const int y = line + h * NL;
        const TableLine row{lds_mem + y * XS, 1, 1};
        float2 v[E];
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = row(l + L * j);
        if (ck) {
          GLOBAL_AS float2* cp = gp(J.ckpt) + img_off(w * J.n_ck + s / J.ck_stride, N, N) + (size_t)y * N;
#pragma unroll
          for (int j = 0; j < E; ++j) cp[l + L * j] = v[j];
        }
        LineFFT<P>::template run<true>(v, tw, row, l);
        const GLOBAL_AS float* vrow = gp(J.V) + ((size_t)(t * S + s) * N + y) * N;
        float vv[E];
#pragma unroll
        for (int j = 0; j < E; ++j) vv[j] = vrow[l + L * j];
#pragma unroll
        for (int j = 0; j < E; ++j) {
          float sn, csn;
          sincos_phase(sigma * vv[j], &sn, &csn);
          v[j] = cmul(v[j], make_float2(csn, sn));
        }
        LineFFT<P>::template run<false>(v, tw, row, l);
        wave_lds_sync();
#pragma unroll
        for (int j = 0; j < E; ++j) row(l + L * j) = v[j];
      }
      __syncthreads();
      // y pass on columns c: F_y, band-limited propagator M P_s, then G_y (or the exit wave after
      // the last slice)
      const bool last = s == S - 1;
      const GLOBAL_AS float2* pys = gp(J.py) + (size_t)s * N;
#pragma unroll 1
      for (int h = 0; h < H; ++h) {
        const int c = line + h * NL;
        const TableLine col{lds_mem + P::pad(c), XS, 0};
        float2 v[E];
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = col(l + L * j);
        LineFFT<P>::template run<false>(v, tw, col, l);
        const int nm = gp(J.nmax)[c];
        const float2 pxs = cscale(gp(J.px)[(size_t)s * N + c], last ? J.scale_last : inv_n);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int n = l + L * j;
          const int ns = n < N / 2 ? n : n - N;
          float2 d = cmul(pxs, pys[n]);
          if ((ns < 0 ? -ns : ns) > nm) d = make_float2(0.f, 0.f);
          v[j] = cmul(v[j], d);
        }
        if (last) {
#pragma unroll
          for (int j = 0; j < E; ++j) img[(size_t)(l + L * j) * N + c] = v[j];
        } else {
          LineFFT<P>::template run<true>(v, tw, col, l);
          wave_lds_sync();
#pragma unroll
          for (int j = 0; j < E; ++j) col(l + L * j) = v[j];
        }
      }
      __syncthreads();
    }
  }
}

// plane wave: W(kx, y) = delta_{kx,0} / sqrt(nx ny)
__global__ __launch_bounds__(kThreads) void k_plane_init(ColArgs a) {
  const int nx = a.nx;
  for (long wi = blockIdx.x; wi < a.n_waves; wi += gridDim.x) {
    const int4 wv = a.waves[wi];
    CJob& J = job_at(a.jobs, wv.x);
    const int w = wv.y * J.P + wv.z;
    GLOBAL_AS float2* out = pick_buf(J, a.out_buf, w, 0);
    const size_t n = (size_t)nx * J.ny;
    for (size_t i = threadIdx.x; i < n; i += kThreads)
      out[i] = make_float2((i % nx) == 0 ? J.scale_last : 0.f, 0.f);
  }
}

// Entrance waves of the later snapshots of a probe job: the probe depends on the beam and the
// position only, so the listed wave (job, t, p) is a copy of the wave (job, 0, p) that the probe
// kernel wrote.  Tasks are (wave, span of kCopySpan 16-byte units); each thread issues its four
// loads before its four stores.  All listed waves belong to one grid class (one nx, ny).
constexpr int kCopySpan = 4 * kThreads;
__global__ __launch_bounds__(kThreads) void k_wave_copy(ColArgs a) {
  const int4 w0 = a.waves[0];
  const long n = (long)job_at(a.jobs, w0.x).nx * job_at(a.jobs, w0.x).ny / 2;   // nx is even
  const long spans = (n + kCopySpan - 1) / kCopySpan;
  const long n_tasks = (long)a.n_waves * spans;
  for (long t = blockIdx.x; t < n_tasks; t += gridDim.x) {
    // waves copied at the same time share a few sources: each starts at its own span
    const long wi = t / spans;
    const int4 wv = a.waves[wi];
    CJob& J = job_at(a.jobs, wv.x);
    const GLOBAL_AS float4* src = (const GLOBAL_AS float4*)pick_buf(J, a.out_buf, wv.z, 0);
    GLOBAL_AS float4* dst = (GLOBAL_AS float4*)pick_buf(J, a.out_buf, wv.y * J.P + wv.z, 0);
    const long b = ((t % spans + wi * 37) % spans) * kCopySpan + threadIdx.x;
    if (b + 3 * kThreads < n) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = src[b + u * kThreads];
#pragma unroll
      for (int u = 0; u < 4; ++u) dst[b + u * kThreads] = v[u];
    } else {
      for (long i = b; i < n; i += kThreads) dst[i] = src[i];
    }
  }
}

// ------------------------------------------------------------------------------------------------
// plain batched 2-D transforms of contiguous images
// column tiles of width C that hold a column kept by the band kxb (all of them for kxb < 0):
// tiles [0, lo) and [hs, nx / C)
__host__ __device__ inline void plain_live_tiles(int nx, int C, int kxb, int& lo, int& hs) {
  const int tpi = nx / C;
  lo = tpi;
  hs = tpi;
  if (kxb >= 0) {
    lo = min(tpi, kxb / C + 1);
    hs = max(lo, (nx - kxb) / C);
  }
}

template <class P, bool INV, bool REAL_IN, bool REAL_OUT>
__global__ __launch_bounds__(kThreads, min_waves<P>()) void k_row_plain(PlainArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES;
  __shared__ float2 lds_all[kWaves * LINES * P::LDS_LINE];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  float2* lds = lds_all + (wave * LINES + line) * P::LDS_LINE;
  float2 tw[P::NTW];
  PlanOps<P>::twiddles(tw, l);
  const float2* tab = fft_table_init<P>();
  // paired (real output only): task = (pair p, row y) reads row y of image 2p and writes the real
  // part to image 2p and the imaginary part to image 2p + 1 (if there is one)
  const bool pair = REAL_OUT && a.pair;
  const long n_rows = pair ? (long)((a.n_img + 1) / 2) * a.ny : (long)a.n_img * a.ny;
  const long n_tasks = n_rows;
  const long stride = (long)gridDim.x * kWaves * LINES;
  for (long base = ((long)blockIdx.x * kWaves + wave) * LINES; base < n_tasks; base += stride) {
    const long task = base + line;
    if ((!P::FULL && line >= LINES) || task >= n_tasks) continue;
    const long img = pair ? 2 * (task / a.ny) : task / a.ny;
    const size_t off = ((size_t)img * a.ny + (size_t)(task % a.ny)) * N;
    float2 v[E];
    if constexpr (REAL_IN) {
      const float* in = (const float*)a.in + off;
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = make_float2(in[l + L * j], 0.f);
    } else {
      const float2* in = (const float2*)a.in + off;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int m = l + L * j;
        v[j] = (a.kxb >= 0 && m > a.kxb && m < N - a.kxb) ? make_float2(0.f, 0.f) : in[m];
      }
    }
    FFT<P>::template run<INV>(v, tw, lds, l, tab);
    if constexpr (REAL_OUT) {
      auto empty = [&](long m) {
        if (!a.csr) return false;
        const int* o = a.csr + (size_t)(a.csr_t0 + m / a.csr_S) * (a.csr_S * a.csr_nsp + 1) +
                       (m % a.csr_S) * a.csr_nsp;
        return o[0] == o[a.csr_nsp];
      };
      float* out = (float*)a.out + off;
      const bool za = pair && empty(img);
#pragma unroll
      for (int j = 0; j < E; ++j) out[l + L * j] = za ? 0.f : v[j].x;
      if (pair && img + 1 < a.n_img) {
        float* out2 = out + (size_t)a.ny * N;
        const bool zb = empty(img + 1);
#pragma unroll
        for (int j = 0; j < E; ++j) out2[l + L * j] = zb ? 0.f : v[j].y;
      }
    } else if (REAL_IN && a.kxb >= 0 && a.C > 0) {
      // band-limited forward transform: columns of the column pass's dead tiles are not written,
      // the other columns outside the band are written as zeros (their column transforms are zero)
      float2* out = (float2*)a.out + off;
      int lo, hs;
      plain_live_tiles(N, a.C, a.kxb, lo, hs);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int m = l + L * j;
        if (m < lo * a.C || m >= hs * a.C)
          out[m] = (m > a.kxb && m < N - a.kxb) ? make_float2(0.f, 0.f) : v[j];
      }
    } else {
      float2* out = (float2*)a.out + off;
#pragma unroll
      for (int j = 0; j < E; ++j) out[l + L * j] = v[j];
    }
  }
}

template <class P, bool INV>
__global__ __launch_bounds__(kThreads, min_waves<P>()) void k_col_plain(PlainArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES, CS = P::LDS_LINE;
  extern __shared__ float2 tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  float2 tw[P::NTW];
  PlanOps<P>::twiddles(tw, l);
  const float2* tab = fft_table_init<P>();
  const int C = a.C, nx = a.nx;
  const int tpi = nx / C;
  // a tile of columns that are all zero stays zero (and the row pass does not read it): the tasks
  // cover only the tiles [0, lo) and [hs, tpi) that hold a kept column
  int lo, hs;
  plain_live_tiles(nx, C, a.kxb, lo, hs);
  const int nlt = lo + (tpi - hs);
  // paired: task = (pair p, column tile) transforms A + iB of images 2p, 2p + 1 into image 2p
  const int n_im = a.pair ? (a.n_img + 1) / 2 : a.n_img;
  const long n_tasks = (long)n_im * nlt;
  for (long task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    const long img = a.pair ? 2 * (task / nlt) : task / nlt;
    const size_t ioff = (size_t)img * nx * N;
    const int k = (int)(task % nlt);
    const int col0 = (k < lo ? k : hs + (k - lo)) * C;
    const float2* in = (const float2*)a.in + ioff;
    float2* out = (float2*)a.out + ioff;
    const bool second = a.pair && img + 1 < a.n_img;
    __syncthreads();
    for (int idx = threadIdx.x; idx < C * N; idx += kThreads) {
      int c = idx % C, r = idx / C;
      const bool zero = a.kyb >= 0 && r > a.kyb && r < N - a.kyb;
      float2 v = make_float2(0.f, 0.f);
      if (!zero) {
        v = in[(size_t)r * nx + col0 + c];
        if (second) {
          const float2 b = in[(size_t)nx * N + (size_t)r * nx + col0 + c];
          v = make_float2(v.x - b.y, v.y + b.x);
        }
      }
      tile[c * CS + P::pad(r)] = v;
    }
    __syncthreads();
    for (int cb = wave * LINES; cb < C; cb += kWaves * LINES) {
      const int c = cb + line;
      if ((P::FULL || line < LINES) && c < C) {
        float2* lds = tile + c * CS;
        float2 v[E];
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = lds[P::pad(l + L * j)];
        FFT<P>::template run<INV>(v, tw, lds, l, tab);
#pragma unroll
        for (int j = 0; j < E; ++j) lds[P::pad(l + L * j)] = v[j];
      }
    }
    __syncthreads();
    const int rows = a.rows_out > 0 ? a.rows_out : N;
    float mx = 0.f;
    for (int idx = threadIdx.x; idx < C * rows; idx += kThreads) {
      int c = idx % C, r = idx / C;
      const float2 v = tile[c * CS + P::pad(r)];
      out[(size_t)r * nx + col0 + c] = v;
      if constexpr (!INV) mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    if constexpr (!INV) {
      // the map's maximum: a wavefront maximum, then one atomic maximum per wavefront on the bits
      // (non-negative floats order as their bit patterns)
      if (a.absmax) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) atomicMax(reinterpret_cast<unsigned*>(a.absmax) + img, __float_as_uint(mx));
      }
    }
  }
}

// ------------------------------------------------------------------------------------------------
// launchers

int row_lines_per_wave(int n, int plan) {
  int lines = 0;
  with_plan(n, plan, [&](auto p) { lines = decltype(p)::LINES; });
  return lines;
}

int col_lds_bytes(int n, int plan, int C) {
  int b = 0;
  with_plan(n, plan, [&](auto p) { b = C * decltype(p)::LDS_LINE * (int)sizeof(float2); });
  return b;
}

hipError_t launch_row(int n, int plan, bool adj, const RowArgs& a, int grid, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    if (adj) {
      hipLaunchKernelGGL((k_row<P, true>), dim3(grid), dim3(kThreads), 0, st, a);
    } else {
      auto go = [&](auto one) {
        constexpr bool ONE = decltype(one)::value;
        bool done = false;
        if constexpr (P::E >= 8 && P::POW2) {
          if (a.prune) {
            hipLaunchKernelGGL((k_row<P, false, true, ONE>), dim3(grid), dim3(kThreads), 0, st, a);
            done = true;
          }
        }
        if (!done) hipLaunchKernelGGL((k_row<P, false, false, ONE>), dim3(grid), dim3(kThreads), 0, st, a);
      };
      if (a.single_pos) go(std::true_type{});
      else go(std::false_type{});
    }
    e = hipGetLastError();
  });
  return e;
}

// whether a plan of n points can skip its two middle registers for a band limit of kb
// (largest kept |index|)
bool plan_prunable(int n, int plan, int kb) {
  bool ok = false;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    ok = P::E >= 8 && P::POW2 && kb <= P::N / 2 - P::L - 1;
  });
  return ok;
}

// grid sizes with FFT plans: powers of two 16..1024 and the odd-factor lengths
const int kGridSizes[] = {16, 32, 64, 128, 256, 512, 1024, 560, 1000};

bool grid_size_ok(int n) {
  for (int g : kGridSizes)
    if (g == n) return true;
  return false;
}

// LDS a plan's kernels hold besides their dynamic tile (the root table of an LDS last stage)
int plan_static_lds(int n, int plan) {
  int b = 0;
  with_plan(n, plan, [&](auto p) { b = decltype(p)::TABN * (int)sizeof(float2); });
  return b;
}

// whether a plan's block y pass has the split-layout transforms, and their columns per wavefront
int col_block_lx_cols(int n, int plan) {
  int cw = 0;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    if constexpr (colb_lx_ok<P>()) cw = 64 / P::radix(1);
  });
  return cw;
}

// which y-pass kinds a plan supports: 0 and 1 always; 2 (wave per column) whole lines per
// wavefront
bool plan_kind_ok(int n, int plan, int kind) {
  bool ok = false;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    ok = kind == 0 || kind == 1 || (kind == 2 && P::FULL);
  });
  return ok;
}

// Dynamic LDS limits are raised once per context creation (never during graph capture).
void prepare_dynamic_lds(int max_bytes) {
  for (int n : kGridSizes)
    for (int idx = 0; idx < n_plans(n); ++idx)
      with_plan(n, idx, [&](auto p) {
        using P = decltype(p);
        const int attr = hipFuncAttributeMaxDynamicSharedMemorySize;
        (void)hipFuncSetAttribute((const void*)k_col<P, true, true>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_col<P, true, false>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_col<P, false, true>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_probe_init<P>, (hipFuncAttribute)attr, max_bytes);
        if constexpr (res_plan_ok<P>())
          (void)hipFuncSetAttribute((const void*)k_resident<P>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_colb<P, true, true>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_colb<P, true, false>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_colb<P, false, true>, (hipFuncAttribute)attr, max_bytes);
        if constexpr (P::FULL) {
          (void)hipFuncSetAttribute((const void*)k_colw<P, true, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colw<P, true, false>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colw<P, false, true>, (hipFuncAttribute)attr, max_bytes);
        }
        if constexpr (P::E >= 8 && P::POW2) {
          (void)hipFuncSetAttribute((const void*)k_colb<P, true, true, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, true, false, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, false, true, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colw<P, true, true, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colw<P, true, false, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colw<P, false, true, true>, (hipFuncAttribute)attr, max_bytes);
        }
        if constexpr (colb_lx_ok<P>()) {
          (void)hipFuncSetAttribute((const void*)k_colb<P, true, true, false, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, true, false, false, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, false, true, false, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, true, true, true, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, true, false, true, true>, (hipFuncAttribute)attr, max_bytes);
          (void)hipFuncSetAttribute((const void*)k_colb<P, false, true, true, true>, (hipFuncAttribute)attr, max_bytes);
        }
        (void)hipFuncSetAttribute((const void*)k_col_plain<P, true>, (hipFuncAttribute)attr, max_bytes);
        (void)hipFuncSetAttribute((const void*)k_col_plain<P, false>, (hipFuncAttribute)attr, max_bytes);
      });
  (void)hipGetLastError();
}

int plan_lanes(int n, int plan) {
  int L = 0;
  with_plan(n, plan, [&](auto p) { L = decltype(p)::L; });
  return L;
}

int col_block_max_threads(int n, int plan) {
  int t = 0;
  with_plan(n, plan, [&](auto p) { t = colb_max_threads<decltype(p)>(); });
  return t;
}

int col_block_lds_bytes(int n, int plan, int C, int pingpong) {
  int tw = 0;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    tw = (P::L * P::NTW + P::N) * (int)sizeof(float2);
  });
  return (pingpong ? 2 : 1) * col_lds_bytes(n, plan, C) + tw;
}

int col_wave_lds_bytes(int n, int plan, int C) {
  int b = 0;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    b = (C * P::LDS_LINE + P::L * P::NTW + P::N) * (int)sizeof(float2);
  });
  return b;
}

int col_wave_threads(int n, int plan, int C) {
  int t = 0;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    t = (C / P::LINES) * 64;
    // every wavefront must own LINES whole columns, within the kernel's launch bound
    if (!P::FULL || C % P::LINES != 0 || t > colw_max_threads<P>()) t = 1 << 30;
  });
  return t;
}

hipError_t launch_col(int n, int plan, int kind, bool dofwd, bool doinv, const ColArgs& a,
                      int grid, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  if (kind == 2) {
    with_plan(n, plan, [&](auto p) {
      using P = decltype(p);
      if constexpr (!P::FULL) {
        e = hipErrorInvalidValue;
        return;
      } else {
        const int lds = col_wave_lds_bytes(n, plan, a.C);
        const int threads = col_wave_threads(n, plan, a.C);
        auto go = [&](auto pr) {
          constexpr bool PR = decltype(pr)::value;
          if (dofwd && doinv)
            hipLaunchKernelGGL((k_colw<P, true, true, PR>), dim3(grid), dim3(threads), lds, st, a);
          else if (dofwd)
            hipLaunchKernelGGL((k_colw<P, true, false, PR>), dim3(grid), dim3(threads), lds, st, a);
          else
            hipLaunchKernelGGL((k_colw<P, false, true, PR>), dim3(grid), dim3(threads), lds, st, a);
        };
        bool done = false;
        if constexpr (P::E >= 8 && P::POW2) {
          if (a.prune) {
            go(std::true_type{});
            done = true;
          }
        }
        if (!done) go(std::false_type{});
        e = hipGetLastError();
      }
    });
    return e;
  }
  if (kind == 1) {
    with_plan(n, plan, [&](auto p) {
      using P = decltype(p);
      const int lds = ((a.pingpong ? 2 : 1) * a.C * P::LDS_LINE + P::L * P::NTW + P::N) *
                      (int)sizeof(float2);
      const int threads = a.C * P::L;
      auto go2 = [&](auto pr, auto lx) {
        constexpr bool PR = decltype(pr)::value, LX = decltype(lx)::value;
        if (dofwd && doinv)
          hipLaunchKernelGGL((k_colb<P, true, true, PR, LX>), dim3(grid), dim3(threads), lds, st, a);
        else if (dofwd)
          hipLaunchKernelGGL((k_colb<P, true, false, PR, LX>), dim3(grid), dim3(threads), lds, st, a);
        else
          hipLaunchKernelGGL((k_colb<P, false, true, PR, LX>), dim3(grid), dim3(threads), lds, st, a);
      };
      // pingpong == 2: the split-layout transforms where the tile is whole wavefronts of their
      // columns (the same results either way)
      auto go = [&](auto pr) {
        if constexpr (colb_lx_ok<P>()) {
          if (a.pingpong == 2 && a.C % (64 / P::radix(1)) == 0) {
            go2(pr, std::true_type{});
            return;
          }
        }
        go2(pr, std::false_type{});
      };
      bool done = false;
      if constexpr (P::E >= 8 && P::POW2) {
        if (a.prune) {
          go(std::true_type{});
          done = true;
        }
      }
      if (!done) go(std::false_type{});
      e = hipGetLastError();
    });
    return e;
  }
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    const int lds = a.C * P::LDS_LINE * (int)sizeof(float2);
    if (dofwd && doinv)
      hipLaunchKernelGGL((k_col<P, true, true>), dim3(grid), dim3(kThreads), lds, st, a);
    else if (dofwd)
      hipLaunchKernelGGL((k_col<P, true, false>), dim3(grid), dim3(kThreads), lds, st, a);
    else
      hipLaunchKernelGGL((k_col<P, false, true>), dim3(grid), dim3(kThreads), lds, st, a);
    e = hipGetLastError();
  });
  return e;
}

hipError_t launch_probe_init(int n, int plan, const ColArgs& a, int grid, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  with_plan(n, plan, [&](auto p) {
    using P = decltype(p);
    const int lds = a.C * P::LDS_LINE * (int)sizeof(float2);
    hipLaunchKernelGGL((k_probe_init<P>), dim3(grid), dim3(kThreads), lds, st, a);
    e = hipGetLastError();
  });
  return e;
}

// resident slice loop: plan of an N x N grid that fits (0 if none), its threads and LDS bytes
static int res_plan_for(int n) {
  // the first plan of n whose lines fill whole wavefronts and whose wave fits one workgroup
  int found = -1;
  for (int idx = 0; idx < n_plans(n) && found < 0; ++idx)
    with_plan(n, idx, [&](auto p) {
      if constexpr (res_plan_ok<decltype(p)>()) found = idx;
    });
  return found;
}

bool resident_ok(int nx, int ny) { return nx == ny && res_plan_for(nx) >= 0; }

int resident_workgroups_per_cu(int n, int max_lds) {
  const int idx = res_plan_for(n);
  int per = 0;
  if (idx >= 0)
    with_plan(n, idx, [&](auto p) {
      using P = decltype(p);
      if constexpr (res_plan_ok<P>()) {
        const int by_lds = max_lds / (res_lds_words<P>() * 8);
        const int by_threads = 2048 / res_threads<P>();
        per = by_lds < by_threads ? by_lds : by_threads;
      }
    });
  return per > 0 ? per : 1;
}

hipError_t launch_resident(int n, const ColArgs& a, int grid, hipStream_t st) {
  const int idx = res_plan_for(n);
  hipError_t e = hipErrorInvalidValue;
  if (idx < 0) return e;
  with_plan(n, idx, [&](auto p) {
    using P = decltype(p);
    if constexpr (res_plan_ok<P>()) {
      hipLaunchKernelGGL((k_resident<P>), dim3(grid), dim3(res_threads<P>()), res_lds_words<P>() * 8, st, a);
      e = hipGetLastError();
    }
  });
  return e;
}

hipError_t launch_plane_init(const ColArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_plane_init, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_wave_copy(const ColArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_wave_copy, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// columns per tile of the plain column transform: a power of two that divides nx.  Narrow tiles
// keep the LDS tile small enough for several workgroups per CU (measured: 16 columns at 256
// points and 8 from 512 on beat 32 and 16)
static int plain_cols(int nx, int n) {
  int c = (n <= 64) ? 64 : (n <= 128 ? 32 : (n <= 256 ? 16 : 8));
  if (c > nx) c = nx;
  while (c > 1 && nx % c != 0) c /= 2;
  return c;
}

hipError_t launch_ifft2_real(int nx, int ny, float2* vk, float* V, int n_img, int kxb, int kyb,
                             int pair, const int* csr, int t0, int S, int nsp, hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  hipError_t e = hipErrorInvalidValue;
  PlainArgs a{vk, vk, n_img, nx, ny, plain_cols(nx, ny), kxb, kyb, pair};
  const long n_im = pair ? (n_img + 1) / 2 : n_img;
  with_plan(ny, 0, [&](auto p) {
    using P = decltype(p);
    const int lds = a.C * P::LDS_LINE * (int)sizeof(float2);
    int lo, hs;
    plain_live_tiles(nx, a.C, kxb, lo, hs);
    long tasks = n_im * (lo + (nx / a.C - hs));
    int grid = (int)(tasks < 4096 ? tasks : 4096);
    hipLaunchKernelGGL((k_col_plain<P, true>), dim3(grid), dim3(kThreads), lds, st, a);
    e = hipGetLastError();
  });
  if (e != hipSuccess) return e;
  PlainArgs b{vk, V, n_img, nx, ny, 0, kxb, -1, pair, csr, t0, S, nsp};
  with_plan(nx, 0, [&](auto p) {
    using P = decltype(p);
    long tasks = n_im * ny;
    long g = (tasks + kWaves * P::LINES - 1) / (kWaves * P::LINES);
    int grid = (int)(g < 4096 ? g : 4096);
    hipLaunchKernelGGL((k_row_plain<P, true, false, true>), dim3(grid), dim3(kThreads), 0, st, b);
    e = hipGetLastError();
  });
  return e;
}

hipError_t launch_fft2_real(int nx, int ny, const float* g, float2* gk, int n_img, int kxb,
                            int rows_out, float* absmax, hipStream_t st) {
  if (n_img <= 0) return hipSuccess;
  if (rows_out < 0 || rows_out > ny) return hipErrorInvalidValue;
  hipError_t e = hipErrorInvalidValue;
  const int C = plain_cols(nx, ny);
  const int band = kxb >= 0 && kxb < nx / 2 ? kxb : -1;
  PlainArgs b{g, gk, n_img, nx, ny, C, band};
  with_plan(nx, 0, [&](auto p) {
    using P = decltype(p);
    long tasks = (long)n_img * ny;
    long gg = (tasks + kWaves * P::LINES - 1) / (kWaves * P::LINES);
    int grid = (int)(gg < 4096 ? gg : 4096);
    hipLaunchKernelGGL((k_row_plain<P, false, true, false>), dim3(grid), dim3(kThreads), 0, st, b);
    e = hipGetLastError();
  });
  if (e != hipSuccess) return e;
  PlainArgs a{gk, gk, n_img, nx, ny, C, band};
  a.rows_out = rows_out;
  a.absmax = absmax;
  with_plan(ny, 0, [&](auto p) {
    using P = decltype(p);
    const int lds = a.C * P::LDS_LINE * (int)sizeof(float2);
    int lo, hs;
    plain_live_tiles(nx, a.C, band, lo, hs);
    long tasks = (long)n_img * (lo + (nx / a.C - hs));
    int grid = (int)(tasks < 4096 ? tasks : 4096);
    hipLaunchKernelGGL((k_col_plain<P, false>), dim3(grid), dim3(kThreads), lds, st, a);
    e = hipGetLastError();
  });
  return e;
}

}  // namespace tacaw
