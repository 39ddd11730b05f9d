// Time auto-correlation spectrum from the exit-wave stack.
//
// For each momentum q the snapshots of a segment form a line of length n_e along time (stride
// n_pos * nx * ny in memory).  A workgroup owns Qt consecutive q (a 128-byte or wider row segment),
// stages a segment's n_e x Qt block through LDS with coalesced loads, and every wave transforms
// whole time lines with the same register/LDS Stockham FFT as the slice kernels.  |Phi|^2 is
// accumulated in registers over segments and probe positions, so the exit stack is read once per
// segment and the periodogram is written once.  The normalisation sum is a fixed-order two-pass
// reduction in float64 (deterministic, no atomics).
#include "internal.hpp"

namespace tacaw {

template <class F> static bool with_time_plan(int n, F&& f) {
  switch (n) {
    case 16: f(P16a{}); return true;
    case 32: f(P32a{}); return true;
    case 64: f(P64a{}); return true;
    case 128: f(P128a{}); return true;
    case 256: f(P256a{}); return true;
    case 512: f(P512a{}); return true;
    case 1024: f(P1024a{}); return true;
    default: return false;
  }
}

template <class P> constexpr int q_tile() { return 4 * P::LINES > 16 ? 4 * P::LINES : 16; }

template <class P>
__global__ __launch_bounds__(kThreads) void k_periodogram(SpecArgs a) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES, CS = P::LDS_LINE;
  constexpr int QT = q_tile<P>();
  constexpr int QPASS = (QT + kWaves * LINES - 1) / (kWaves * LINES);
  extern __shared__ float2 tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  float2 tw[P::NTW];
  PlanOps<P>::twiddles(tw, l);
  const long n_tasks = a.nq / QT;
  // blocks of at most 16 elements per thread are fetched into registers one (position, segment)
  // block ahead, so that their loads overlap the previous block's transforms
  constexpr int PER = N * QT / kThreads;
  constexpr bool PF = (N * QT) % kThreads == 0 && kThreads % QT == 0 && PER <= 16;
  float2 nxt[PF ? PER : 1];
  for (long task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    const size_t q0 = (size_t)task * QT;
    // thread: q index threadIdx.x % QT, times threadIdx.x / QT + (kThreads / QT) i (kThreads is a
    // multiple of QT), so one per-thread base and uniform offsets per (position, segment, i)
    const size_t tstride = (size_t)a.Ps * a.nq;   // elements from one snapshot to the next
    const float2* mine = a.exit + (size_t)((int)threadIdx.x / QT) * tstride + q0 + (int)threadIdx.x % QT;
    auto fetch = [&](int p, int g) {
      const size_t base = (size_t)(g * a.hop) * tstride + (size_t)(a.p0 + p) * a.nq;
#pragma unroll
      for (int i = 0; i < (PF ? PER : 1); ++i)
        nxt[i] = mine[base + (size_t)(i * (kThreads / QT)) * tstride];
    };
    if constexpr (PF) fetch(0, 0);
    float acc[QPASS][E];
#pragma unroll
    for (int k = 0; k < QPASS; ++k)
#pragma unroll
      for (int j = 0; j < E; ++j) acc[k][j] = 0.f;
    for (int p = 0; p < a.Pn; ++p) {
      for (int g = 0; g < a.G; ++g) {
        __syncthreads();
        if constexpr (PF) {
#pragma unroll
          for (int i = 0; i < PER; ++i) {
            const int idx = (int)threadIdx.x + i * kThreads, qi = idx % QT, t = idx / QT;
            tile[qi * CS + lds_pad(t)] = nxt[i];
          }
          const int gn = g + 1 < a.G ? g + 1 : 0, pn = g + 1 < a.G ? p : p + 1;
          if (pn < a.Pn) fetch(pn, gn);
        } else {
          for (int idx = threadIdx.x; idx < N * QT; idx += kThreads) {
            const int qi = idx % QT, t = idx / QT;
            tile[qi * CS + lds_pad(t)] =
                a.exit[((size_t)(g * a.hop + t) * a.Ps + a.p0 + p) * a.nq + q0 + qi];
          }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < QPASS; ++k) {
          const int qi = (k * kWaves + wave) * LINES + line;
          if (qi < QT) {
            float2* lds = tile + qi * CS;
            float2 v[E];
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = lds[lds_pad(l + L * j)];
            FFT<P>::template run<false>(v, tw, lds, l);
#pragma unroll
            for (int j = 0; j < E; ++j) acc[k][j] = fmaf(v[j].x, v[j].x, fmaf(v[j].y, v[j].y, acc[k][j]));
          }
        }
      }
    }
    // stage through LDS as float [QT][N] and store rows k with QT consecutive q
    __syncthreads();
    float* ft = (float*)tile;
    const float invG = 1.0f / (float)a.G;
#pragma unroll
    for (int k = 0; k < QPASS; ++k) {
      const int qi = (k * kWaves + wave) * LINES + line;
      if (qi < QT) {
#pragma unroll
        for (int j = 0; j < E; ++j) ft[qi * (N + 1) + l + L * j] = acc[k][j] * invG;
      }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * QT; idx += kThreads) {
      const int qi = idx % QT, kk = idx / QT;
      float v = ft[qi * (N + 1) + kk];
      float* dst = a.P + (size_t)kk * a.nq + q0 + qi;
      *dst = a.accumulate ? (*dst + v) : v;
    }
  }
}

hipError_t launch_periodogram(const SpecArgs& a, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  with_time_plan(a.n_e, [&](auto p) {
    using P = decltype(p);
    constexpr int QT = q_tile<P>();
    int lds = QT * P::LDS_LINE * (int)sizeof(float2);
    int lds2 = QT * (P::N + 1) * (int)sizeof(float);
    if (lds2 > lds) lds = lds2;
    hipFuncSetAttribute((const void*)k_periodogram<P>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        lds);
    long tasks = a.nq / QT;
    int grid = (int)(tasks < 8192 ? tasks : 8192);
    hipLaunchKernelGGL((k_periodogram<P>), dim3(grid), dim3(kThreads), lds, st, a);
    e = hipGetLastError();
  });
  return e;
}

int spectrum_q_tile(int n_e) {
  int qt = 0;
  with_time_plan(n_e, [&](auto p) { qt = q_tile<decltype(p)>(); });
  return qt;
}

// ---------------------------------------------------------------------------------------------
// normalisation: Z = sum_k sum_q K[k] P[k][q]  (fixed-order two-pass, float64)
constexpr int kRedThreads = 256;

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kRedThreads) void k_fin_partial(FinArgs a) {
  __shared__ double sh[kRedThreads];
  const size_t nq = (size_t)a.nx * a.ny, total = nq * a.n_e;
  const size_t per = (total + a.n_part - 1) / a.n_part;
  const size_t b0 = (size_t)blockIdx.x * per, b1 = b0 + per < total ? b0 + per : total;
  double acc = 0.0;
  for (size_t i = b0 + threadIdx.x; i < b1; i += kRedThreads)
    acc += (double)a.K[i / nq] * (double)a.P[i];
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_fin_total(const double* partial, int n,
                                                          double* out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRedThreads) acc += partial[i];
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) *out = s;
}

__device__ __forceinline__ int unshift(int i, int nout, int n) {
  int f = i - nout / 2;            // signed frequency
  return f < 0 ? f + n : f;        // storage index
}

__global__ __launch_bounds__(256) void k_fin_write(FinArgs a) {
  const size_t nout = (size_t)a.n_e * a.nqy * a.nqx;
  const double invZ = 1.0 / *a.norm;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < nout; i += (size_t)gridDim.x * 256) {
    const int ix = (int)(i % a.nqx), iy = (int)((i / a.nqx) % a.nqy), ie = (int)(i / ((size_t)a.nqx * a.nqy));
    const int k = unshift(ie, a.n_e, a.n_e), qy = unshift(iy, a.nqy, a.ny), qx = unshift(ix, a.nqx, a.nx);
    const double v = (double)a.K[k] * (double)a.P[(size_t)k * a.nx * a.ny + (size_t)qy * a.nx + qx];
    a.S[i] = (float)(v * invZ);
  }
}

// Kubo factors in DFT order computed on the device, in the host's float64 order of operations:
// E_k = 2 pi hbar k' / (n_e dt), x = beta E_k, K = 1 + x/2 + x^2/12 for |x| < 1e-4, else
// x / (-expm1(-x)) (eq:kubo_vs_normal)
__global__ __launch_bounds__(256) void k_kubo_fill(float* K, int n_e, double dt_fs, double beta) {
  const double two_pi_hbar = 2.0 * 3.14159265358979323846 * 0.6582119569;
  for (int i = (int)threadIdx.x; i < n_e; i += 256) {
    const int kp = i < n_e / 2 ? i : i - n_e;
    const double e = two_pi_hbar * (double)kp / ((double)n_e * dt_fs);
    const double x = beta * e;
    const double k = fabs(x) < 1e-4 ? 1.0 + x / 2.0 + x * x / 12.0 : x / (-expm1(-x));
    K[i] = (float)k;
  }
}

hipError_t launch_kubo_fill(float* K, int n_e, double dt_fs, double beta, hipStream_t st) {
  hipLaunchKernelGGL(k_kubo_fill, dim3(1), dim3(256), 0, st, K, n_e, dt_fs, beta);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_fin_partial, dim3(a.n_part), dim3(kRedThreads), 0, st, a);
  hipLaunchKernelGGL(k_fin_total, dim3(1), dim3(kRedThreads), 0, st, a.partial, a.n_part, a.norm);
  const size_t nout = (size_t)a.n_e * a.nqy * a.nqx;
  size_t blocks = (nout + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fin_write, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// adjoint: D = sum(g S); dL/dP = (K/Z)(g - D); G_phi(g hop + t) += (2/G) IDFT_t[dL/dP Phi_g]
__global__ __launch_bounds__(kRedThreads) void k_dot_partial(const float* x, const float* y,
                                                            size_t n, int n_part, double* partial) {
  __shared__ double sh[kRedThreads];
  const size_t per = (n + n_part - 1) / n_part;
  const size_t b0 = (size_t)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  double acc = 0.0;
  for (size_t i = b0 + threadIdx.x; i < b1; i += kRedThreads) acc += (double)x[i] * (double)y[i];
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <class P>
__global__ __launch_bounds__(kThreads) void k_spec_bwd(SpecBwdArgs a, const double* dsum) {
  constexpr int N = P::N, L = P::L, E = P::E, LINES = P::LINES, CS = P::LDS_LINE;
  constexpr int QT = q_tile<P>();
  constexpr int QPASS = (QT + kWaves * LINES - 1) / (kWaves * LINES);
  extern __shared__ float2 tile[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int line = lane / L, l = lane % L;
  float2 tw[P::NTW];
  PlanOps<P>::twiddles(tw, l);
  const double Z = *a.norm, D = *dsum;
  const float two_over_G = 2.0f / (float)a.G;
  const long n_tasks = a.nq / QT;
  for (long task = blockIdx.x; task < n_tasks; task += gridDim.x) {
    const size_t q0 = (size_t)task * QT;
    // dL/dP for the lines this lane owns (independent of segment and position)
    float gp[QPASS][E];
#pragma unroll
    for (int k = 0; k < QPASS; ++k) {
      const int qi = (k * kWaves + wave) * LINES + line;
      const size_t q = q0 + (qi < QT ? qi : 0);
      const int qy = (int)(q / a.nx), qx = (int)(q % a.nx);
      const int fy = qy < a.ny / 2 ? qy : qy - a.ny, fx = qx < a.nx / 2 ? qx : qx - a.nx;
      const int iy = fy + a.nqy / 2, ix = fx + a.nqx / 2;
      const bool inside = iy >= 0 && iy < a.nqy && ix >= 0 && ix < a.nqx;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int kk = l + L * j;
        const int fe = kk < N / 2 ? kk : kk - N;
        const int ie = fe + N / 2;
        double g = inside ? (double)a.gS[((size_t)ie * a.nqy + iy) * a.nqx + ix] : 0.0;
        gp[k][j] = (float)((double)a.K[kk] / Z * (g - D)) * two_over_G;
      }
    }
    for (int p = 0; p < a.Pn; ++p) {
      // zero this tile of the output for every snapshot of position p
      for (int idx = threadIdx.x; idx < a.T * QT; idx += kThreads) {
        const int qi = idx % QT, t = idx / QT;
        a.gexit[((size_t)t * a.Pn + p) * a.nq + q0 + qi] = make_float2(0.f, 0.f);
      }
      for (int g = 0; g < a.G; ++g) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < N * QT; idx += kThreads) {
          const int qi = idx % QT, t = idx / QT;
          tile[qi * CS + lds_pad(t)] = a.exit[((size_t)(g * a.hop + t) * a.Pn + p) * a.nq + q0 + qi];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < QPASS; ++k) {
          const int qi = (k * kWaves + wave) * LINES + line;
          if (qi < QT) {
            float2* lds = tile + qi * CS;
            float2 v[E];
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = lds[lds_pad(l + L * j)];
            FFT<P>::template run<false>(v, tw, lds, l);
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = cscale(v[j], gp[k][j]);
            FFT<P>::template run<true>(v, tw, lds, l);
#pragma unroll
            for (int j = 0; j < E; ++j) lds[lds_pad(l + L * j)] = v[j];
          }
        }
        __syncthreads();
        for (int idx = threadIdx.x; idx < N * QT; idx += kThreads) {
          const int qi = idx % QT, t = idx / QT;
          float2* dst = a.gexit + ((size_t)(g * a.hop + t) * a.Pn + p) * a.nq + q0 + qi;
          *dst = cadd(*dst, tile[qi * CS + lds_pad(t)]);
        }
      }
      __syncthreads();
    }
  }
}

hipError_t launch_spectrum_backward(const SpecBwdArgs& a, hipStream_t st) {
  // D = sum(gS * S) over the output grid
  const size_t nout = (size_t)a.n_e * a.nqy * a.nqx;
  hipLaunchKernelGGL(k_dot_partial, dim3(a.n_part), dim3(kRedThreads), 0, st, a.gS, a.S, nout,
                     a.n_part, a.partial);
  hipLaunchKernelGGL(k_fin_total, dim3(1), dim3(kRedThreads), 0, st, a.partial, a.n_part,
                     a.partial + a.n_part);
  hipError_t e = hipErrorInvalidValue;
  with_time_plan(a.n_e, [&](auto p) {
    using P = decltype(p);
    constexpr int QT = q_tile<P>();
    const int lds = QT * P::LDS_LINE * (int)sizeof(float2);
    hipFuncSetAttribute((const void*)k_spec_bwd<P>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    long tasks = a.nq / QT;
    int grid = (int)(tasks < 8192 ? tasks : 8192);
    hipLaunchKernelGGL((k_spec_bwd<P>), dim3(grid), dim3(kThreads), lds, st, a,
                       (const double*)(a.partial + a.n_part));
    e = hipGetLastError();
  });
  return e;
}

}  // namespace tacaw
