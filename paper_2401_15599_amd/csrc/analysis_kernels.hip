// Analysis outputs of the spectra (the paper's diffraction-pattern and dispersion figures).
//
// Patterns: a per-q sum (over the energy bins of a periodogram, optionally weighted by the Kubo
// factors, or over chosen snapshots and all probe positions of |phi|^2) in float64, a fixed-order
// two-pass total over the full grid, then the normalised, centred and cropped map.  Every sum
// runs in a fixed order (no atomics), so results are deterministic.  Line profiles and dispersion
// cuts read the centred maps and spectra the spectrum kernels produce.
#include "internal.hpp"

namespace tacaw {

constexpr int kAnThreads = 256;

// sp[q] = sum_k P[k][q] and, when K is given, skp[q] = sum_k K[k] P[k][q]; one thread per q
// (consecutive q read consecutive words of each bin's map)
__global__ __launch_bounds__(kAnThreads) void k_energy_sums(const float* P, const float* K,
                                                            int n_e, long nq, double* sp,
                                                            double* skp) {
  for (long q = blockIdx.x * (long)kAnThreads + threadIdx.x; q < nq;
       q += (long)gridDim.x * kAnThreads) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < n_e; ++k) {
      const double p = (double)P[(size_t)k * nq + q];
      a += p;
      if (K) b += (double)K[k] * p;
    }
    sp[q] = a;
    if (skp) skp[q] = b;
  }
}

// s[q] = sum_{j < count} sum_p |exit[t0 + j ts][p][q]|^2
__global__ __launch_bounds__(kAnThreads) void k_snapshot_sums(const float2* exit, int n_pos, long nq,
                                                              int t0, int ts, int count,
                                                              double* s) {
  for (long q = blockIdx.x * (long)kAnThreads + threadIdx.x; q < nq;
       q += (long)gridDim.x * kAnThreads) {
    double a = 0.0;
    for (int j = 0; j < count; ++j) {
      const float2* img = exit + (size_t)(t0 + (long)j * ts) * n_pos * nq;
      for (int p = 0; p < n_pos; ++p) {
        const float2 v = img[(size_t)p * nq + q];
        a += (double)v.x * v.x + (double)v.y * v.y;
      }
    }
    s[q] = a;
  }
}

__device__ double an_block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kAnThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

// block b sums the contiguous range [b per, (b + 1) per) of x in a fixed order
__global__ __launch_bounds__(kAnThreads) void k_range_sums(const double* x, long n, int n_part,
                                                           double* partial) {
  __shared__ double sh[kAnThreads];
  const long per = (n + n_part - 1) / n_part;
  const long b0 = (long)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  double acc = 0.0;
  for (long i = b0 + threadIdx.x; i < b1; i += kAnThreads) acc += x[i];
  const double s = an_block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kAnThreads) void k_range_total(const double* partial, int n_part,
                                                            double* total) {
  __shared__ double sh[kAnThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n_part; i += kAnThreads) acc += partial[i];
  const double s = an_block_sum(acc, sh);
  if (threadIdx.x == 0) *total = s;
}

// centred index i of an output axis of length nout -> storage index of an n-point DFT axis
__device__ __forceinline__ int an_unshift(int i, int nout, int n) {
  const int f = i - nout / 2;
  return f < 0 ? f + n : f;
}

// out[iy][ix] = x[storage q of (iy, ix)] / total
__global__ __launch_bounds__(kAnThreads) void k_norm_crop(const double* x, const double* total,
                                                          int nx, int ny, int nqx, int nqy,
                                                          float* out) {
  const double inv = 1.0 / *total;
  const long nout = (long)nqx * nqy;
  for (long i = blockIdx.x * (long)kAnThreads + threadIdx.x; i < nout;
       i += (long)gridDim.x * kAnThreads) {
    const int ix = (int)(i % nqx), iy = (int)(i / nqx);
    const int qy = an_unshift(iy, nqy, ny), qx = an_unshift(ix, nqx, nx);
    out[i] = (float)(x[(size_t)qy * nx + qx] * inv);
  }
}

// (A - B) / (A + B) along row nqy / 2 (q_y = 0) of two centred maps; 0 where A + B = 0
__global__ __launch_bounds__(kAnThreads) void k_rel_diff_row(const float* A, const float* B,
                                                             int nqx, int nqy, float* out) {
  const size_t row = (size_t)(nqy / 2) * nqx;
  for (int i = blockIdx.x * kAnThreads + threadIdx.x; i < nqx; i += gridDim.x * kAnThreads) {
    const double a = A[row + i], b = B[row + i], s = a + b;
    out[i] = s != 0.0 ? (float)((a - b) / s) : 0.f;
  }
}

// out[e][n] = bilinear sample of S[e] at fractional pixel uv[n] (outside pixels count as zero)
__global__ __launch_bounds__(kAnThreads) void k_path_cut(const float* S, int n_e, int nqx, int nqy,
                                                         const double2* uv, int n_pts, float* out) {
  const long total = (long)n_e * n_pts;
  for (long i = blockIdx.x * (long)kAnThreads + threadIdx.x; i < total;
       i += (long)gridDim.x * kAnThreads) {
    const int n = (int)(i % n_pts), e = (int)(i / n_pts);
    const double u = uv[n].x, v = uv[n].y;
    const double fu = floor(u), fv = floor(v);
    const double fx = u - fu, fy = v - fv;
    const float* img = S + (size_t)e * nqx * nqy;
    auto pix = [&](double y, double x) -> double {
      if (x < 0.0 || y < 0.0 || x >= (double)nqx || y >= (double)nqy) return 0.0;
      return (double)img[(size_t)y * nqx + (size_t)x];
    };
    const double val = (1.0 - fx) * (1.0 - fy) * pix(fv, fu) + fx * (1.0 - fy) * pix(fv, fu + 1.0) +
                       (1.0 - fx) * fy * pix(fv + 1.0, fu) + fx * fy * pix(fv + 1.0, fu + 1.0);
    out[i] = (float)val;
  }
}

// x[i] *= s
__global__ __launch_bounds__(kAnThreads) void k_scale(float* x, long n, float s) {
  for (long i = blockIdx.x * (long)kAnThreads + threadIdx.x; i < n; i += (long)gridDim.x * kAnThreads)
    x[i] *= s;
}

static int an_grid(long n) {
  const long b = (n + kAnThreads - 1) / kAnThreads;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_energy_sums(const float* P, const float* K, int n_e, long nq, double* sp,
                              double* skp, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_sums, dim3(an_grid(nq)), dim3(kAnThreads), 0, st, P, K, n_e, nq, sp, skp);
  return hipGetLastError();
}

hipError_t launch_snapshot_sums(const float2* exit, int n_pos, long nq, int t0, int ts, int count,
                                double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_snapshot_sums, dim3(an_grid(nq)), dim3(kAnThreads), 0, st, exit, n_pos, nq,
                     t0, ts, count, s);
  return hipGetLastError();
}

hipError_t launch_norm_crop(const double* x, long nq, int nx, int ny, int nqx, int nqy,
                            double* partial, int n_part, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_range_sums, dim3(n_part), dim3(kAnThreads), 0, st, x, nq, n_part, partial);
  hipLaunchKernelGGL(k_range_total, dim3(1), dim3(kAnThreads), 0, st, partial, n_part,
                     partial + n_part);
  hipLaunchKernelGGL(k_norm_crop, dim3(an_grid((long)nqx * nqy)), dim3(kAnThreads), 0, st, x,
                     partial + n_part, nx, ny, nqx, nqy, out);
  return hipGetLastError();
}

hipError_t launch_rel_diff_row(const float* A, const float* B, int nqx, int nqy, float* out,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_rel_diff_row, dim3(an_grid(nqx)), dim3(kAnThreads), 0, st, A, B, nqx, nqy, out);
  return hipGetLastError();
}

hipError_t launch_path_cut(const float* S, int n_e, int nqx, int nqy, const double2* uv, int n_pts,
                           float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_path_cut, dim3(an_grid((long)n_e * n_pts)), dim3(kAnThreads), 0, st, S, n_e,
                     nqx, nqy, uv, n_pts, out);
  return hipGetLastError();
}

hipError_t launch_scale(float* x, long n, float s, hipStream_t st) {
  hipLaunchKernelGGL(k_scale, dim3(an_grid(n)), dim3(kAnThreads), 0, st, x, n, s);
  return hipGetLastError();
}

}  // namespace tacaw
