// Host side of the C ABI declared in include/tacaw.h.
//
// Responsibilities: argument validation before any launch, float64 precomputation of the small
// tables the kernels read (propagator factors, exact band-limit and aperture tables, slice
// boundaries, Kubo factors), a content-addressed cache of those tables in device memory, grid-class
// batching of uneven jobs, hipGraph capture of the batched slice loop, the checkpointed adjoint
// schedule, and the FFT schedule autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tacaw.h"
#include "internal.hpp"

namespace tacaw {
hipError_t launch_position_grad_chunks(const PgArgs& a, const int4* chunks, int cap,
                                       const int* count, hipStream_t st);
int spectrum_q_tile(int n_e);
hipError_t launch_chunk_list(const int* offsets, int t0, int n_snap_chunk, int S, int nsp,
                             int4* chunks, int capacity, int* count, hipStream_t st);
void prepare_dynamic_lds(int max_bytes);
}  // namespace tacaw

using namespace tacaw;

// Scratch memory of tacaw_spectrum_finalize_noalloc (partial sums of the normalisation and the
// Kubo table), one copy per GPU, held until the process ends.  In host code this name is not a
// device address: the context keeps the address hipGetSymbolAddress returns for its device.
namespace {
constexpr int kNoallocParts = 512;                     // partial sums of Z
constexpr size_t kNoallocKuboOff = 4352;               // (kNoallocParts + 2) doubles, rounded up
constexpr size_t kScratchBytes = 16384;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// ------------------------------------------------------------------------------------------------
// errors
static thread_local std::string g_err;

namespace {

struct Fail {
  int code;
};

[[noreturn]] void fail(int code, const std::string& msg) {
  g_err = msg;
  throw Fail{code};
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(TACAW_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F> int guarded(F&& f) {
  try {
    f();
    return TACAW_OK;
  } catch (const Fail& x) {
    return x.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return TACAW_E_NOMEM;
  } catch (...) {
    g_err = "unexpected error";
    return TACAW_E_STATE;
  }
}

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }

// ------------------------------------------------------------------------------------------------
// physics (float64, host)
constexpr double kHc = 12398.419843320026;     // eV Angstrom
constexpr double kM0c2 = 510998.95;            // eV
constexpr double kHbar = 0.6582119569;         // eV fs
constexpr double kKb = 8.617333262e-5;         // eV/K
constexpr double kA0 = 0.529177210903;         // Angstrom
constexpr double kE4pe0 = 14.399645478425;     // V Angstrom
constexpr double kPi = 3.14159265358979323846;

double wavelength(double e) { return kHc / std::sqrt(e * (2.0 * kM0c2 + e)); }
double sigma_of(double e) {
  return (2.0 * kPi / (wavelength(e) * e)) * (kM0c2 + e) / (2.0 * kM0c2 + e);
}
int signed_index(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

// largest |n| kept in column m (or -1) for the predicate pred(kx, ky); pred must be monotone in |ky|
template <class Pred> std::vector<int> column_limits(int nx, int ny, double lx, double ly, Pred pred) {
  std::vector<int> out(nx, -1);
  for (int m = 0; m < nx; ++m) {
    const double kx = (double)signed_index(m, nx) / lx;
    int best = -1;
    for (int a = 0; a <= ny / 2; ++a) {
      // both +a and -a (when they exist on the grid) share the same ky^2
      const double ky = (double)a / ly;
      if (pred(kx, ky)) best = a; else break;
    }
    out[m] = best;
  }
  return out;
}

std::vector<int> bandlimit_table(const tacaw_specimen& s) {
  if (s.bandlimit <= 0.0) return std::vector<int>(s.nx, s.ny);   // keep everything
  const double kn = std::min(s.nx / (2.0 * s.lx), s.ny / (2.0 * s.ly));
  const double kmax = s.bandlimit * kn;
  const double kmax2 = kmax * kmax;
  return column_limits(s.nx, s.ny, s.lx, s.ly, [&](double kx, double ky) {
    volatile double k2 = ky * ky + kx * kx;   // no contraction: same rounding as the reference
    return k2 < kmax2;
  });
}

std::vector<int> aperture_table(const tacaw_specimen& s, const tacaw_beam& b) {
  const double lam = wavelength(b.energy_ev);
  const double l2 = lam * lam, a2 = b.alpha_rad * b.alpha_rad;
  return column_limits(s.nx, s.ny, s.lx, s.ly, [&](double kx, double ky) {
    volatile double k2 = ky * ky + kx * kx;
    volatile double lhs = l2 * k2;
    return lhs <= a2;
  });
}

// Largest |signed kx index| of a column that keeps some ky.  The kernels skip the columns m with
// kxb < m < nx - kxb; a table whose kept columns are not exactly the others (never the case for
// a disk) gets nx/2, which skips nothing.
int band_columns(const std::vector<int>& nmax) {
  const int nx = (int)nmax.size();
  int kxb = -1;
  for (int m = 0; m < nx; ++m)
    if (nmax[m] >= 0) kxb = std::max(kxb, m < nx / 2 ? m : nx - m);
  for (int m = 0; m < nx; ++m) {
    const bool inside = m <= kxb || m >= nx - kxb;
    if (inside != (nmax[m] >= 0)) return nx / 2;
  }
  return std::max(kxb, 0);
}

// number of grid points kept by a column-limit table
long count_kept(const std::vector<int>& t, int ny) {
  long c = 0;
  for (int v : t) {
    if (v < 0) continue;
    if (v >= ny / 2) c += ny; else c += 2 * v + 1;
  }
  return c;
}

std::vector<float2> propagator_axis(int n, double len, double lam, const double* dz, int S) {
  std::vector<float2> out((size_t)S * n);
  for (int s = 0; s < S; ++s)
    for (int i = 0; i < n; ++i) {
      const double k = (double)signed_index(i, n) / len;
      const double ph = -kPi * lam * dz[s] * k * k;
      out[(size_t)s * n + i] = make_float2((float)std::cos(ph), (float)std::sin(ph));
    }
  return out;
}

std::vector<double> kubo_dft_order(int n_e, double dt, double temp) {
  std::vector<double> k(n_e);
  const double beta = 1.0 / (kKb * temp);
  for (int i = 0; i < n_e; ++i) {
    const int kp = i < n_e / 2 ? i : i - n_e;
    const double e = 2.0 * kPi * kHbar * kp / (n_e * dt);
    const double x = beta * e;
    k[i] = std::fabs(x) < 1e-4 ? 1.0 + x / 2.0 + x * x / 12.0 : x / (-std::expm1(-x));
  }
  return k;
}

// ------------------------------------------------------------------------------------------------
// device memory helpers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct Cached {
  void* dev = nullptr;
  void* host = nullptr;
  size_t bytes = 0;
};

struct Sched {
  int row_plan = 0, col_plan = 0, C = 0;
  int col_kind = 1;    // 0 staged tile, 1 block kernel
  int pp = 1;          // block kernel: ping-pong LDS exchange regions; 2: and the split-layout
                       // transforms (plans with them, tiles of whole wavefronts of columns)
};

}  // namespace

struct tacaw_ctx {
  int device = 0;
  int max_lds = 65536;
  int n_cu = 256;
  std::map<std::string, DevBuf> ws;
  // content-addressed device copies of small host tables; trimmed only when an API call starts
  // (never while a call holds pointers into it), once it exceeds either limit
  std::unordered_map<std::string, Cached> cache;
  size_t cache_bytes = 0;
  size_t cache_max_entries = 4096, cache_max_bytes = (size_t)256 << 20;
  int depth = 0;                     // nesting of API calls in progress (entry points call others)
  // captured batched slice loops, keyed by the structure of the call (shapes, slice counts, band,
  // class lists, schedule); buffer addresses are read from the graph's own job table, which each
  // replay refreshes, so calls on new tensors replay the same graph.  Least recently used
  // entries beyond max_graphs are destroyed.
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    MsJobDev* jobs_dev = nullptr;    // job table the captured kernels read
    size_t jobs_bytes = 0;
    hipEvent_t done = nullptr;       // recorded after the last replay
    unsigned long long last_use = 0;
  };
  std::unordered_map<std::string, GraphEntry> graphs;
  unsigned long long use_clock = 0;
  size_t max_graphs = 32;
  std::map<int, Sched> sched;
  hipStream_t cap_stream = nullptr;
  hipStream_t up_stream = nullptr;   // table uploads (waited for before the call goes on)
  unsigned char* scratch_dev = nullptr;   // this device's copy of `scratch`
  // side streams (default priority) of the persistent mode's concurrent grid classes
  static constexpr size_t kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};
  std::string desc;
  // opt-in timing instrumentation
  struct Timed {
    std::string kind;
    hipEvent_t a, b;
    double bytes;
  };
  bool timing = false;
  int sf_split16 = 1;
  // batched slice loop: waves per block (bytes of their band-limited columns) and streams
  int64_t block_bytes = (int64_t)192 << 20;
  int block_streams = 2;
  std::vector<Timed> timed;                          // launches whose events are still pending
  std::map<std::string, tacaw_kernel_stats> timed_sums;   // folded launches per kind
  std::vector<hipEvent_t> ev_pool;

  ~tacaw_ctx() {
    (void)hipSetDevice(device);
    (void)hipDeviceSynchronize();
    for (auto& g : graphs) {
      (void)hipGraphExecDestroy(g.second.exec);
      (void)hipFree(g.second.jobs_dev);
      (void)hipEventDestroy(g.second.done);
    }
    for (auto& t : timed) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto& c : cache) {
      if (c.second.dev) (void)hipFree(c.second.dev);
      if (c.second.host) (void)hipHostFree(c.second.host);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (up_stream) (void)hipStreamDestroy(up_stream);
    for (auto& x : side)
      if (x) (void)hipStreamDestroy(x);
    for (auto& e : join_ev)
      if (e) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
  }
};

namespace {

void use_device(tacaw_ctx* c) {
  if (!c) fail(TACAW_E_ARG, "null context");
  hip_check(hipSetDevice(c->device), "hipSetDevice");
}

// grow-only named workspace; growing waits for the device so no queued kernel still uses it
void* workspace(tacaw_ctx* c, const std::string& name, size_t bytes) {
  DevBuf& b = c->ws[name];
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) {
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    hip_check(hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t sz = std::max<size_t>(bytes, 256);
  if (hipMalloc(&b.p, sz) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    fail(TACAW_E_NOMEM, "workspace '" + name + "' of " + std::to_string(sz) + " bytes");
  }
  b.bytes = sz;
  return b.p;
}

hipEvent_t pool_event(tacaw_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hip_check(hipEventCreate(&e), "hipEventCreate");
  return e;
}

// wait for the recorded events, add their launches to the per-kind sums, recycle the events
void fold_timed(tacaw_ctx* c) {
  for (auto& t : c->timed) {
    hip_check(hipEventSynchronize(t.b), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, t.a, t.b), "hipEventElapsedTime");
    tacaw_kernel_stats& k = c->timed_sums[t.kind];
    k.launches += 1;
    k.total_ms += ms;
    k.algo_bytes += t.bytes;
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->timed.clear();
}

// run `launch`; with timing enabled, bracket it with events on its stream and record the
// launch's algorithmic bytes under `kind`
template <class F> void timed_launch(tacaw_ctx* c, hipStream_t st, const char* kind, double bytes,
                                     F&& launch) {
  if (!c->timing) {
    launch();
    return;
  }
  hipEvent_t a = pool_event(c), b = pool_event(c);
  hip_check(hipEventRecord(a, st), "hipEventRecord");
  launch();
  hip_check(hipEventRecord(b, st), "hipEventRecord");
  c->timed.push_back({kind, a, b, bytes});
  // a call can issue tens of thousands of launches: fold the recorded pairs into per-kind sums
  // every few thousand launches, so that at most that many events are alive
  if (c->timed.size() >= 2048) fold_timed(c);
}

void destroy_graph(tacaw_ctx::GraphEntry& g) {
  (void)hipGraphExecDestroy(g.exec);
  (void)hipFree(g.jobs_dev);
  (void)hipEventDestroy(g.done);
  g = tacaw_ctx::GraphEntry{};
}

// drop every cached table and every captured graph (they hold table addresses); waits for the
// device so that no queued kernel still reads them
void evict_tables(tacaw_ctx* c) {
  hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
  for (auto& g : c->graphs) destroy_graph(g.second);
  c->graphs.clear();
  for (auto& e : c->cache) {
    (void)hipFree(e.second.dev);
    (void)hipHostFree(e.second.host);
  }
  c->cache.clear();
  c->cache_bytes = 0;
}

// Every entry point holds one while it runs.  The outermost one trims the table cache before the
// call uploads anything, so a pointer returned by upload() stays valid until the call returns.
struct CallScope {
  tacaw_ctx* c;
  explicit CallScope(tacaw_ctx* c_) : c(c_) {
    if (c->depth == 0 &&
        (c->cache_bytes > c->cache_max_bytes || c->cache.size() > c->cache_max_entries))
      evict_tables(c);
    ++c->depth;
  }
  ~CallScope() { --c->depth; }
  CallScope(const CallScope&) = delete;
  CallScope& operator=(const CallScope&) = delete;
};

// Content-addressed copy of a small host table in device memory (pinned staging kept alive).
// The copy runs on the library's upload stream and is waited for, so the table is resident
// before any stream uses it; entries are never freed during an API call.
void* upload(tacaw_ctx* c, const void* data, size_t bytes, hipStream_t, const char* tag) {
  std::string key(tag);
  key.append((const char*)data, bytes);
  auto it = c->cache.find(key);
  if (it != c->cache.end()) return it->second.dev;
  Cached e;
  e.bytes = bytes;
  hip_check(hipHostMalloc(&e.host, std::max<size_t>(bytes, 16), hipHostMallocDefault), "hipHostMalloc");
  std::memcpy(e.host, data, bytes);
  if (hipMalloc(&e.dev, std::max<size_t>(bytes, 16)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(e.host);
    fail(TACAW_E_NOMEM, std::string("device table '") + tag + "'");
  }
  hipError_t err = hipMemcpyAsync(e.dev, e.host, bytes, hipMemcpyHostToDevice, c->up_stream);
  if (err == hipSuccess) err = hipStreamSynchronize(c->up_stream);
  if (err != hipSuccess) {
    (void)hipFree(e.dev);
    (void)hipHostFree(e.host);
    hip_check(err, "table upload");
  }
  c->cache.emplace(key, e);
  c->cache_bytes += bytes;
  return e.dev;
}

template <class T> T* upload_vec(tacaw_ctx* c, const std::vector<T>& v, hipStream_t st, const char* tag) {
  return (T*)upload(c, v.data(), v.size() * sizeof(T), st, tag);
}

void validate_spec(const tacaw_specimen* s) {
  if (!s) fail(TACAW_E_ARG, "null specimen");
  if (!grid_size_ok(s->nx) || !grid_size_ok(s->ny))
    fail(TACAW_E_SIZE, "grid must be a power of two in [16, 1024], 560 or 1000 per axis, got " +
                           std::to_string(s->nx) + "x" + std::to_string(s->ny));
  if (!(s->lx > 0) || !(s->ly > 0)) fail(TACAW_E_ARG, "cell lengths must be positive");
  if (s->n_slices < 1 || !s->dz) fail(TACAW_E_ARG, "need n_slices >= 1 and dz");
  for (int i = 0; i < s->n_slices; ++i)
    if (!(s->dz[i] > 0)) fail(TACAW_E_ARG, "slice thickness must be positive");
}

void validate_beam(const tacaw_beam* b) {
  if (!b) fail(TACAW_E_ARG, "null beam");
  if (!(b->energy_ev > 0)) fail(TACAW_E_ARG, "beam energy must be positive");
  if (b->kind != TACAW_PLANE_WAVE && b->kind != TACAW_PROBE) fail(TACAW_E_ARG, "unknown beam kind");
  if (b->n_pos < 1) fail(TACAW_E_ARG, "n_pos must be >= 1");
  if (b->kind == TACAW_PLANE_WAVE && b->n_pos != 1) fail(TACAW_E_ARG, "a plane wave has n_pos = 1");
  if (b->kind == TACAW_PROBE && (!b->pos_xy || !(b->alpha_rad > 0)))
    fail(TACAW_E_ARG, "a probe needs positions and alpha > 0");
}

Sched schedule_for(tacaw_ctx* c, int n) {
  auto it = c->sched.find(n);
  if (it != c->sched.end()) return it->second;
  // built-in choices: tacaw_autotune on an MI355X over 1 GiB batches of waves per grid size
  // {n, row plan, column plan, C, kind, pp}
  static const int table[][6] = {{16, 1, 1, 16, 1, 1},  {32, 0, 0, 16, 2, 0},  {64, 0, 0, 64, 1, 0},
                                 {128, 0, 0, 32, 1, 0}, {256, 0, 1, 32, 1, 1}, {512, 0, 0, 16, 1, 2},
                                 {1024, 0, 0, 8, 1, 1}, {560, 2, 3, 16, 1, 0},  {1000, 1, 1, 8, 1, 1}};
  Sched s;
  s.row_plan = 0;
  s.col_plan = 0;
  s.col_kind = 1;
  s.pp = 1;
  s.C = 16;   // 128-byte row segments
  for (const auto& e : table)
    if (e[0] == n) {
      s.row_plan = e[1];
      s.col_plan = e[2];
      s.C = e[3];
      s.col_kind = e[4];
      s.pp = e[5];
    }
  return s;
}

// fit the column tile to the image width (C divides nx), the workgroup size and the LDS budget
// (dynamic tile plus the plan's static root table); a kind the plan cannot run falls back to 0
Sched fit_cols(tacaw_ctx* c, int ny, Sched s, int nx) {
  s.C = std::min(s.C, nx);
  while (s.C > 1 && nx % s.C != 0) s.C /= 2;
  if (!plan_kind_ok(ny, s.col_plan, s.col_kind)) s.col_kind = 0;
  const int budget = c->max_lds - plan_static_lds(ny, s.col_plan);
  if (s.col_kind == 1) {
    const int L = plan_lanes(ny, s.col_plan);
    while (s.C > 1 && s.C * L > col_block_max_threads(ny, s.col_plan)) s.C /= 2;
    if (s.pp && col_block_lds_bytes(ny, s.col_plan, s.C, 1) > budget) s.pp = 0;
    while (s.C > 1 && col_block_lds_bytes(ny, s.col_plan, s.C, s.pp) > budget) s.C /= 2;
    const int cw = col_block_lx_cols(ny, s.col_plan);
    if (s.pp == 2 && (cw == 0 || s.C % cw != 0)) s.pp = 1;
  } else if (s.col_kind == 2) {
    const int C0 = s.C;
    while (s.C > 1 && (col_wave_threads(ny, s.col_plan, s.C) > 1024 ||
                       col_wave_lds_bytes(ny, s.col_plan, s.C) > budget))
      s.C /= 2;
    if (col_wave_threads(ny, s.col_plan, s.C) > 1024 ||
        col_wave_lds_bytes(ny, s.col_plan, s.C) > budget) {
      // no column count both divides nx and gives whole lines per wavefront: staged kind
      s.col_kind = 0;
      s.C = C0;
      while (s.C > 1 && col_lds_bytes(ny, s.col_plan, s.C) > budget) s.C /= 2;
    }
  } else {
    while (s.C > 1 && col_lds_bytes(ny, s.col_plan, s.C) > budget) s.C /= 2;
  }
  return s;
}

// ------------------------------------------------------------------------------------------------
// multislice planning
struct ClassPlan {
  int nx = 0, ny = 0;
  std::vector<int2> groups;        // (job, t) sorted by S descending
  std::vector<int4> waves;         // (job, t, p, S) same order
  std::vector<int> group_S, wave_S;
  std::vector<long> group_wave_prefix;   // waves in groups [0, g)
  std::vector<int4> plane_waves, probe_waves;   // entrance waves: plane waves; probes at t = 0
  std::vector<int4> probe_copies;              // probe waves at t > 0: copies of (job, 0, p)
  int Smax = 0;
  int kxb = 0;                     // widest band of the class's jobs (kx index)
  int kyb = 0;                     // largest |ky index| any column of the class's jobs keeps
  int maxP = 0;                    // most waves per snapshot (probe positions) of the class's jobs
};

int active_prefix(const std::vector<int>& S_sorted_desc, int s) {
  // number of entries with S > s; upper_bound calls comp(value, element) and returns the first
  // element for which it holds, i.e. the first element <= s in the descending list
  return (int)(std::upper_bound(S_sorted_desc.begin(), S_sorted_desc.end(), s,
                                [](int value, int element) { return element <= value; }) -
               S_sorted_desc.begin());
}

struct MsBuild {
  std::vector<MsJobDev> jobs;
  std::vector<ClassPlan> classes;
  MsJobDev* jobs_dev = nullptr;
  bool entrance = false;   // probe jobs have shared entrance buffers (MsJobDev::entr)
};

// Batched forward: every probe job gets an entrance buffer of its P positions in the context's
// workspace; the probe init writes it once and the first x pass of every snapshot reads it (no
// copy of the entrance wave per snapshot).
void attach_entrance(tacaw_ctx* c, MsBuild& b) {
  size_t total = 0;
  for (const MsJobDev& d : b.jobs)
    if (d.nap) total += (size_t)d.P * d.nx * d.ny;
  if (total == 0) return;
  float2* e = (float2*)workspace(c, "entrance", total * sizeof(float2));
  for (MsJobDev& d : b.jobs)
    if (d.nap) {
      d.entr = e;
      e += (size_t)d.P * d.nx * d.ny;
    }
  b.entrance = true;
}

MsBuild build_ms(tacaw_ctx* c, int n_jobs, const tacaw_ms_job* jobs, int ckpt_stride, hipStream_t st,
                 bool adjoint, const tacaw_c64* const* gexit, float* const* gV) {
  if (n_jobs < 1 || !jobs) fail(TACAW_E_ARG, "need at least one job");
  if (ckpt_stride < 0) fail(TACAW_E_ARG, "ckpt_stride must be >= 0");
  MsBuild b;
  b.jobs.resize(n_jobs);
  std::vector<int> kyb_of(n_jobs, 0);
  std::map<std::pair<int, int>, int> class_of;
  for (int j = 0; j < n_jobs; ++j) {
    const tacaw_ms_job& J = jobs[j];
    validate_spec(J.spec);
    validate_beam(J.beam);
    if (J.n_snap < 1) fail(TACAW_E_ARG, "job " + std::to_string(j) + ": n_snap must be >= 1");
    if (!J.V) fail(TACAW_E_ARG, "job " + std::to_string(j) + ": null V");
    if (!adjoint && !J.exit) fail(TACAW_E_ARG, "job " + std::to_string(j) + ": null exit");
    if (ckpt_stride > 0 && !J.ckpt) fail(TACAW_E_ARG, "job " + std::to_string(j) + ": null ckpt");
    if (adjoint && (!gexit || !gexit[j] || !gV || !gV[j]))
      fail(TACAW_E_ARG, "job " + std::to_string(j) + ": null gradient buffer");
    const tacaw_specimen& S = *J.spec;
    const tacaw_beam& B = *J.beam;
    const double lam = wavelength(B.energy_ev);
    MsJobDev d{};
    d.V = J.V;
    d.W = (float2*)J.exit;
    d.ckpt = (float2*)J.ckpt;
    d.px = upload_vec(c, propagator_axis(S.nx, S.lx, lam, S.dz, S.n_slices), st, "px");
    d.py = upload_vec(c, propagator_axis(S.ny, S.ly, lam, S.dz, S.n_slices), st, "py");
    {
      const std::vector<int> bl = bandlimit_table(S);
      d.nmax = upload_vec(c, bl, st, "bl");
      d.kxb = band_columns(bl);
      kyb_of[j] = *std::max_element(bl.begin(), bl.end());
    }
    long n_ap = 1;
    if (B.kind == TACAW_PROBE) {
      std::vector<int> ap = aperture_table(S, B);
      n_ap = count_kept(ap, S.ny);
      if (n_ap < 1) fail(TACAW_E_ARG, "probe aperture holds no grid point");
      d.nap = upload_vec(c, ap, st, "ap");
      std::vector<double> pxy(B.pos_xy, B.pos_xy + 2 * B.n_pos);
      d.pxy = upload_vec(c, pxy, st, "pxy");
    }
    d.T = J.n_snap;
    d.P = B.n_pos;
    d.S = S.n_slices;
    d.nx = S.nx;
    d.ny = S.ny;
    d.ck_stride = ckpt_stride > 0 ? ckpt_stride : 1;
    d.n_ck = ckpt_stride > 0 ? (S.n_slices + ckpt_stride - 1) / ckpt_stride : 0;
    d.stash_k = ckpt_stride > 0 ? ckpt_stride : 1;
    d.sigma = (float)sigma_of(B.energy_ev);
    const double npix = (double)S.nx * S.ny;
    d.scale_mid = (float)(1.0 / npix);
    d.scale_last = (float)(1.0 / std::sqrt(npix));
    d.scale_probe = (float)(1.0 / (std::sqrt(npix) * std::sqrt((double)n_ap)));
    d.lx = S.lx;
    d.ly = S.ly;
    d.lambda = lam;
    d.defocus = B.defocus_a;
    d.cs = B.cs_a;
    if (adjoint) {
      d.gexit = (const float2*)gexit[j];
      d.gV = gV[j];
    }
    b.jobs[j] = d;
    auto key = std::make_pair(S.nx, S.ny);
    if (!class_of.count(key)) {
      class_of[key] = (int)b.classes.size();
      b.classes.emplace_back();
      b.classes.back().nx = S.nx;
      b.classes.back().ny = S.ny;
    }
  }
  for (int j = 0; j < n_jobs; ++j) {
    ClassPlan& cp = b.classes[class_of[{b.jobs[j].nx, b.jobs[j].ny}]];
    for (int t = 0; t < b.jobs[j].T; ++t) cp.groups.push_back(make_int2(j, t));
    cp.kxb = std::max(cp.kxb, b.jobs[j].kxb);
    cp.kyb = std::max(cp.kyb, kyb_of[j]);
    cp.maxP = std::max(cp.maxP, b.jobs[j].P);
  }
  for (auto& cp : b.classes) {
    std::stable_sort(cp.groups.begin(), cp.groups.end(), [&](int2 a, int2 x) {
      return b.jobs[a.x].S > b.jobs[x.x].S;
    });
    cp.group_wave_prefix.push_back(0);
    for (auto g : cp.groups) {
      const MsJobDev& d = b.jobs[g.x];
      cp.group_S.push_back(d.S);
      cp.group_wave_prefix.push_back(cp.group_wave_prefix.back() + d.P);
      for (int p = 0; p < d.P; ++p) {
        int4 w = make_int4(g.x, g.y, p, d.S);
        cp.waves.push_back(w);
        cp.wave_S.push_back(d.S);
        if (jobs[g.x].beam->kind == TACAW_PROBE) (g.y == 0 ? cp.probe_waves : cp.probe_copies).push_back(w);
        else cp.plane_waves.push_back(w);
      }
    }
    cp.Smax = cp.group_S.empty() ? 0 : cp.group_S.front();
  }
  return b;
}

struct Launcher {
  tacaw_ctx* c;
  hipStream_t st;
  // waves: number of waves the launch covers (for the byte model only)
  // kxb: the class's widest band (algorithmic bytes count the band-limited columns only)
  void row(int n, const Sched& sc, bool adj, RowArgs a, long waves, int kxb) {
    if (a.n_groups <= 0) return;
    const int lines = row_lines_per_wave(n, sc.row_plan);
    const long tasks = (long)a.n_groups * ((a.ny + lines - 1) / lines * lines);
    long g = (tasks + (long)kWaves * lines - 1) / ((long)kWaves * lines);
    g = std::min<long>(g, (long)c->n_cu * 8);
    // bytes per image element: wave in 8, out 8, checkpoint 8, stash 8; per V row 4 (+4 for dL/dV)
    const double img = (double)n * a.ny;
    const double band = (double)std::min(n, 2 * kxb + 1) / n;
    double per_wave = 8.0 * (a.band_in ? band : 1.0) +
                      (a.write_out ? 8.0 * (a.band_out ? band : 1.0) : 0.0) +
                      (a.store_ckpt ? 8.0 : 0.0) + (a.stash_slot >= 0 ? 8.0 : 0.0);
    double bytes = img * (per_wave * waves + (adj ? 8.0 : 4.0) * a.n_groups);
    timed_launch(c, st, adj ? "row_adj" : "row", bytes, [&] {
      hip_check(launch_row(n, sc.row_plan, adj, a, (int)std::max<long>(g, 1), st), "row kernel");
    });
  }
  // all_tiles: the output is read by the caller (exit waves), so every column is written
  void col(int ny, const Sched& sc, bool f, bool i, ColArgs a, int kxb, bool all_tiles) {
    if (a.n_waves <= 0) return;
    a.C = sc.C;
    a.pingpong = sc.pp;
    const int tpi = a.nx / a.C;
    a.tiles_lo = a.tiles_hi = 0;
    if (!all_tiles && kxb < a.nx / 2) {
      const int lo = std::min(tpi, kxb / a.C + 1);
      const int hi = tpi - (a.nx - kxb) / a.C;
      if (lo + hi < tpi) {
        a.tiles_lo = lo;
        a.tiles_hi = hi;
      }
    }
    const int tiles = (a.tiles_lo + a.tiles_hi) > 0 ? a.tiles_lo + a.tiles_hi : tpi;
    const long tasks = (long)a.n_waves * tiles;
    // block kernel: one or two resident workgroups per CU (LDS bound); staged: up to 8
    const long per_cu =
        sc.col_kind == 1 ? std::max(1, c->max_lds / std::max(1, col_block_lds_bytes(ny, sc.col_plan, sc.C, sc.pp)))
        : sc.col_kind == 2 ? std::max(1, c->max_lds / std::max(1, col_wave_lds_bytes(ny, sc.col_plan, sc.C)))
                           : 8;
    long g = std::min<long>(tasks, (long)c->n_cu * per_cu);
    // columns outside the band are never read; they are written only when all_tiles is set
    const double nband = std::min(a.nx, 2 * kxb + 1);
    const double bytes = 8.0 * (nband + (all_tiles ? a.nx : nband)) * ny * a.n_waves;
    timed_launch(c, st, a.conj_prop ? "col_adj" : "col", bytes, [&] {
      hip_check(launch_col(ny, sc.col_plan, sc.col_kind, f, i, a, (int)std::max<long>(g, 1), st),
                "column kernel");
    });
  }
};

void run_forward(tacaw_ctx* c, const MsBuild& b, int ckpt_stride, int mode, hipStream_t st_main) {
  // persistent mode: the grid classes run concurrently on the context's side streams, forked from
  // and joined back into the caller's stream (inside a capture they become parallel branches)
  const bool fork = mode == TACAW_MODE_PERSISTENT && b.classes.size() > 1;
  const int n_side = fork ? (int)std::min<size_t>(b.classes.size(), tacaw_ctx::kSide) : 0;
  if (fork) {
    hip_check(hipEventRecord(c->fork_ev, st_main), "hipEventRecord");
    for (int i = 0; i < n_side; ++i)
      hip_check(hipStreamWaitEvent(c->side[i], c->fork_ev, 0), "hipStreamWaitEvent");
  }
  for (size_t ci = 0; ci < b.classes.size(); ++ci) {
    const ClassPlan& cp = b.classes[ci];
    const hipStream_t st = fork ? c->side[ci % n_side] : st_main;
    const Sched rs = schedule_for(c, cp.nx);
    const Sched cs = fit_cols(c, cp.ny, schedule_for(c, cp.ny), cp.nx);
    // the staged init kernels use the same column count (their LDS tile is the smaller one)
    // entr: probe entrance waves go to (and the first x pass reads them from) the jobs' shared
    // entrance buffers instead of a copy per snapshot
    auto do_range = [&](hipStream_t sst, const int2* groups, int ng, const int4* waves, const std::vector<int>& gS,
                        const std::vector<int>& wS, const int4* plane, int nplane,
                        const int4* probe, int nprobe, const int4* copies, int ncopy, bool entr) {
      Launcher L{c, sst};
      ColArgs ia{};
      ia.jobs = b.jobs_dev;
      ia.out_buf = BUF_W;
      ia.C = cs.C;
      ia.nx = cp.nx;
      if (nplane > 0) {
        ia.waves = plane;
        ia.n_waves = nplane;
        long g = std::min<long>(nplane, (long)c->n_cu * 8);
        hip_check(launch_plane_init(ia, (int)g, sst), "plane-wave init");
      }
      if (nprobe > 0) {
        ia.waves = probe;
        ia.n_waves = nprobe;
        ia.out_buf = entr ? BUF_ENTR : BUF_W;
        long g = std::min<long>((long)nprobe * (cp.nx / cs.C), (long)c->n_cu * 8);
        hip_check(launch_probe_init(cp.ny, cs.col_plan, ia, (int)g, sst), "probe init");
        ia.out_buf = BUF_W;
      }
      if (ncopy > 0 && !entr) {
        ia.waves = copies;
        ia.n_waves = ncopy;
        const long spans = ((long)cp.nx * cp.ny / 2 + 1023) / 1024;
        long g = std::min<long>((long)ncopy * spans, (long)c->n_cu * 16);
        hip_check(launch_wave_copy(ia, (int)g, sst), "probe copies");
      }
      const int Smax = gS.empty() ? 0 : gS.front();
      for (int s = 0; s < Smax; ++s) {
        RowArgs ra{};
        ra.jobs = b.jobs_dev;
        ra.groups = groups;
        ra.n_groups = active_prefix(gS, s);
        ra.s = s;
        ra.in_buf = (entr && s == 0) ? BUF_ENTR : BUF_W;
        ra.out_buf = BUF_W;
        ra.store_ckpt = (ckpt_stride > 0 && s % ckpt_stride == 0) ? 1 : 0;
        ra.stash_slot = -1;
        ra.write_out = 1;
        ra.ny = cp.ny;
        ra.band_in = s > 0 ? 1 : 0;   // the initial wave is not band-limited
        ra.band_out = 1;
        ra.prune = (s > 0 && plan_prunable(cp.nx, rs.row_plan, cp.kxb)) ? 1 : 0;
        ra.single_pos = cp.maxP == 1 ? 1 : 0;
        L.row(cp.nx, rs, false, ra, active_prefix(wS, s), cp.kxb);
        const int n_mid = active_prefix(wS, s + 1), n_all = active_prefix(wS, s);
        ColArgs ca{};
        ca.jobs = b.jobs_dev;
        ca.s = s;
        ca.in_buf = BUF_W;
        ca.out_buf = BUF_W;
        ca.conj_prop = 0;
        ca.prune = plan_prunable(cp.ny, cs.col_plan, cp.kyb) ? 1 : 0;
        ca.C = cs.C;
        ca.nx = cp.nx;
        if (n_mid > 0) {
          ca.waves = waves;
          ca.n_waves = n_mid;
          ca.scale = (float)(1.0 / ((double)cp.nx * cp.ny));
          L.col(cp.ny, cs, true, true, ca, cp.kxb, false);
        }
        if (n_all > n_mid) {
          ca.waves = waves + n_mid;
          ca.n_waves = n_all - n_mid;
          ca.scale = (float)(1.0 / std::sqrt((double)cp.nx * cp.ny));
          L.col(cp.ny, cs, true, false, ca, cp.kxb, true);   // exit waves
        }
      }
    };
    // device copies of the class lists
    int2* groups_dev = upload_vec(c, cp.groups, st, "groups");
    int4* waves_dev = upload_vec(c, cp.waves, st, "waves");
    int4* plane_dev = cp.plane_waves.empty() ? nullptr : upload_vec(c, cp.plane_waves, st, "pw");
    int4* probe_dev = cp.probe_waves.empty() ? nullptr : upload_vec(c, cp.probe_waves, st, "pr");
    int4* copy_dev = cp.probe_copies.empty() ? nullptr : upload_vec(c, cp.probe_copies, st, "pc");
    const int ncopy = (int)cp.probe_copies.size();
    if (mode == TACAW_MODE_PERSISTENT && resident_ok(cp.nx, cp.ny)) {
      // entrance waves by the init kernels, then one launch for every wave of the class: each
      // workgroup keeps a wave on its CU through all of that wave's slices and then takes the next
      {
        ColArgs ia{};
        ia.jobs = b.jobs_dev;
        ia.out_buf = BUF_W;
        ia.C = cs.C;
        ia.nx = cp.nx;
        if (!cp.plane_waves.empty()) {
          ia.waves = plane_dev;
          ia.n_waves = (int)cp.plane_waves.size();
          long g = std::min<long>(ia.n_waves, (long)c->n_cu * 8);
          hip_check(launch_plane_init(ia, (int)g, st), "plane-wave init");
        }
        if (!cp.probe_waves.empty()) {
          ia.waves = probe_dev;
          ia.n_waves = (int)cp.probe_waves.size();
          long g = std::min<long>((long)ia.n_waves * (cp.nx / cs.C), (long)c->n_cu * 8);
          hip_check(launch_probe_init(cp.ny, cs.col_plan, ia, (int)g, st), "probe init");
        }
        if (ncopy > 0) {
          ia.waves = copy_dev;
          ia.n_waves = ncopy;
          const long spans = ((long)cp.nx * cp.ny / 2 + 1023) / 1024;
          long g = std::min<long>((long)ncopy * spans, (long)c->n_cu * 16);
          hip_check(launch_wave_copy(ia, (int)g, st), "probe copies");
        }
      }
      ColArgs ra{};
      ra.jobs = b.jobs_dev;
      ra.waves = waves_dev;
      ra.n_waves = (int)cp.waves.size();
      ra.scale = (float)(1.0 / ((double)cp.nx * cp.ny));
      ra.nx = cp.nx;
      const long g = std::min<long>(ra.n_waves, (long)c->n_cu * resident_workgroups_per_cu(cp.nx, c->max_lds));
      // HBM bytes: V of every slice, the exit wave, the checkpoints
      double bytes = 0.0;
      const double img = (double)cp.nx * cp.ny;
      for (const int4& w : cp.waves) {
        const MsJobDev& d = b.jobs[w.x];
        bytes += img * (4.0 * d.S + 16.0 + 8.0 * d.n_ck);   // + entrance wave read
      }
      timed_launch(c, st, "resident", bytes, [&] {
        hip_check(launch_resident(cp.nx, ra, (int)std::max<long>(g, 1), st), "resident slice loop");
      });
    } else if (mode == TACAW_MODE_PLAIN) {
      // one snapshot (all its probe positions) per launch sequence
      size_t wi = 0;
      for (size_t gi = 0; gi < cp.groups.size(); ++gi) {
        const MsJobDev& d = b.jobs[cp.groups[gi].x];
        std::vector<int> gS(1, d.S), wS(d.P, d.S);
        const bool probe = d.nap != nullptr;
        // the group's waves are contiguous in the class wave list and in the init lists
        const int4* w = waves_dev + wi;
        do_range(st, groups_dev + gi, 1, w, gS, wS, probe ? nullptr : w, probe ? 0 : d.P,
                 probe ? w : nullptr, probe ? d.P : 0, nullptr, 0, false);
        wi += d.P;
      }
    } else {
      const double block = (double)c->block_bytes;
      const double wave_bytes = 8.0 * cp.ny * std::min(cp.nx, 2 * cp.kxb + 1);
      const int ng = (int)cp.groups.size();
      if (block <= 0.0 || ng < 2) {
        do_range(st, groups_dev, ng, waves_dev, cp.group_S, cp.wave_S, plane_dev,
                 (int)cp.plane_waves.size(), probe_dev, (int)cp.probe_waves.size(), copy_dev, ncopy,
                 b.entrance);
      } else {
        // entrance waves of the whole class first, then blocks of consecutive snapshots whose
        // waves fit the memory-side cache run all their slices before the next block starts;
        // successive blocks alternate between two streams (forked from and joined back into the
        // caller's), so that one block's launches fill the other's ramp-up and tail
        do_range(st, groups_dev, 0, waves_dev, {}, {}, plane_dev, (int)cp.plane_waves.size(), probe_dev,
                 (int)cp.probe_waves.size(), copy_dev, ncopy, b.entrance);
        const int chains = fork ? 1 : c->block_streams;
        if (chains > 1) {
          hip_check(hipEventRecord(c->fork_ev, st), "hipEventRecord");
          for (int i = 0; i < chains; ++i)
            hip_check(hipStreamWaitEvent(c->side[i], c->fork_ev, 0), "hipStreamWaitEvent");
        }
        int g0 = 0, k = 0;
        while (g0 < ng) {
          int g1 = g0;
          double bytes = 0.0;
          do {
            bytes += wave_bytes * b.jobs[cp.groups[g1].x].P;
            ++g1;
          } while (g1 < ng && bytes + wave_bytes * b.jobs[cp.groups[g1].x].P <= block);
          const long w0 = cp.group_wave_prefix[g0], w1 = cp.group_wave_prefix[g1];
          const std::vector<int> gS(cp.group_S.begin() + g0, cp.group_S.begin() + g1);
          const std::vector<int> wS(cp.wave_S.begin() + w0, cp.wave_S.begin() + w1);
          do_range(chains > 1 ? c->side[k % chains] : st, groups_dev + g0, g1 - g0, waves_dev + w0, gS,
                   wS, nullptr, 0, nullptr, 0, nullptr, 0, b.entrance);
          g0 = g1;
          ++k;
        }
        if (chains > 1)
          for (int i = 0; i < chains; ++i) {
            hip_check(hipEventRecord(c->join_ev[i], c->side[i]), "hipEventRecord");
            hip_check(hipStreamWaitEvent(st, c->join_ev[i], 0), "hipStreamWaitEvent");
          }
      }
    }
  }
  if (fork) {
    for (int i = 0; i < n_side; ++i) {
      hip_check(hipEventRecord(c->join_ev[i], c->side[i]), "hipEventRecord");
      hip_check(hipStreamWaitEvent(st_main, c->join_ev[i], 0), "hipStreamWaitEvent");
    }
  }
}

// Key of a captured batched slice loop: everything that shapes its launches (per job: grid,
// snapshots, positions, slices, band columns, checkpoint layout, illumination kind; per class:
// the S-sorted lists, band extents and FFT schedule), but no buffer or table address: those
// reach the kernels through the job table, which is copied into the graph's own table before
// every replay.
std::string graph_key(const MsBuild& b, int ckpt_stride, int mode, tacaw_ctx* c) {
  std::ostringstream k;
  k << ckpt_stride << '|' << mode << '|' << c->block_bytes << '|' << c->block_streams;
  for (const MsJobDev& d : b.jobs)
    k << "|j" << d.T << ',' << d.P << ',' << d.S << ',' << d.nx << ',' << d.ny << ',' << d.kxb << ','
      << d.ck_stride << ',' << d.n_ck << ',' << (d.nap != nullptr);
  std::string out = k.str();
  for (auto& cp : b.classes) {
    Sched a = schedule_for(c, cp.nx), s2 = fit_cols(c, cp.ny, schedule_for(c, cp.ny), cp.nx);
    out += "|c" + std::to_string(cp.nx) + "," + std::to_string(cp.ny) + "," +
           std::to_string(cp.kxb) + "," + std::to_string(cp.kyb) + "," +
           std::to_string(a.row_plan) + "," + std::to_string(s2.col_plan) + "," +
           std::to_string(s2.C) + "," + std::to_string(s2.col_kind) + "," + std::to_string(s2.pp);
    out.append((const char*)cp.groups.data(), cp.groups.size() * sizeof(int2));
  }
  return out;
}

}  // namespace

// =================================================================================================
extern "C" {

int tacaw_version(void) { return 100; }

const char* tacaw_last_error(void) { return g_err.c_str(); }

int tacaw_create(int hip_device, tacaw_ctx** out) {
  return guarded([&] {
    if (!out) fail(TACAW_E_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= n) fail(TACAW_E_ARG, "no such HIP device");
    hip_check(hipSetDevice(hip_device), "hipSetDevice");
    auto c = std::make_unique<tacaw_ctx>();
    c->device = hip_device;
    hipDeviceProp_t prop;
    hip_check(hipGetDeviceProperties(&prop, hip_device), "hipGetDeviceProperties");
    c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) == hipSuccess &&
        lds > 0)
      c->max_lds = lds;
    hip_check(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipStreamCreateWithFlags(&c->up_stream, hipStreamNonBlocking), "hipStreamCreate");
    for (auto& x : c->side) hip_check(hipStreamCreateWithFlags(&x, hipStreamNonBlocking), "hipStreamCreate");
    hip_check(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming), "hipEventCreate");
    for (auto& e : c->join_ev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    void* sp = nullptr;
    hip_check(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    c->scratch_dev = (unsigned char*)sp;
    prepare_dynamic_lds(c->max_lds);
    const char* tc = std::getenv("TACAW_TUNE_CACHE");
    if (tc && *tc) tacaw_load_tuning(c.get(), tc);
    *out = c.release();
  });
}

void tacaw_destroy(tacaw_ctx* ctx) { delete ctx; }

double tacaw_wavelength(double e) { return wavelength(e); }
double tacaw_interaction_parameter(double e) { return sigma_of(e); }

int tacaw_energy_axis(int32_t n_e, double dt_fs, double* e_ev) {
  return guarded([&] {
    if (n_e < 1 || !(dt_fs > 0) || !e_ev) fail(TACAW_E_ARG, "bad energy-axis arguments");
    for (int j = 0; j < n_e; ++j) e_ev[j] = 2.0 * kPi * kHbar * (j - n_e / 2) / (n_e * dt_fs);
  });
}

// ------------------------------------------------------------------------------------------------
static std::vector<double> slice_bounds(const tacaw_specimen& s) {
  std::vector<double> b(s.n_slices + 1);
  b[0] = s.z0;
  for (int i = 0; i < s.n_slices; ++i) {
    volatile double nb = b[i] + s.dz[i];
    b[i + 1] = nb;
  }
  return b;
}

static void validate_atoms(const tacaw_specimen* spec, int n_snap, int n_atoms, const float* xyz,
                           const int* species, int n_species) {
  validate_spec(spec);
  if (n_snap < 1 || n_atoms < 1) fail(TACAW_E_ARG, "need n_snap >= 1 and n_atoms >= 1");
  if (!xyz || !species) fail(TACAW_E_ARG, "null positions or species");
  if (n_species < 1 || n_species > kMaxSpecies) fail(TACAW_E_SIZE, "n_species must be in [1, 8]");
  if ((long)spec->n_slices * n_species > 16384) fail(TACAW_E_SIZE, "n_slices * n_species > 16384");
}

int tacaw_bin_atoms(tacaw_ctx* ctx, const tacaw_specimen* spec, int32_t n_snap, int32_t n_atoms,
                    const float* xyz, const int32_t* species, int32_t n_species, int32_t* offsets,
                    int32_t* order, int32_t* n_outside, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_atoms(spec, n_snap, n_atoms, xyz, species, n_species);
    if (!offsets || !order) fail(TACAW_E_ARG, "null outputs");
    hipStream_t st = (hipStream_t)stream;
    double* bnd = upload_vec(ctx, slice_bounds(*spec), st, "bounds");
    hip_check(launch_bin_atoms(xyz, species, n_snap, n_atoms, n_species, bnd, spec->n_slices,
                               offsets, order, n_outside, st),
              "bin kernel");
  });
}

// pref M(k) f_Z(|k|) w(k) on the rows the position gradient visits (ky >= 0 with weight 2 for
// ky > 0 in half-plane mode), per species; *bound = max |v| max(1, |ky|) (the H scale of the kernel)
static std::vector<float> pos_grad_table(const tacaw_specimen& s, const double* ff, int nsp,
                                         const std::vector<int>& nmax, bool herm, double pref,
                                         double* bound) {
  const int nx = s.nx, ny = s.ny, ny_h = herm ? ny / 2 : ny;
  std::vector<float> t((size_t)nsp * ny_h * nx, 0.f);
  double b = 0.0;
  for (int z = 0; z < nsp; ++z) {
    const double* f = ff + 12 * z;
    for (int n = 0; n < ny_h; ++n) {
      const int ns = n < ny / 2 ? n : n - ny;
      const double ky = ns / s.ly;
      for (int m = 0; m < nx; ++m) {
        if (std::abs(ns) > nmax[m]) continue;
        const int ms = m < nx / 2 ? m : m - nx;
        const double kx = ms / s.lx, q2 = kx * kx + ky * ky;
        const double fz = f[0] / (q2 + f[1]) + f[2] / (q2 + f[3]) + f[4] / (q2 + f[5]) +
                          f[6] * std::exp(-f[7] * q2) + f[8] * std::exp(-f[9] * q2) +
                          f[10] * std::exp(-f[11] * q2);
        const double v = ((herm && n > 0) ? 2.0 : 1.0) * pref * fz;
        t[((size_t)z * ny_h + n) * nx + m] = (float)v;
        b = std::max(b, std::abs(v) * std::max(1.0, std::abs(ky)));
      }
    }
  }
  *bound = b;
  return t;
}

static std::vector<float> ff_f32(const double* ff, int nsp) {
  std::vector<float> f(12 * nsp);
  for (int i = 0; i < 12 * nsp; ++i) f[i] = (float)ff[i];
  return f;
}

int tacaw_build_potentials(tacaw_ctx* ctx, const tacaw_specimen* spec, int32_t n_snap,
                           int32_t n_atoms, const float* xyz, const int32_t* species,
                           int32_t n_species, const double* ff, float* V, int32_t* n_outside,
                           void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_atoms(spec, n_snap, n_atoms, xyz, species, n_species);
    if (!ff || !V) fail(TACAW_E_ARG, "null form factors or output");
    for (int i = 0; i < 12 * n_species; ++i)
      if (!std::isfinite(ff[i])) fail(TACAW_E_ARG, "form-factor coefficients must be finite");
    hipStream_t st = (hipStream_t)stream;
    const int S = spec->n_slices, K = S * n_species;
    int* offs = (int*)workspace(ctx, "offsets", (size_t)n_snap * (K + 1) * sizeof(int));
    int* ord = (int*)workspace(ctx, "order", (size_t)n_snap * n_atoms * sizeof(int));
    double* bnd = upload_vec(ctx, slice_bounds(*spec), st, "bounds");
    hip_check(launch_bin_atoms(xyz, species, n_snap, n_atoms, n_species, bnd, S, offs, ord,
                               n_outside, st),
              "bin kernel");
    float* ffd = upload_vec(ctx, ff_f32(ff, n_species), st, "ff");
    const std::vector<int> bl = bandlimit_table(*spec);
    int* nmax = upload_vec(ctx, bl, st, "bl");
    // the inverse FFT skips the columns and rows the band limit leaves zero
    int kxb = band_columns(bl), kyb = *std::max_element(bl.begin(), bl.end());
    if (kxb >= spec->nx / 2) kxb = -1;
    if (kyb >= spec->ny / 2) kyb = -1;
    // bytes per pixel of the inverse FFT: column pass reads the kept rows of the kept columns and
    // writes the kept columns, row pass reads those and writes every real pixel; with two maps per
    // transform (A + iB) the column writes and row reads are shared by the pair
    const double fc = kxb < 0 ? 1.0 : (2.0 * kxb + 1.0) / spec->nx;
    const double fr = kyb < 0 ? 1.0 : (2.0 * kyb + 1.0) / spec->ny;
    const bool paired = spec->bandlimit > 0.0 && spec->bandlimit < 1.0;
    const double ifft_bytes = 8.0 * fc * fr + (paired ? 8.0 : 16.0) * fc + 4.0;
    const size_t img = (size_t)spec->nx * spec->ny;
    // bytes of complex k-space maps per pass: enough maps per launch that the structure factor's
    // live tiles fill the GPU many times over (a 1024^2 snapshot of 100 slices holds 800 MB)
    const size_t budget = (size_t)4 << 30;
    int snaps_per = (int)std::max<size_t>(1, budget / (img * 8 * S));
    snaps_per = std::min(snaps_per, (int)n_snap);
    float2* vk = (float2*)workspace(ctx, "vk", (size_t)snaps_per * S * img * sizeof(float2));
    void* arec = workspace(ctx, "atom_phase", (size_t)snaps_per * n_atoms * 24);
    // quarter-plane tiles (64 x 64 over 0 <= kx < nx/2, 0 <= ky < ny/2) with a kept k first
    std::vector<int> order, dead;
    {
      const int tx_n = (spec->nx / 2 + 63) / 64, ty_n = (spec->ny / 2 + 63) / 64;
      for (int ty = 0; ty < ty_n; ++ty)
        for (int tx = 0; tx < tx_n; ++tx) {
          bool live = false;
          for (int m = 64 * tx; m < std::min(64 * tx + 64, spec->nx / 2); ++m) live |= bl[m] >= 64 * ty;
          (live ? order : dead).push_back(ty * tx_n + tx);
        }
    }
    const int n_live = (int)order.size();
    order.insert(order.end(), dead.begin(), dead.end());
    const int* tile_order = upload_vec(ctx, order, st, "sf_tiles");
    for (int t0 = 0; t0 < n_snap; t0 += snaps_per) {
      const int nt = std::min(snaps_per, n_snap - t0);
      SfArgs a{};
      a.arec = arec;
      a.xyz = xyz;
      a.order = ord;
      a.offsets = offs;
      a.ff = ffd;
      a.vk = vk;
      a.t0 = t0;
      a.s_count = S;
      a.n_atoms = n_atoms;
      a.n_species = n_species;
      a.nx = spec->nx;
      a.ny = spec->ny;
      a.lx = spec->lx;
      a.ly = spec->ly;
      a.pref = (float)(2.0 * kPi * kA0 * kE4pe0 / (spec->lx * spec->ly));
      a.nmax = nmax;
      a.n_maps = nt * S;
      // V(-k) = conj V(k) holds exactly when the band limit removes the Nyquist row and column
      a.hermitian = (spec->bandlimit > 0.0 && spec->bandlimit < 1.0 && spec->ny >= 128) ? 1 : 0;
      a.split16 = ctx->sf_split16;
      a.tile_order = tile_order;
      a.n_live = n_live;
      timed_launch(ctx, st, "sf", 8.0 * img * nt * S, [&] {
        hip_check(launch_structure_factor(a, st), "structure-factor kernel");
      });
      timed_launch(ctx, st, "pot_ifft", ifft_bytes * img * nt * S, [&] {
        // two maps per complex transform when the band limit removes every Nyquist term
        const int pair = (spec->bandlimit > 0.0 && spec->bandlimit < 1.0) ? 1 : 0;
        hip_check(launch_ifft2_real(spec->nx, spec->ny, vk, V + (size_t)t0 * S * img, nt * S, kxb,
                                    kyb, pair, offs, t0, S, n_species, st),
                  "potential inverse FFT");
      });
    }
  });
}

int tacaw_build_potentials_backward(tacaw_ctx* ctx, const tacaw_specimen* spec, int32_t n_snap,
                                    int32_t n_atoms, const float* xyz, const int32_t* species,
                                    int32_t n_species, const double* ff, const float* grad_V,
                                    float* grad_xy, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_atoms(spec, n_snap, n_atoms, xyz, species, n_species);
    if (!ff || !grad_V || !grad_xy) fail(TACAW_E_ARG, "null form factors or gradient buffers");
    hipStream_t st = (hipStream_t)stream;
    const int S = spec->n_slices, K = S * n_species;
    int* offs = (int*)workspace(ctx, "offsets", (size_t)n_snap * (K + 1) * sizeof(int));
    int* ord = (int*)workspace(ctx, "order", (size_t)n_snap * n_atoms * sizeof(int));
    double* bnd = upload_vec(ctx, slice_bounds(*spec), st, "bounds");
    hip_check(launch_bin_atoms(xyz, species, n_snap, n_atoms, n_species, bnd, S, offs, ord,
                               nullptr, st),
              "bin kernel");
    hip_check(launch_zero(grad_xy, (size_t)n_snap * n_atoms * 2 * sizeof(float), st), "zero");
    float* ffd = upload_vec(ctx, ff_f32(ff, n_species), st, "ff");
    int* nmax = upload_vec(ctx, bandlimit_table(*spec), st, "bl");
    const size_t img = (size_t)spec->nx * spec->ny;
    const size_t budget = (size_t)4 << 30;
    int snaps_per = (int)std::max<size_t>(1, budget / (img * 8 * S));
    snaps_per = std::min(snaps_per, (int)n_snap);
    float2* gk = (float2*)workspace(ctx, "vk", (size_t)snaps_per * S * img * sizeof(float2));
    const int cap = snaps_per * K + (int)(((long)snaps_per * n_atoms + 63) / 64) + 1;
    int4* chunks = (int4*)workspace(ctx, "chunks", (size_t)cap * sizeof(int4) + 16);
    int* count = (int*)(chunks + cap);
    void* arec = workspace(ctx, "atom_phase", (size_t)snaps_per * n_atoms * 24);
    const bool herm = spec->bandlimit > 0.0 && spec->bandlimit < 1.0 && spec->ny >= 128;
    const double pref = 2.0 * kPi * kA0 * kE4pe0 / (spec->lx * spec->ly);
    double hbound = 0.0;
    const float* vtab = upload_vec(
        ctx, pos_grad_table(*spec, ff, n_species, bandlimit_table(*spec), herm, pref, &hbound), st,
        "pg_vtab");
    float* absmax = (float*)workspace(ctx, "pg_absmax", (size_t)snaps_per * S * sizeof(float));
    // liveness of every (64-wide kx tile, 32-row ky fill) of the visited rows, as the kernel's
    // tiles and fills are laid out
    const int* fill_live;
    {
      const std::vector<int> blt = bandlimit_table(*spec);
      const int TW = std::min(64, spec->nx), tx_n = (spec->nx + TW - 1) / TW;
      const int ny_h = herm ? spec->ny / 2 : spec->ny, nf = (ny_h + 31) / 32;
      std::vector<int> live((size_t)tx_n * nf, 0);
      for (int tx = 0; tx < tx_n; ++tx)
        for (int f = 0; f < nf; ++f) {
          int minabs = 1 << 30;
          for (int n = 32 * f; n < std::min(32 * f + 32, ny_h); ++n) {
            const int ns = n < spec->ny / 2 ? n : n - spec->ny;
            minabs = std::min(minabs, ns < 0 ? -ns : ns);
          }
          for (int m = tx * TW; m < std::min(tx * TW + TW, spec->nx); ++m)
            if (blt[m] >= minabs) live[(size_t)tx * nf + f] = 1;
        }
      fill_live = upload_vec(ctx, live, st, "pg_fills");
    }
    // the gradient kernels visit only the band's columns (nx / 2: every column)
    const int kxb_g = band_columns(bandlimit_table(*spec));
    for (int t0 = 0; t0 < n_snap; t0 += snaps_per) {
      const int nt = std::min(snaps_per, n_snap - t0);
      hip_check(launch_zero(absmax, (size_t)nt * S * sizeof(float), st), "zero");
      hip_check(launch_fft2_real(spec->nx, spec->ny, grad_V + (size_t)t0 * S * img, gk, nt * S,
                                 kxb_g, herm ? spec->ny / 2 : spec->ny, absmax, st),
                "gradient FFT");
      hip_check(launch_chunk_list(offs, t0, nt, S, n_species, chunks, cap, count, st), "chunk list");
      hip_check(launch_atom_phase(xyz, ord, t0, nt, n_atoms, spec->lx, spec->ly, arec, st),
                "atom phases");
      PgArgs a{};
      a.xyz = xyz;
      a.order = ord;
      a.offsets = offs;
      a.ff = ffd;
      a.gk = gk;
      a.gxy = grad_xy;
      a.t0 = t0;
      a.s_count = S;
      a.n_atoms = n_atoms;
      a.n_species = n_species;
      a.nx = spec->nx;
      a.ny = spec->ny;
      a.n_maps = nt * S;
      a.lx = spec->lx;
      a.ly = spec->ly;
      a.pref = (float)(2.0 * kPi * kA0 * kE4pe0 / (spec->lx * spec->ly));
      a.nmax = nmax;
      a.arec = arec;
      a.hermitian = herm ? 1 : 0;
      a.vtab = vtab;
      a.hbound = (float)hbound;
      a.absmax = absmax;
      a.fill_live = fill_live;
      timed_launch(ctx, st, "pos_grad", 0.0, [&] {
        hip_check(launch_position_grad_chunks(a, chunks, cap, count, st), "position-gradient kernel");
      });
    }
  });
}

// ------------------------------------------------------------------------------------------------
int tacaw_multislice(tacaw_ctx* ctx, int32_t n_jobs, const tacaw_ms_job* jobs, int32_t ckpt_stride,
                     int32_t mode, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (mode != TACAW_MODE_PLAIN && mode != TACAW_MODE_BATCHED && mode != TACAW_MODE_PERSISTENT)
      fail(TACAW_E_ARG, "unknown mode");
    hipStream_t st = (hipStream_t)stream;
    MsBuild b = build_ms(ctx, n_jobs, jobs, ckpt_stride, st, false, nullptr, nullptr);
    if (mode != TACAW_MODE_PLAIN) attach_entrance(ctx, b);
    b.jobs_dev = upload_vec(ctx, b.jobs, st, "jobs");
    if (mode == TACAW_MODE_PLAIN || ctx->timing) {
      run_forward(ctx, b, ckpt_stride, mode, st);   // timing: eager launches bracketed by events
      return;
    }
    const std::string key = graph_key(b, ckpt_stride, mode, ctx);
    const size_t jbytes = b.jobs.size() * sizeof(MsJobDev);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
      // lists must be resident before capture (uploads are not captured)
      for (auto& cp : b.classes) {
        upload_vec(ctx, cp.groups, st, "groups");
        upload_vec(ctx, cp.waves, st, "waves");
        if (!cp.plane_waves.empty()) upload_vec(ctx, cp.plane_waves, st, "pw");
        if (!cp.probe_waves.empty()) upload_vec(ctx, cp.probe_waves, st, "pr");
        if (!cp.probe_copies.empty()) upload_vec(ctx, cp.probe_copies, st, "pc");
      }
      if (ctx->graphs.size() >= ctx->max_graphs) {
        auto lru = ctx->graphs.begin();
        for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
          if (g->second.last_use < lru->second.last_use) lru = g;
        hip_check(hipEventSynchronize(lru->second.done), "hipEventSynchronize");
        destroy_graph(lru->second);
        ctx->graphs.erase(lru);
      }
      tacaw_ctx::GraphEntry e;
      e.jobs_bytes = jbytes;
      if (hipMalloc(&e.jobs_dev, jbytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(TACAW_E_NOMEM, "graph job table");
      }
      hipError_t er = hipEventCreateWithFlags(&e.done, hipEventDisableTiming);
      if (er == hipSuccess) er = hipEventRecord(e.done, st);
      if (er != hipSuccess) {
        (void)hipFree(e.jobs_dev);
        if (e.done) (void)hipEventDestroy(e.done);
        hip_check(er, "graph event");
      }
      MsBuild cb = b;
      cb.jobs_dev = e.jobs_dev;
      hipGraph_t g = nullptr;
      er = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
      if (er == hipSuccess) {
        try {
          run_forward(ctx, cb, ckpt_stride, mode, ctx->cap_stream);
        } catch (...) {
          hipGraph_t dummy = nullptr;
          (void)hipStreamEndCapture(ctx->cap_stream, &dummy);
          if (dummy) (void)hipGraphDestroy(dummy);
          destroy_graph(e);
          throw;
        }
        er = hipStreamEndCapture(ctx->cap_stream, &g);
      }
      if (er == hipSuccess) er = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (er != hipSuccess) {
        destroy_graph(e);
        hip_check(er, "graph capture");
      }
      it = ctx->graphs.emplace(key, e).first;
    }
    tacaw_ctx::GraphEntry& e = it->second;
    e.last_use = ++ctx->use_clock;
    // the previous replay (on any stream) has read the table before it is rewritten
    hip_check(hipStreamWaitEvent(st, e.done, 0), "hipStreamWaitEvent");
    hip_check(hipMemcpyAsync(e.jobs_dev, b.jobs_dev, jbytes, hipMemcpyDeviceToDevice, st),
              "job table copy");
    hip_check(hipGraphLaunch(e.exec, st), "hipGraphLaunch");
    hip_check(hipEventRecord(e.done, st), "hipEventRecord");
  });
}

int tacaw_multislice_adjoint(tacaw_ctx* ctx, int32_t n_jobs, const tacaw_ms_job* jobs,
                             int32_t ckpt_stride, const tacaw_c64* const* grad_exit,
                             float* const* grad_V, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (ckpt_stride < 1) fail(TACAW_E_ARG, "the adjoint needs the forward checkpoints (stride >= 1)");
    hipStream_t st = (hipStream_t)stream;
    MsBuild b = build_ms(ctx, n_jobs, jobs, ckpt_stride, st, true, grad_exit, grad_V);
    // workspace per job: adjoint state, recompute buffer, stash of one segment
    size_t total = 0;
    std::vector<size_t> offs(n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
      const MsJobDev& d = b.jobs[j];
      const size_t img = (size_t)d.nx * d.ny * sizeof(float2);
      offs[j] = total;
      total += img * d.T * d.P * (2 + ckpt_stride);
    }
    char* base = (char*)workspace(ctx, "adjoint", total);
    for (int j = 0; j < n_jobs; ++j) {
      MsJobDev& d = b.jobs[j];
      const size_t img = (size_t)d.nx * d.ny * sizeof(float2);
      const size_t n = (size_t)d.T * d.P;
      d.adj = (float2*)(base + offs[j]);
      d.rec = (float2*)(base + offs[j] + img * n);
      d.stash = (float2*)(base + offs[j] + 2 * img * n);
    }
    b.jobs_dev = upload_vec(ctx, b.jobs, st, "jobs");
    Launcher L{ctx, st};
    for (const ClassPlan& cp : b.classes) {
      const Sched rs = schedule_for(ctx, cp.nx);
      const Sched cs = fit_cols(ctx, cp.ny, schedule_for(ctx, cp.ny), cp.nx);
      // process jobs of equal slice count together: segments then align
      std::map<int, std::pair<std::vector<int2>, std::vector<int4>>, std::greater<int>> byS;
      for (auto g : cp.groups) byS[b.jobs[g.x].S].first.push_back(g);
      for (auto w : cp.waves) byS[b.jobs[w.x].S].second.push_back(w);
      for (auto& kv : byS) {
        const int S = kv.first;
        int2* groups = upload_vec(ctx, kv.second.first, st, "groups");
        int4* waves = upload_vec(ctx, kv.second.second, st, "waves");
        const int ng = (int)kv.second.first.size(), nw = (int)kv.second.second.size();
        const float scale_mid = (float)(1.0 / ((double)cp.nx * cp.ny));
        const float scale_last = (float)(1.0 / std::sqrt((double)cp.nx * cp.ny));
        ColArgs ca{};
        ca.jobs = b.jobs_dev;
        ca.waves = waves;
        ca.n_waves = nw;
        ca.C = cs.C;
        ca.nx = cp.nx;
        ca.prune = plan_prunable(cp.ny, cs.col_plan, cp.kyb) ? 1 : 0;
        // chi_{S-1} in (kx, y): G_y[conj(M P_{S-1}) G_phi] / sqrt(N)
        ca.s = S - 1;
        ca.in_buf = BUF_GEXIT;
        ca.out_buf = BUF_ADJ;
        ca.conj_prop = 1;
        ca.scale = scale_last;
        L.col(cp.ny, cs, false, true, ca, cp.kxb, false);
        const int nck = (S + ckpt_stride - 1) / ckpt_stride;
        for (int c = nck - 1; c >= 0; --c) {
          const int s0 = c * ckpt_stride, s1 = std::min(S, s0 + ckpt_stride);
          for (int s = s0; s < s1; ++s) {
            RowArgs ra{};
            ra.jobs = b.jobs_dev;
            ra.groups = groups;
            ra.n_groups = ng;
            ra.s = s;
            ra.in_buf = (s == s0) ? BUF_CKPT : BUF_REC;
            ra.out_buf = BUF_REC;
            ra.store_ckpt = 0;
            ra.stash_slot = s - s0;
            ra.write_out = (s < s1 - 1) ? 1 : 0;
            ra.ny = cp.ny;
            ra.band_in = s > 0 ? 1 : 0;
            ra.band_out = 1;
            ra.prune = (s > 0 && plan_prunable(cp.nx, rs.row_plan, cp.kxb)) ? 1 : 0;
            ra.single_pos = cp.maxP == 1 ? 1 : 0;
            L.row(cp.nx, rs, false, ra, nw, cp.kxb);
            if (s < s1 - 1) {
              ColArgs fa = ca;
              fa.s = s;
              fa.in_buf = BUF_REC;
              fa.out_buf = BUF_REC;
              fa.conj_prop = 0;
              fa.scale = scale_mid;
              L.col(cp.ny, cs, true, true, fa, cp.kxb, false);
            }
          }
          for (int s = s1 - 1; s >= s0; --s) {
            RowArgs ra{};
            ra.jobs = b.jobs_dev;
            ra.groups = groups;
            ra.n_groups = ng;
            ra.s = s;
            ra.in_buf = BUF_ADJ;
            ra.out_buf = BUF_ADJ;
            ra.store_ckpt = 0;
            ra.stash_slot = s - s0;
            ra.write_out = s > 0 ? 1 : 0;
            ra.ny = cp.ny;
            ra.band_in = 1;    // adjoint states leave the adjoint y pass band-limited
            ra.band_out = 1;
            L.row(cp.nx, rs, true, ra, nw, cp.kxb);
            if (s > 0) {
              ColArgs aa = ca;
              aa.s = s - 1;
              aa.in_buf = BUF_ADJ;
              aa.out_buf = BUF_ADJ;
              aa.conj_prop = 1;
              aa.scale = scale_mid;
              L.col(cp.ny, cs, true, true, aa, cp.kxb, false);
            }
          }
        }
      }
    }
  });
}

// ------------------------------------------------------------------------------------------------
static void validate_spectrum(int nx, int ny, int n_snap, int n_pos, const tacaw_c64* exit,
                              int n_e, int hop) {
  if (!grid_size_ok(nx) || !grid_size_ok(ny)) fail(TACAW_E_SIZE, "grid size");
  if (n_snap < 1 || n_pos < 1 || !exit) fail(TACAW_E_ARG, "bad exit stack");
  if (!pow2_in(n_e, 16, 1024)) fail(TACAW_E_SIZE, "n_e must be a power of two in [16, 1024]");
  // the time-line kernels take whole tiles of consecutive q
  if (((long)nx * ny) % spectrum_q_tile(n_e) != 0)
    fail(TACAW_E_SIZE, "nx * ny must be a multiple of " + std::to_string(spectrum_q_tile(n_e)) +
                           " for n_e = " + std::to_string(n_e));
  if (hop < 1) fail(TACAW_E_ARG, "hop must be >= 1");
  if (n_e > n_snap) fail(TACAW_E_ARG, "segment longer than the trajectory");
}

int tacaw_periodogram_positions(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap,
                                int32_t n_pos, const tacaw_c64* exit, int32_t pos0,
                                int32_t n_pos_used, int32_t n_e, int32_t hop, float* P_acc,
                                int32_t accumulate, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_spectrum(nx, ny, n_snap, n_pos, exit, n_e, hop);
    if (!P_acc) fail(TACAW_E_ARG, "null P_acc");
    if (pos0 < 0 || n_pos_used < 1 || (long)pos0 + n_pos_used > n_pos)
      fail(TACAW_E_ARG, "position range outside the stack");
    SpecArgs a{};
    a.exit = (const float2*)exit;
    a.P = P_acc;
    a.T = n_snap;
    a.Ps = n_pos;
    a.p0 = pos0;
    a.Pn = n_pos_used;
    a.nq = nx * ny;
    a.n_e = n_e;
    a.hop = hop;
    a.G = (n_snap - n_e) / hop + 1;
    a.accumulate = accumulate ? 1 : 0;
    const double bytes = 8.0 * nx * ny * (double)n_e * a.G * n_pos_used +
                         (accumulate ? 8.0 : 4.0) * nx * ny * (double)n_e;
    timed_launch(ctx, (hipStream_t)stream, "pgram", bytes, [&] {
      hip_check(launch_periodogram(a, (hipStream_t)stream), "periodogram kernel");
    });
  });
}

int tacaw_periodogram(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap, int32_t n_pos,
                      const tacaw_c64* exit, int32_t n_e, int32_t hop, float* P_acc,
                      int32_t accumulate, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_spectrum(nx, ny, n_snap, n_pos, exit, n_e, hop);
    if (!P_acc) fail(TACAW_E_ARG, "null P_acc");
    SpecArgs a{};
    a.exit = (const float2*)exit;
    a.P = P_acc;
    a.T = n_snap;
    a.Ps = n_pos;
    a.p0 = 0;
    a.Pn = n_pos;
    a.nq = nx * ny;
    a.n_e = n_e;
    a.hop = hop;
    a.G = (n_snap - n_e) / hop + 1;
    a.accumulate = accumulate ? 1 : 0;
    const double bytes = 8.0 * nx * ny * (double)n_e * a.G * n_pos +
                         (accumulate ? 8.0 : 4.0) * nx * ny * (double)n_e;
    timed_launch(ctx, (hipStream_t)stream, "pgram", bytes, [&] {
      hip_check(launch_periodogram(a, (hipStream_t)stream), "periodogram kernel");
    });
  });
}

static void validate_opts(const tacaw_spectrum_opts* o, int nx, int ny) {
  if (!o) fail(TACAW_E_ARG, "null spectrum options");
  if (!(o->dt_fs > 0) || !(o->temperature_k > 0)) fail(TACAW_E_ARG, "dt and temperature must be > 0");
  if (o->nqx_out < 1 || o->nqx_out > nx || o->nqy_out < 1 || o->nqy_out > ny)
    fail(TACAW_E_ARG, "output crop outside the q grid");
}

int tacaw_spectrum_finalize(tacaw_ctx* ctx, int32_t nx, int32_t ny, const float* P_acc,
                            const tacaw_spectrum_opts* opts, float* S, double* norm, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_opts(opts, nx, ny);
    if (!pow2_in(opts->n_e, 16, 1024)) fail(TACAW_E_SIZE, "n_e must be a power of two in [16, 1024]");
    if (!P_acc || !S) fail(TACAW_E_ARG, "null buffers");
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> kd = kubo_dft_order(opts->n_e, opts->dt_fs, opts->temperature_k);
    std::vector<float> kf(kd.begin(), kd.end());
    FinArgs a{};
    a.P = P_acc;
    a.K = upload_vec(ctx, kf, st, "kubo");
    a.S = S;
    a.n_part = 512;
    double* part = (double*)workspace(ctx, "partial", (a.n_part + 2) * sizeof(double));
    a.partial = part;
    a.norm = norm ? norm : part + a.n_part;
    a.n_e = opts->n_e;
    a.nx = nx;
    a.ny = ny;
    a.nqx = opts->nqx_out;
    a.nqy = opts->nqy_out;
    hip_check(launch_finalize(a, st), "finalize kernels");
  });
}

int tacaw_spectrum_finalize_noalloc(tacaw_ctx* ctx, int32_t nx, int32_t ny, const float* P_acc,
                                    const tacaw_spectrum_opts* opts, float* S, double* norm,
                                    void* stream) {
  return guarded([&] {
    // no CallScope: it may drop cached tables (hipFree); nothing here allocates or frees
    use_device(ctx);
    validate_opts(opts, nx, ny);
    if (!pow2_in(opts->n_e, 16, 1024)) fail(TACAW_E_SIZE, "n_e must be a power of two in [16, 1024]");
    if (!P_acc || !S) fail(TACAW_E_ARG, "null buffers");
    if (kNoallocKuboOff + (size_t)opts->n_e * sizeof(float) > kScratchBytes ||
        (size_t)(kNoallocParts + 2) * sizeof(double) > kNoallocKuboOff)
      fail(TACAW_E_SIZE, "n_e = " + std::to_string(opts->n_e) + " does not fit the " +
                             std::to_string(kScratchBytes) + "-byte scratch");
    if (!ctx->scratch_dev) fail(TACAW_E_STATE, "no scratch address for this device");
    hipStream_t st = (hipStream_t)stream;
    double* part = (double*)ctx->scratch_dev;
    float* K = (float*)(ctx->scratch_dev + kNoallocKuboOff);
    hip_check(launch_kubo_fill(K, opts->n_e, opts->dt_fs, 1.0 / (kKb * opts->temperature_k), st),
              "Kubo table");
    FinArgs a{};
    a.P = P_acc;
    a.K = K;
    a.S = S;
    a.n_part = kNoallocParts;
    a.partial = part;
    a.norm = norm ? norm : part + kNoallocParts;
    a.n_e = opts->n_e;
    a.nx = nx;
    a.ny = ny;
    a.nqx = opts->nqx_out;
    a.nqy = opts->nqy_out;
    hip_check(launch_finalize(a, st), "finalize kernels");
  });
}

int tacaw_autocorr_spectrum(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap, int32_t n_pos,
                            const tacaw_c64* exit, const tacaw_spectrum_opts* opts, float* S,
                            double* norm, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_opts(opts, nx, ny);
    validate_spectrum(nx, ny, n_snap, n_pos, exit, opts->n_e, opts->hop);
    if (!S) fail(TACAW_E_ARG, "null S");
    float* P = (float*)workspace(ctx, "pacc", (size_t)opts->n_e * nx * ny * sizeof(float));
    int r = tacaw_periodogram(ctx, nx, ny, n_snap, n_pos, exit, opts->n_e, opts->hop, P, 0, stream);
    if (r != TACAW_OK) throw Fail{r};
    r = tacaw_spectrum_finalize(ctx, nx, ny, P, opts, S, norm, stream);
    if (r != TACAW_OK) throw Fail{r};
  });
}

int tacaw_autocorr_spectrum_backward(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap,
                                     int32_t n_pos, const tacaw_c64* exit,
                                     const tacaw_spectrum_opts* opts, const float* S,
                                     const double* norm, const float* grad_S,
                                     tacaw_c64* grad_exit, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_opts(opts, nx, ny);
    validate_spectrum(nx, ny, n_snap, n_pos, exit, opts->n_e, opts->hop);
    if (!S || !norm || !grad_S || !grad_exit) fail(TACAW_E_ARG, "null buffers");
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> kd = kubo_dft_order(opts->n_e, opts->dt_fs, opts->temperature_k);
    std::vector<float> kf(kd.begin(), kd.end());
    SpecBwdArgs a{};
    a.exit = (const float2*)exit;
    a.S = S;
    a.norm = norm;
    a.gS = grad_S;
    a.K = upload_vec(ctx, kf, st, "kubo");
    a.gexit = (float2*)grad_exit;
    a.n_part = 512;
    a.partial = (double*)workspace(ctx, "partial_b", (a.n_part + 2) * sizeof(double));
    a.T = n_snap;
    a.Pn = n_pos;
    a.nx = nx;
    a.ny = ny;
    a.nq = nx * ny;
    a.n_e = opts->n_e;
    a.hop = opts->hop;
    a.G = (n_snap - opts->n_e) / opts->hop + 1;
    a.nqx = opts->nqx_out;
    a.nqy = opts->nqy_out;
    hip_check(launch_spectrum_backward(a, st), "spectrum backward");
  });
}

// ------------------------------------------------------------------------------------------------
// streamed segment periodograms
struct tacaw_segstream {
  tacaw_ctx* ctx = nullptr;
  int nx = 0, ny = 0, n_pos = 0, n_e = 0, hop = 0;
  float* P = nullptr;            // caller's accumulator [n_e][ny][nx]
  float2* win = nullptr;         // window of snapshots [cap][n_pos][nx ny] (library-owned)
  long cap = 0;                  // window capacity (snapshots)
  long w0 = 0;                   // trajectory index of window slot 0
  long len = 0;                  // snapshots held
  long pushed = 0;               // snapshots received so far
  long done = 0;                 // segments accumulated
  bool finished = false;
  ~tacaw_segstream() {
    if (win) {
      (void)hipSetDevice(ctx->device);
      (void)hipDeviceSynchronize();
      (void)hipFree(win);
    }
  }
};

int tacaw_segstream_create(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_pos, int32_t n_e,
                           int32_t hop, float* P_acc, tacaw_segstream** out) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (!out) fail(TACAW_E_ARG, "out is NULL");
    *out = nullptr;
    if (!grid_size_ok(nx) || !grid_size_ok(ny)) fail(TACAW_E_SIZE, "grid size");
    if (n_pos < 1 || hop < 1 || !P_acc) fail(TACAW_E_ARG, "need n_pos >= 1, hop >= 1 and P_acc");
    if (!pow2_in(n_e, 16, 1024)) fail(TACAW_E_SIZE, "n_e must be a power of two in [16, 1024]");
    if (((long)nx * ny) % spectrum_q_tile(n_e) != 0)
      fail(TACAW_E_SIZE, "nx * ny must be a multiple of " + std::to_string(spectrum_q_tile(n_e)));
    auto s = std::make_unique<tacaw_segstream>();
    s->ctx = ctx;
    s->nx = nx;
    s->ny = ny;
    s->n_pos = n_pos;
    s->n_e = n_e;
    s->hop = hop;
    s->P = P_acc;
    *out = s.release();
  });
}

int tacaw_segstream_push(tacaw_segstream* s, int32_t n_snap, const tacaw_c64* exit, void* stream) {
  return guarded([&] {
    if (!s) fail(TACAW_E_ARG, "null stream object");
    use_device(s->ctx);
    if (s->finished) fail(TACAW_E_STATE, "the stream was finished");
    if (n_snap < 1 || !exit) fail(TACAW_E_ARG, "need n_snap >= 1 and exit waves");
    hipStream_t st = (hipStream_t)stream;
    const size_t snap = (size_t)s->n_pos * s->nx * s->ny;   // complex values per snapshot
    if (s->len + n_snap > s->cap) {
      const long cap = std::max<long>({2 * s->cap, s->len + n_snap, (long)s->n_e + n_snap});
      float2* nw = nullptr;
      if (hipMalloc(&nw, (size_t)cap * snap * sizeof(float2)) != hipSuccess) {
        (void)hipGetLastError();
        fail(TACAW_E_NOMEM, "segment stream window of " + std::to_string(cap) + " snapshots");
      }
      if (s->len > 0)
        hip_check(hipMemcpyAsync(nw, s->win, (size_t)s->len * snap * sizeof(float2),
                                 hipMemcpyDeviceToDevice, st), "window copy");
      if (s->win) {
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        hip_check(hipFree(s->win), "hipFree");
      }
      s->win = nw;
      s->cap = cap;
    }
    hip_check(hipMemcpyAsync(s->win + (size_t)s->len * snap, exit, (size_t)n_snap * snap * sizeof(float2),
                             hipMemcpyDeviceToDevice, st), "window append");
    s->len += n_snap;
    s->pushed += n_snap;
    // every segment whose snapshots have all arrived: its periodogram, added to P
    while (s->done * s->hop + s->n_e <= s->pushed) {
      const long off = s->done * s->hop - s->w0;
      SpecArgs a{};
      a.exit = s->win + (size_t)off * snap;
      a.P = s->P;
      a.T = s->n_e;
      a.Ps = s->n_pos;
      a.p0 = 0;
      a.Pn = s->n_pos;
      a.nq = s->nx * s->ny;
      a.n_e = s->n_e;
      a.hop = s->n_e;
      a.G = 1;
      a.accumulate = s->done > 0 ? 1 : 0;
      hip_check(launch_periodogram(a, st), "periodogram kernel");
      ++s->done;
    }
    // drop the snapshots before the next segment's start (moved down in pieces that do not
    // overlap their destination)
    const long keep_from = s->done * s->hop;
    const long shift = std::min(std::max(0L, keep_from - s->w0), s->len);
    if (shift > 0) {
      for (long o = 0; o < s->len - shift; o += shift) {
        const long m = std::min(shift, s->len - shift - o);
        hip_check(hipMemcpyAsync(s->win + (size_t)o * snap, s->win + (size_t)(shift + o) * snap,
                                 (size_t)m * snap * sizeof(float2), hipMemcpyDeviceToDevice, st),
                  "window shift");
      }
      s->w0 += shift;
      s->len -= shift;
    }
  });
}

int tacaw_segstream_finish(tacaw_segstream* s, int32_t* n_segments, void* stream) {
  return guarded([&] {
    if (!s) fail(TACAW_E_ARG, "null stream object");
    use_device(s->ctx);
    if (s->finished) fail(TACAW_E_STATE, "the stream was finished");
    if (s->done < 1) fail(TACAW_E_STATE, "no complete segment was pushed");
    hip_check(launch_scale(s->P, (long)s->n_e * s->nx * s->ny, (float)(1.0 / (double)s->done),
                           (hipStream_t)stream), "scale");
    s->finished = true;
    if (n_segments) *n_segments = (int32_t)s->done;
  });
}

int tacaw_segstream_window(const tacaw_segstream* s, int32_t* capacity, int32_t* held) {
  return guarded([&] {
    if (!s) fail(TACAW_E_ARG, "null stream object");
    if (capacity) *capacity = (int32_t)s->cap;
    if (held) *held = (int32_t)s->len;
  });
}

void tacaw_segstream_destroy(tacaw_segstream* s) { delete s; }

// ------------------------------------------------------------------------------------------------
// analysis outputs
static void validate_crop(int nx, int ny, int nqx, int nqy) {
  if (nx < 1 || ny < 1 || (long)nx * ny > (1L << 30)) fail(TACAW_E_ARG, "bad grid");
  if (nqx < 1 || nqx > nx || nqy < 1 || nqy > ny) fail(TACAW_E_ARG, "output crop outside the q grid");
}

int tacaw_energy_integrals(tacaw_ctx* ctx, int32_t nx, int32_t ny, const float* P_acc,
                           const tacaw_spectrum_opts* opts, float* c_tilde, float* c,
                           void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_opts(opts, nx, ny);
    validate_crop(nx, ny, opts->nqx_out, opts->nqy_out);
    if (!pow2_in(opts->n_e, 16, 1024)) fail(TACAW_E_SIZE, "n_e must be a power of two in [16, 1024]");
    if (!P_acc || (!c_tilde && !c)) fail(TACAW_E_ARG, "null buffers");
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> kd = kubo_dft_order(opts->n_e, opts->dt_fs, opts->temperature_k);
    std::vector<float> kf(kd.begin(), kd.end());
    const float* K = upload_vec(ctx, kf, st, "kubo");
    const long nq = (long)nx * ny;
    const int n_part = 512;
    double* sums = (double*)workspace(ctx, "an_sums", 2 * nq * sizeof(double));
    double* part = (double*)workspace(ctx, "an_partial", (n_part + 1) * sizeof(double));
    hip_check(launch_energy_sums(P_acc, K, opts->n_e, nq, sums, sums + nq, st), "energy sums");
    if (c_tilde)
      hip_check(launch_norm_crop(sums, nq, nx, ny, opts->nqx_out, opts->nqy_out, part, n_part,
                                 c_tilde, st), "pattern");
    if (c)
      hip_check(launch_norm_crop(sums + nq, nq, nx, ny, opts->nqx_out, opts->nqy_out, part, n_part,
                                 c, st), "pattern");
  });
}

int tacaw_qep_pattern(tacaw_ctx* ctx, int32_t nx, int32_t ny, int32_t n_snap, int32_t n_pos,
                      const tacaw_c64* exit, int32_t t0, int32_t t_stride, int32_t t_count,
                      int32_t nqx_out, int32_t nqy_out, float* out, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    validate_crop(nx, ny, nqx_out, nqy_out);
    if (n_snap < 1 || n_pos < 1 || !exit || !out) fail(TACAW_E_ARG, "bad exit stack or output");
    if (t0 < 0 || t_stride < 1 || t_count < 1 || (long)t0 + (long)(t_count - 1) * t_stride >= n_snap)
      fail(TACAW_E_ARG, "snapshot selection outside the stack");
    hipStream_t st = (hipStream_t)stream;
    const long nq = (long)nx * ny;
    const int n_part = 512;
    double* sums = (double*)workspace(ctx, "an_sums", 2 * nq * sizeof(double));
    double* part = (double*)workspace(ctx, "an_partial", (n_part + 1) * sizeof(double));
    hip_check(launch_snapshot_sums((const float2*)exit, n_pos, nq, t0, t_stride, t_count, sums, st),
              "snapshot sums");
    hip_check(launch_norm_crop(sums, nq, nx, ny, nqx_out, nqy_out, part, n_part, out, st), "pattern");
  });
}

int tacaw_relative_difference(tacaw_ctx* ctx, int32_t nqx, int32_t nqy, const float* A,
                              const float* B, float* out_row, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (nqx < 1 || nqy < 1 || !A || !B || !out_row) fail(TACAW_E_ARG, "bad maps or output");
    hip_check(launch_rel_diff_row(A, B, nqx, nqy, out_row, (hipStream_t)stream), "profile");
  });
}

int tacaw_path_cut(tacaw_ctx* ctx, double lx, double ly, int32_t nqx, int32_t nqy, int32_t n_e,
                   const float* S, int32_t n_vert, const double* vertices, int32_t n_per_seg,
                   float* out, void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (!(lx > 0) || !(ly > 0)) fail(TACAW_E_ARG, "cell lengths must be positive");
    if (nqx < 1 || nqy < 1 || n_e < 1 || !S || !out) fail(TACAW_E_ARG, "bad spectrum or output");
    if (n_vert < 2 || !vertices || n_per_seg < 1) fail(TACAW_E_ARG, "need >= 2 vertices and >= 1 point per segment");
    for (int i = 0; i < 2 * n_vert; ++i)
      if (!std::isfinite(vertices[i])) fail(TACAW_E_ARG, "vertices must be finite");
    // points along the polyline (n_per_seg per segment from its first vertex, then the last
    // vertex) as fractional pixel positions of the centred map: q l + nq / 2
    std::vector<double2> uv;
    auto push = [&](double qx, double qy) {
      uv.push_back(make_double2(qx * lx + (double)(nqx / 2), qy * ly + (double)(nqy / 2)));
    };
    for (int sgm = 0; sgm + 1 < n_vert; ++sgm)
      for (int j = 0; j < n_per_seg; ++j) {
        const double f = (double)j / n_per_seg;
        push(vertices[2 * sgm] + f * (vertices[2 * sgm + 2] - vertices[2 * sgm]),
             vertices[2 * sgm + 1] + f * (vertices[2 * sgm + 3] - vertices[2 * sgm + 1]));
      }
    push(vertices[2 * n_vert - 2], vertices[2 * n_vert - 1]);
    hipStream_t st = (hipStream_t)stream;
    const double2* d_uv = upload_vec(ctx, uv, st, "path");
    hip_check(launch_path_cut(S, n_e, nqx, nqy, d_uv, (int)uv.size(), out, st), "path cut");
  });
}

// ------------------------------------------------------------------------------------------------
// timing instrumentation
int tacaw_set_timing(tacaw_ctx* ctx, int32_t enable) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    ctx->timing = enable != 0;
  });
}

int tacaw_set_potential_precision(tacaw_ctx* ctx, int32_t split16) {
  return guarded([&] {
    if (!ctx) fail(TACAW_E_ARG, "null context");
    if (split16 != 0 && split16 != 1) fail(TACAW_E_ARG, "split16 must be 0 or 1");
    ctx->sf_split16 = split16;
  });
}

int tacaw_set_slice_blocking(tacaw_ctx* ctx, int64_t block_bytes, int32_t streams) {
  return guarded([&] {
    if (!ctx) fail(TACAW_E_ARG, "null context");
    if (block_bytes < 0) fail(TACAW_E_ARG, "block_bytes must be >= 0");
    if (streams < 1 || streams > (int32_t)tacaw_ctx::kSide) fail(TACAW_E_ARG, "streams must be 1..3");
    ctx->block_bytes = block_bytes;
    ctx->block_streams = streams;
  });
}

int tacaw_get_timing(tacaw_ctx* ctx, const char* kind, tacaw_kernel_stats* out) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (!out) fail(TACAW_E_ARG, "null output");
    *out = tacaw_kernel_stats{0, 0.0, 0.0};
    fold_timed(ctx);
    for (auto it = ctx->timed_sums.begin(); it != ctx->timed_sums.end();) {
      if (kind && *kind && it->first != kind) {
        ++it;
        continue;
      }
      out->launches += it->second.launches;
      out->total_ms += it->second.total_ms;
      out->algo_bytes += it->second.algo_bytes;
      it = ctx->timed_sums.erase(it);
    }
  });
}

int tacaw_set_cache_limits(tacaw_ctx* ctx, int64_t max_entries, int64_t max_bytes,
                           int32_t max_graphs) {
  return guarded([&] {
    if (!ctx) fail(TACAW_E_ARG, "null context");
    if (max_entries < 1 || max_bytes < 1 || max_graphs < 1) fail(TACAW_E_ARG, "cache limits must be >= 1");
    ctx->cache_max_entries = (size_t)max_entries;
    ctx->cache_max_bytes = (size_t)max_bytes;
    ctx->max_graphs = (size_t)max_graphs;
  });
}

int tacaw_cache_stats(tacaw_ctx* ctx, int64_t* n_tables, int64_t* table_bytes, int32_t* n_graphs) {
  return guarded([&] {
    if (!ctx) fail(TACAW_E_ARG, "null context");
    if (n_tables) *n_tables = (int64_t)ctx->cache.size();
    if (table_bytes) *table_bytes = (int64_t)ctx->cache_bytes;
    if (n_graphs) *n_graphs = (int32_t)ctx->graphs.size();
  });
}

// ------------------------------------------------------------------------------------------------
// autotuning
static std::string sched_line(int n, const Sched& s) {
  std::ostringstream o;
  o << "row=" << plan_name(n, s.row_plan) << " col=" << plan_name(n, s.col_plan) << " C=" << s.C
    << (s.col_kind == 1 ? " block" : s.col_kind == 2 ? " wave-per-column" : " staged")
    << (s.col_kind == 1 && s.pp ? " pingpong" : "") << (s.col_kind == 1 && s.pp == 2 ? " split-layout" : "");
  return o.str();
}

int tacaw_plan_count(int32_t n) { return grid_size_ok(n) ? n_plans(n) : 0; }

const char* tacaw_describe_schedule(tacaw_ctx* ctx, int32_t n) {
  if (!ctx || !grid_size_ok(n)) return "";
  ctx->desc = sched_line(n, schedule_for(ctx, n));
  return ctx->desc.c_str();
}

int tacaw_load_tuning(tacaw_ctx* ctx, const char* path) {
  return guarded([&] {
    if (!ctx || !path) fail(TACAW_E_ARG, "null argument");
    std::ifstream f(path);
    if (!f) return;
    // one entry per line: {"arch": "gfx950", "n": 512, "row": 0, "col": 0, "C": 16}
    std::string line;
    while (std::getline(f, line)) {
      if (line.find("\"n\"") == std::string::npos) continue;
      auto num = [&](const char* k) -> int {
        auto p = line.find(std::string("\"") + k + "\"");
        if (p != std::string::npos) p = line.find(':', p);
        if (p == std::string::npos) fail(TACAW_E_ARG, std::string("tuning line lacks ") + k);
        return std::atoi(line.c_str() + p + 1);
      };
      int n = num("n");
      Sched s;
      s.row_plan = num("row");
      s.col_plan = num("col");
      s.C = num("C");
      s.col_kind = num("kind");
      s.pp = num("pp");
      if (!grid_size_ok(n) || s.row_plan < 0 || s.row_plan >= n_plans(n) || s.col_plan < 0 ||
          s.col_plan >= n_plans(n) || !pow2_in(s.C, 1, 64) || n % s.C != 0 || s.col_kind < 0 ||
          s.col_kind > 2 || s.pp < 0 || s.pp > 2 || !plan_kind_ok(n, s.col_plan, s.col_kind) ||
          (s.pp == 2 && (s.col_kind != 1 || col_block_lx_cols(n, s.col_plan) == 0 ||
                         s.C % col_block_lx_cols(n, s.col_plan) != 0)))
        fail(TACAW_E_ARG, "malformed tuning entry");
      ctx->sched[n] = s;
    }
  });
}

int tacaw_autotune(tacaw_ctx* ctx, int32_t n, int32_t n_waves, const char* cache_path,
                   void* stream) {
  return guarded([&] {
    use_device(ctx);
    CallScope scope(ctx);
    if (!grid_size_ok(n)) fail(TACAW_E_SIZE, "grid must be a power of two in [16, 1024], 560 or 1000");
    if (n_waves < 1) fail(TACAW_E_ARG, "n_waves must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    const size_t img = (size_t)n * n;
    const int S = 4;
    float* V = (float*)workspace(ctx, "tune_v", img * S * n_waves * sizeof(float));
    float2* W = (float2*)workspace(ctx, "tune_w", img * n_waves * sizeof(float2));
    hip_check(launch_zero(V, img * S * n_waves * sizeof(float), st), "zero");
    hip_check(launch_zero(W, img * n_waves * sizeof(float2), st), "zero");
    std::vector<double> dz(S, 2.0);
    tacaw_specimen sp{n, n, n * 0.25, n * 0.25, S, dz.data(), 0.0, 2.0 / 3.0};
    tacaw_beam bm{100e3, TACAW_PLANE_WAVE, 0, 0, 0, 1, nullptr};
    tacaw_ms_job job{&sp, &bm, n_waves, V, (tacaw_c64*)W, nullptr};
    MsBuild b = build_ms(ctx, 1, &job, 0, st, false, nullptr, nullptr);
    b.jobs_dev = upload_vec(ctx, b.jobs, st, "jobs");
    const ClassPlan& cp = b.classes[0];
    int2* groups = upload_vec(ctx, cp.groups, st, "groups");
    int4* waves = upload_vec(ctx, cp.waves, st, "waves");
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "hipEventCreate");
    hip_check(hipEventCreate(&e1), "hipEventCreate");
    Launcher L{ctx, st};
    auto time_it = [&](auto&& fn) {
      fn();   // warm-up
      hip_check(hipEventRecord(e0, st), "hipEventRecord");
      for (int r = 0; r < 5; ++r) fn();
      hip_check(hipEventRecord(e1, st), "hipEventRecord");
      hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
      float ms = 0;
      hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
      return ms;
    };
    Sched best = schedule_for(ctx, n);
    float best_row = 1e30f, best_col = 1e30f;
    for (int rp = 0; rp < n_plans(n); ++rp) {
      Sched sc = best;
      sc.row_plan = rp;
      float ms = time_it([&] {
        RowArgs ra{};
        ra.jobs = b.jobs_dev;
        ra.groups = groups;
        ra.n_groups = (int)cp.groups.size();
        ra.s = 1;
        ra.in_buf = BUF_W;
        ra.out_buf = BUF_W;
        ra.stash_slot = -1;
        ra.write_out = 1;
        ra.ny = n;
        ra.single_pos = 1;
        L.row(n, sc, false, ra, (long)cp.waves.size(), n / 2);
      });
      if (std::getenv("TACAW_TUNE_VERBOSE"))
        std::fprintf(stderr, "[tune] n=%d row plan %s: %.3f ms\n", n, plan_name(n, rp), ms / 5);
      if (ms < best_row) { best_row = ms; best.row_plan = rp; }
    }
    for (int cpn = 0; cpn < n_plans(n); ++cpn)
      for (int kind = 0; kind < 3; ++kind)
      for (int pp = 0; pp < (kind == 1 ? 3 : 1); ++pp)
      for (int C = 4; C <= 64; C *= 2) {
        if (C > n || n % C != 0 || !plan_kind_ok(n, cpn, kind)) continue;
        if (pp == 2 && (col_block_lx_cols(n, cpn) == 0 || C % col_block_lx_cols(n, cpn) != 0)) continue;
        const int budget = ctx->max_lds - plan_static_lds(n, cpn);
        if (kind == 0 && col_lds_bytes(n, cpn, C) > budget) continue;
        if (kind == 1 && (C * plan_lanes(n, cpn) > col_block_max_threads(n, cpn) ||
                          col_block_lds_bytes(n, cpn, C, pp) > budget)) continue;
        if (kind == 2 && (col_wave_threads(n, cpn, C) > 1024 ||
                          col_wave_lds_bytes(n, cpn, C) > budget)) continue;
        Sched sc = best;
        sc.col_plan = cpn;
        sc.C = C;
        sc.col_kind = kind;
        sc.pp = pp;
        float ms = time_it([&] {
          ColArgs ca{};
          ca.jobs = b.jobs_dev;
          ca.waves = waves;
          ca.n_waves = (int)cp.waves.size();
          ca.s = 1;
          ca.in_buf = BUF_W;
          ca.out_buf = BUF_W;
          ca.C = C;
          ca.nx = n;
          ca.scale = 1.0f / (float)img;
          L.col(n, sc, true, true, ca, n / 2, true);
        });
        if (std::getenv("TACAW_TUNE_VERBOSE"))
          std::fprintf(stderr, "[tune] n=%d col plan %s kind=%d pp=%d C=%d: %.3f ms\n", n,
                       plan_name(n, cpn), kind, pp, C, ms / 5);
        if (ms < best_col) {
          best_col = ms;
          best.col_plan = cpn;
          best.C = C;
          best.col_kind = kind;
          best.pp = pp;
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->sched[n] = best;
    if (cache_path) {
      std::map<int, Sched> all;
      {
        std::ifstream f(cache_path);
        std::string line;
        while (f && std::getline(f, line)) {
          auto p = line.find("\"n\"");
          if (p == std::string::npos) continue;
          bool ok = true;
          auto num = [&](const char* k) {
            auto q = line.find(std::string("\"") + k + "\"");
            if (q != std::string::npos) q = line.find(':', q);
            if (q == std::string::npos) {
              ok = false;
              return 0;
            }
            return std::atoi(line.c_str() + q + 1);
          };
          Sched s;
          s.row_plan = num("row");
          s.col_plan = num("col");
          s.C = num("C");
          s.col_kind = num("kind");
          s.pp = num("pp");
          const int nn = num("n");
          if (ok) all[nn] = s;   // lines that are not complete entries are dropped
        }
      }
      all[n] = best;
      std::ofstream o(cache_path);
      for (auto& kv : all)
        o << "{\"arch\": \"gfx950\", \"n\": " << kv.first << ", \"row\": " << kv.second.row_plan
          << ", \"col\": " << kv.second.col_plan << ", \"C\": " << kv.second.C
          << ", \"kind\": " << kv.second.col_kind << ", \"pp\": " << kv.second.pp << "}\n";
    }
  });
}

}  // extern "C"
