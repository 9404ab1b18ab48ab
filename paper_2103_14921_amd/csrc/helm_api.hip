// C ABI of the solver: set-up (operator, decomposition, factorisations), the
// batched FGMRES driver and the operator-level entry points.  The host only
// plans and sequences launches; every arithmetic step runs in the kernels of
// ops_operator.hip, ops_local.hip and ops_krylov.hip.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <mutex>
#include <stdexcept>
#include <thread>
#include <vector>

#include "../../include/helm.h"
#include "kernels.h"

struct HelmError : std::runtime_error {
  helm_status code;
  HelmError(helm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

thread_local WorkBound* g_work = nullptr;

namespace {

thread_local std::string g_last_error;

helm_status fail(helm_status c, const std::string& m) {
  g_last_error = m;
  return c;
}

// the message of a failed call on a handle is also kept with the handle
void note_handle_error(helm_handle* H, const std::string& m);
helm_status fail_h(helm_handle* H, helm_status c, const std::string& m) {
  if (H) note_handle_error(H, m);
  return fail(c, m);
}

template <typename F>
helm_status guarded(F&& f, helm_handle* H = nullptr) {
  try {
    return f();
  } catch (const HelmError& e) {
    return fail_h(H, e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail_h(H, HELM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail_h(H, HELM_EDEVICE, e.what());
  }
}

// ---------------------------------------------------------------------------
// Device memory.  Freed blocks go to a process-wide cache and are handed out
// again for requests of the same size class (handles of the same geometry,
// repeated solves); the cache is returned to the runtime when an allocation
// fails.
// ---------------------------------------------------------------------------
}  // namespace

// Stream capture (one outer iteration recorded into a graph) may run on one
// handle's thread while other handles allocate, free, set up or are destroyed
// on theirs.  Device-wide operations (hipMalloc, hipFree), the creation and
// destruction of runtime objects (events, executable graphs) and captures are
// serialised by this lock; everything the library enqueues goes to the
// handles' own non-blocking streams, never to the legacy stream.
std::recursive_mutex& capture_lock() {
  static std::recursive_mutex* m = new std::recursive_mutex();
  return *m;
}
hipError_t locked_event_create(hipEvent_t* e) {
  std::lock_guard<std::recursive_mutex> cl(capture_lock());
  return hipEventCreate(e);
}
void locked_event_destroy(hipEvent_t e) {
  std::lock_guard<std::recursive_mutex> cl(capture_lock());
  (void)hipEventDestroy(e);
}

namespace {

// Streams of handles.  A handle takes a non-blocking stream from this pool at
// set-up and gives it back (idle: the handle synchronised it) when destroyed;
// streams are never destroyed, so evicting a problem while other handles
// capture or trace their iterations touches no stream object.
struct StreamPool {
  std::map<int, std::vector<hipStream_t>> idle;  // per device
  hipStream_t acquire(int dev) {
    std::lock_guard<std::recursive_mutex> cl(capture_lock());
    auto& v = idle[dev];
    if (!v.empty()) {
      hipStream_t s = v.back();
      v.pop_back();
      return s;
    }
    hipStream_t s = nullptr;
    HELM_CHECK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  void release(int dev, hipStream_t s) {
    std::lock_guard<std::recursive_mutex> cl(capture_lock());
    idle[dev].push_back(s);
  }
};
StreamPool& streams() {
  static StreamPool* p = new StreamPool();  // never destroyed: streams live until process exit
  return *p;
}

struct DevicePool {
  std::mutex mu;
  std::multimap<size_t, void*> blocks;
  size_t cached = 0;

  void* get(size_t want, size_t* got) {
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = blocks.lower_bound(want);
      if (it != blocks.end() && it->first <= want + want / 8) {
        void* p = it->second;
        *got = it->first;
        cached -= it->first;
        blocks.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    std::lock_guard<std::recursive_mutex> cl(capture_lock());
    // never take the last free bytes: the runtime allocates for itself at
    // dispatch (kernel arguments, signals, graph instantiation), and a failure
    // there aborts the queue instead of returning an error
    if (free_bytes() < want + headroom_bytes()) {
      trim();
      if (free_bytes() < want + headroom_bytes()) return nullptr;
    }
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      trim();
      if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    *got = want;
    return p;
  }
  static size_t free_bytes() {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      return 0;
    }
    return fr;
  }
  // Device memory left to the runtime: 1% of the device, at least 1 GiB.
  static size_t headroom_bytes() {
    static const size_t h = [] {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) (void)hipGetLastError();
      return std::max<size_t>(size_t(1) << 30, tot / 100);
    }();
    return h;
  }
  void put(void* p, size_t b) {
    std::lock_guard<std::mutex> lk(mu);
    blocks.insert({b, p});
    cached += b;
  }
  // Cached blocks are idle (their owners synchronised before releasing them).
  void trim() {
    std::lock_guard<std::recursive_mutex> cl(capture_lock());
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : blocks) (void)hipFree(kv.second);
    blocks.clear();
    cached = 0;
  }
  size_t cached_bytes() {
    std::lock_guard<std::mutex> lk(mu);
    return cached;
  }
};
DevicePool& pool() {
  static DevicePool* p = new DevicePool();  // never destroyed: blocks live until process exit
  return *p;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) pool().put(p, bytes);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 16;
    b = (b + 255) / 256 * 256;
    p = pool().get(b, &bytes);
    if (!p) throw HelmError(HELM_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed");
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

struct Level {
  int nx = 0, ny = 0, nz = 0;
  long long n = 0;
  std::vector<Sub> subs;
  int nsub = 0, bpmax = 0, maxez = 0;
  long long nodes_total = 0, mat_total = 0, vec_total = 0, maxnodes = 0, maxcore = 0;
  int prec = 0;  // 0 = complex FP64 factors, 1 = complex FP32 factors
  bool half = false;  // approximate local solves: factors kept as complex FP16 (sinv16, sexp) after set-up
  DevBuf d_subs, aloc, sinv, E;
  DevBuf sinv16, sexp;  // [mat_total / 4] 16-byte blocks; [nsub][maxez] scale exponents
  DevBuf cpl;  // plane couplings [node][18] in the factor precision (aloc is set-up only)
};

// Box planning (host): core ranges split each axis into p contiguous ranges of
// floor(n/p) nodes, the first n mod p one longer; the extended box adds
// `overlap` layers on every side that is not a global boundary.
std::vector<std::pair<int, int>> split_axis(int n, int p) {
  std::vector<std::pair<int, int>> out;
  int q = n / p, r = n % p, lo = 0;
  for (int i = 0; i < p; ++i) {
    int sz = q + (i < r ? 1 : 0);
    out.push_back({lo, lo + sz});
    lo += sz;
  }
  return out;
}

int round_up(int a, int m) { return (a + m - 1) / m * m; }

void plan_level(Level& L, int nx, int ny, int nz, const std::vector<Sub>& cores, int delta, int prec) {
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  L.n = (long long)nx * ny * nz;
  L.prec = prec;
  L.subs.clear();
  const int dims[3] = {nx, ny, nz};
  long long node_off = 0, mat_off = 0, vec_off = 0;
  L.bpmax = 0;
  L.maxez = 0;
  L.maxnodes = 0;
  L.maxcore = 0;
  for (const Sub& c : cores) {
    Sub s = c;
    for (int d = 0; d < 3; ++d) {
      s.elo[d] = std::max(0, s.lo[d] - delta);
      s.ehi[d] = std::min(dims[d], s.hi[d] + delta);
    }
    s.ex = s.ehi[0] - s.elo[0];
    s.ey = s.ehi[1] - s.elo[1];
    s.ez = s.ehi[2] - s.elo[2];
    s.b = s.ex * s.ey;
    s.bp = round_up(s.b, 16);
    s.node_off = node_off;
    s.mat_off = mat_off;
    s.vec_off = vec_off;
    const long long nodes = (long long)s.b * s.ez;
    node_off += nodes;
    mat_off += (long long)s.ez * s.bp * s.bp;
    vec_off += (long long)s.ez * s.bp;
    L.bpmax = std::max(L.bpmax, s.bp);
    L.maxez = std::max(L.maxez, s.ez);
    L.maxnodes = std::max(L.maxnodes, nodes);
    L.maxcore = std::max(L.maxcore, (long long)(s.hi[0] - s.lo[0]) * (s.hi[1] - s.lo[1]) * (s.hi[2] - s.lo[2]));
    s.id = (int)L.subs.size();
    L.subs.push_back(s);
  }
  L.nsub = (int)L.subs.size();
  L.nodes_total = node_off;
  L.mat_total = mat_off;
  L.vec_total = vec_off;
}

std::vector<Sub> fine_cores(int nx, int ny, int nz, int px, int py, int pz) {
  auto rx = split_axis(nx, px), ry = split_axis(ny, py), rz = split_axis(nz, pz);
  std::vector<Sub> out;
  for (int kz = 0; kz < pz; ++kz)
    for (int ky = 0; ky < py; ++ky)
      for (int kx = 0; kx < px; ++kx) {
        Sub s{};
        s.lo[0] = rx[kx].first; s.hi[0] = rx[kx].second;
        s.lo[1] = ry[ky].first; s.hi[1] = ry[ky].second;
        s.lo[2] = rz[kz].first; s.hi[2] = rz[kz].second;
        out.push_back(s);
      }
  return out;
}

// coarse core = coarse nodes I whose fine position 2I lies in the fine core
std::vector<Sub> coarse_cores(const std::vector<Sub>& fine) {
  std::vector<Sub> out;
  for (const Sub& f : fine) {
    Sub s{};
    for (int d = 0; d < 3; ++d) {
      s.lo[d] = (f.lo[d] + 1) / 2;
      s.hi[d] = (f.hi[d] + 1) / 2;
    }
    out.push_back(s);
  }
  return out;
}

size_t elem_size(int prec) { return prec ? sizeof(c32) : sizeof(z64); }

// Bytes of the handle's resident data for a level (operators and factors).
size_t level_resident_bytes(const Level& L) {
  return (size_t)L.nodes_total * 18 * elem_size(L.prec) + (size_t)L.mat_total * (L.half ? 4 : elem_size(L.prec)) +
         (size_t)L.nsub * sizeof(Sub) * 2 + (L.half ? (size_t)L.nsub * L.maxez * sizeof(int) : 0);
}
// Temporary set-up bytes of a level (local operator rows, Schur blocks, pivots).
size_t level_setup_bytes(const Level& L) {
  return (size_t)L.nodes_total * 27 * sizeof(z64) + (size_t)L.nsub * L.bpmax * L.bpmax * elem_size(L.prec) * 2 +
         (size_t)L.nsub * (16 + 64) * L.bpmax * elem_size(L.prec) + (size_t)L.nsub * L.bpmax * sizeof(int) * 2 + 64 +
         (L.half ? (size_t)L.mat_total * elem_size(L.prec) : 0);  // complex FP32 factors before conversion
}
size_t level_ws_bytes(const Level& L, int nr) {
  return ((size_t)L.vec_total * nr + (size_t)sweep_tbuf_elems(L.nsub, L.bpmax, nr)) * elem_size(L.prec);
}

}  // namespace

struct KrylovArrays {
  DevBuf Rm, g, cs, sn, y, h, h2, nrm2, w0, w1, bnorm, beta, est, fac, it, kc, active, done, conv, counter, skip,
      extra;
  KrylovState st{};
  void alloc(int m, int nr) {
    Rm.alloc(sizeof(z64) * (size_t)(m + 1) * m * nr);
    g.alloc(sizeof(z64) * (size_t)(m + 1) * nr);
    cs.alloc(sizeof(double) * (size_t)m * nr);
    sn.alloc(sizeof(z64) * (size_t)m * nr);
    y.alloc(sizeof(z64) * (size_t)m * nr);
    h.alloc(sizeof(z64) * (size_t)(m + 1) * nr);
    h2.alloc(sizeof(z64) * (size_t)(m + 1) * nr);
    for (DevBuf* b : {&nrm2, &w0, &w1, &bnorm, &beta, &est, &fac}) b->alloc(sizeof(double) * nr);
    skip.alloc(sizeof(int));
    extra.alloc(sizeof(double));
    for (DevBuf* b : {&it, &kc, &active, &done, &conv}) b->alloc(sizeof(int) * nr);
    counter.alloc(sizeof(int) * 4);
    st.m = m;
    st.nrhs = nr;
    st.Rm = Rm.as<z64>();
    st.g = g.as<z64>();
    st.cs = cs.as<double>();
    st.sn = sn.as<z64>();
    st.y = y.as<z64>();
    st.h = h.as<z64>();
    st.h2 = h2.as<z64>();
    st.nrm2 = nrm2.as<double>();
    st.w0 = w0.as<double>();
    st.bnorm = bnorm.as<double>();
    st.beta = beta.as<double>();
    st.est = est.as<double>();
    st.fac = fac.as<double>();
    st.it = it.as<int>();
    st.kc = kc.as<int>();
    st.active = active.as<int>();
    st.done = done.as<int>();
    st.conv = conv.as<int>();
    st.counter = counter.as<int>();
    st.w1 = w1.as<double>();
    st.skip = skip.as<int>();
    st.extra = extra.as<double>();
  }
  static size_t bytes(int m, int nr) {
    return sizeof(z64) * (size_t)nr * ((size_t)(m + 1) * m + 3 * (m + 1) + 2 * m) + sizeof(double) * (size_t)nr * (m + 7) +
           sizeof(int) * (5 * (size_t)nr + 4) + 23 * 256;
  }
};

struct Workspace {
  int nr = 0;
  DevBuf b, x, w, V, Zv, q, t, cc, Vc, Zc, wc, ec, yl_f, tb_f, yl_c, tb_c, zpart, dpart, bn2, beta2, cols;
  DevBuf bpart, bcoef;  // block FGMRES: block-dot partial sums, coefficient blocks [m + 1][32][32]
  KrylovArrays ko, kc;
};

// Launches timed live when sweep timing is on: 0 fine sweep, 1 coarse sweep,
// 2 fine product y = A x, 3 fine residual y = b - A x.
constexpr int NTIMED = 4;

// One outer FGMRES iteration (preconditioner, operator, Arnoldi step) captured
// as an executable HIP graph.  Kernel arguments are baked in, so an entry is
// valid for one iteration index, batch width, tolerance, iteration limit and
// workspace generation.  With sweep timing on, the sweeps are bracketed by
// external event nodes whose times are harvested at the next host sync.
struct Captured {
  int j = 0, nr = 0, maxit = 0, policy = 0;
  double tol = 0;
  unsigned gen = 0;
  bool timed = false;
  hipGraphExec_t exec = nullptr;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[NTIMED];
  std::vector<double> fl[NTIMED], by[NTIMED];
  bool pending = false;  // replayed with timing, events not yet read
  WorkBound work;        // algorithmic work of one replay

  ~Captured() {
    std::lock_guard<std::recursive_mutex> cl(capture_lock());
    if (exec) (void)hipGraphExecDestroy(exec);
    for (int lv = 0; lv < NTIMED; ++lv)
      for (auto& e : ev[lv]) {
        locked_event_destroy(e.first);
        locked_event_destroy(e.second);
      }
  }
};

struct helm_handle {
  int device = 0;
  hipStream_t own = nullptr, stream = nullptr;
  int nx = 0, ny = 0, nz = 0;
  long long n = 0;
  double h = 0, freq = 0, omega = 0;
  helm_pml_t pml{};
  helm_weights_t w{};
  helm_decomp_t dec{};
  DevBuf c, sigma, diag, xi_int, xi_half, i2_int, i2_half, flat, vmax, err;
  DevBuf wtab, wnode;  // adaptive coefficients: weight table [n][7], per-node weights [n][8]
  OpDev op{};
  Level fine, coarse;
  Workspace ws;
  double t_setup = 0, t_solve = 0, t_fact = 0, t_coarse = 0, its = 0;
  // live timing of the local-solve sweeps (HIP events around each launch, per level)
  bool timing = false;
  // (slots: 0 fine sweep, 1 coarse sweep, 2 fine product A x, 3 fine residual b - A x)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> sweep_ev[NTIMED];
  std::vector<double> sweep_flops[NTIMED], sweep_bytes[NTIMED];
  double sweep_stat[NTIMED][4] = {};  // launches, ms, flops, bytes
  // captured outer iterations
  bool graphs = true;
  bool graph_timing = true;  // event-record nodes accepted inside captured graphs
  unsigned ws_gen = 0;  // bumped whenever workspace buffers move
  std::vector<std::unique_ptr<Captured>> captured;
  Captured* capturing = nullptr;
  double graph_stat[2] = {0, 0};  // captures, replays
  WorkBound work_solve;           // lower bound of the last solve
  // the asynchronous solve in flight, if any (helm_solve_async)
  helm_request* pending = nullptr;
  std::mutex pending_mu;
  // message of the last failed call on this handle (helm_last_error(h))
  std::string err_msg;
  mutable std::mutex err_mu;

  ~helm_handle() {
    captured.clear();
    if (own) {
      (void)hipStreamSynchronize(own);
      streams().release(device, own);
    }
  }
  bool two_level() const { return dec.levels == 2; }
};

namespace {

void note_handle_error(helm_handle* H, const std::string& m) {
  std::lock_guard<std::mutex> lk(H->err_mu);
  H->err_msg = m;
}

void fit_weights_host(double gmin, double gmax, int ng, int nang, helm_weights_t* out) {
  // unknowns p = (w2, w3, wm2, wm3, wm4); w1 = 1 - w2 - w3, wm1 = 1 - 6wm2 - 12wm3 - 8wm4
  static const int dirs[13][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1},
                                  {0, 1, 1}, {0, 1, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
  // least squares by Householder QR of the tall system (rows x 5)
  std::vector<std::array<double, 5>> J;
  std::vector<double> rv;
  const double pi = 3.14159265358979323846;
  for (int ig = 0; ig < ng; ++ig) {
    const double G = ng == 1 ? gmin : gmin + (gmax - gmin) * ig / (ng - 1);
    const double kh = 2.0 * pi / G;
    for (int it = 0; it < nang; ++it) {
      const double th = nang == 1 ? 0.0 : 0.5 * pi * it / (nang - 1);
      for (int ip = 0; ip < nang; ++ip) {
        const double ph = nang == 1 ? 0.0 : 0.5 * pi * ip / (nang - 1);
        const double nv[3] = {std::sin(th) * std::cos(ph), std::sin(th) * std::sin(ph), std::cos(th)};
        double st[3] = {0, 0, 0}, cm[3] = {0, 0, 0};
        for (int e = 0; e < 13; ++e) {
          const int cls = e < 3 ? 0 : (e < 9 ? 1 : 2);
          const double ph2 = kh * (nv[0] * dirs[e][0] + nv[1] * dirs[e][1] + nv[2] * dirs[e][2]);
          st[cls] += 2.0 * (1.0 - std::cos(ph2));
          cm[cls] += 2.0 * std::cos(ph2);
        }
        for (int c = 0; c < 3; ++c) st[c] /= kh * kh;
        J.push_back({(-1.0 + 1.0 / 3.0) * st[0] + st[1] / 6.0, -st[0] + st[2] / 4.0, -(cm[0] - 6.0),
                     -(cm[1] - 12.0), -(cm[2] - 8.0)});
        rv.push_back(-(st[0] - 1.0));
      }
    }
  }
  const size_t M = J.size();
  if (M < 5) throw HelmError(HELM_EINVAL, "too few samples for the weight fit");
  for (int k = 0; k < 5; ++k) {
    double nrm = 0.0;
    for (size_t i = k; i < M; ++i) nrm += J[i][k] * J[i][k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) throw HelmError(HELM_EINVAL, "singular weight fit");
    const double alpha = J[k][k] > 0 ? -nrm : nrm;
    std::vector<double> v(M - k);
    for (size_t i = k; i < M; ++i) v[i - k] = J[i][k];
    v[0] -= alpha;
    double vv = 0.0;
    for (double x : v) vv += x * x;
    for (int c = k; c < 5; ++c) {
      double d = 0.0;
      for (size_t i = k; i < M; ++i) d += v[i - k] * J[i][c];
      d = 2.0 * d / vv;
      for (size_t i = k; i < M; ++i) J[i][c] -= d * v[i - k];
    }
    double d = 0.0;
    for (size_t i = k; i < M; ++i) d += v[i - k] * rv[i];
    d = 2.0 * d / vv;
    for (size_t i = k; i < M; ++i) rv[i] -= d * v[i - k];
  }
  double p[5];
  for (int i = 4; i >= 0; --i) {
    double s2 = rv[i];
    for (int j = i + 1; j < 5; ++j) s2 -= J[i][j] * p[j];
    p[i] = s2 / J[i][i];
  }
  out->w2 = p[0];
  out->w3 = p[1];
  out->w1 = 1.0 - p[0] - p[1];
  out->wm2 = p[2];
  out->wm3 = p[3];
  out->wm4 = p[4];
  out->wm1 = 1.0 - 6.0 * p[2] - 12.0 * p[3] - 8.0 * p[4];
}

// The adaptive coefficients' table (helm_fit_weight_table).
constexpr double ADAPT_G0 = 3.0, ADAPT_DG = 0.25;
constexpr int ADAPT_N = 29, ADAPT_NANG = 15;

void fit_weight_table_host(double g0, double dg, int n, int nang, helm_weights_t* out) {
  for (int j = 0; j < n; ++j) {
    const double G = g0 + j * dg;
    fit_weights_host(G / 1.05, G * 1.05, 3, nang, out + j);
  }
}

size_t budget_bytes() {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
    (void)hipGetLastError();
    fr = 0;
  }
  const size_t avail = fr + pool().cached_bytes();
  const size_t head = DevicePool::headroom_bytes();
  size_t b = avail > head ? (size_t)((avail - head) * 0.92) : 0;
  if (const char* e = std::getenv("HELM_MEM_BUDGET")) {
    const size_t v = (size_t)std::strtoull(e, nullptr, 10);
    if (v > 0) b = std::min(b, v);
  }
  return b;
}

void validate(const helm_grid_t* g, const helm_pml_t* pml, const helm_decomp_t* d) {
  if (!g || !pml || !d) throw HelmError(HELM_EINVAL, "null argument");
  if (g->nx < 3 || g->ny < 3 || g->nz < 3) throw HelmError(HELM_EINVAL, "grid must have at least 3 nodes per axis");
  if (!(g->h > 0) || !std::isfinite(g->h)) throw HelmError(HELM_EINVAL, "h must be positive");
  if (pml->npml_x < 0 || pml->npml_y < 0 || pml->npml_zbot < 0 || pml->npml_ztop < 0 ||
      2 * pml->npml_x >= g->nx || 2 * pml->npml_y >= g->ny || pml->npml_zbot + pml->npml_ztop >= g->nz)
    throw HelmError(HELM_EINVAL, "PML thicker than the grid");
  if (d->px < 1 || d->py < 1 || d->pz < 1) throw HelmError(HELM_EINVAL, "subdomain counts must be >= 1");
  if (d->overlap < 1) throw HelmError(HELM_EINVAL, "overlap must be >= 1");
  if (d->levels != 1 && d->levels != 2) throw HelmError(HELM_EINVAL, "levels must be 1 or 2");
  if (d->levels == 2 && d->coarse_iters < 1) throw HelmError(HELM_EINVAL, "coarse_iters must be >= 1");
  if (d->adaptive != 0 && d->adaptive != 1) throw HelmError(HELM_EINVAL, "adaptive must be 0 or 1");
  if (d->restart < 1 || d->restart > 64) throw HelmError(HELM_EINVAL, "restart must be in [1, 64]");
  if (d->precision != HELM_FP64 && d->precision != HELM_MIXED && d->precision != HELM_SINGLE_LOCAL &&
      d->precision != HELM_APPROX_LOCAL)
    throw HelmError(HELM_EINVAL, "bad precision");
  const int n[3] = {g->nx, g->ny, g->nz}, p[3] = {d->px, d->py, d->pz};
  for (int a = 0; a < 3; ++a) {
    if (p[a] > 1 && n[a] / p[a] < 2 * d->overlap + 1)
      throw HelmError(HELM_EINVAL, "decomposition finer than 2*overlap+1 nodes per box");
  }
}

// largest plane the factorisation kernels accept
constexpr int MAX_PLANE = 2048;

void plan(helm_handle* H) {
  const helm_decomp_t& d = H->dec;
  auto cores = fine_cores(H->nx, H->ny, H->nz, d.px, d.py, d.pz);
  plan_level(H->fine, H->nx, H->ny, H->nz, cores, d.overlap, d.precision != HELM_FP64 ? 1 : 0);
  if (H->fine.bpmax > MAX_PLANE) throw HelmError(HELM_EINVAL, "subdomain plane larger than 2048 nodes");
  H->fine.half = d.precision == HELM_APPROX_LOCAL;
  if (H->fine.half && half_group(H->fine.bpmax, 1) == 0)
    throw HelmError(HELM_EINVAL, "approximate local solves need subdomain planes of at most 960 nodes");
  if (H->two_level()) {
    plan_level(H->coarse, (H->nx + 1) / 2, (H->ny + 1) / 2, (H->nz + 1) / 2, coarse_cores(H->fine.subs), d.overlap,
               d.precision == HELM_SINGLE_LOCAL ? 1 : 0);
    if (H->coarse.bpmax > MAX_PLANE) throw HelmError(HELM_EINVAL, "coarse subdomain plane too large");
  }
}

size_t ws_bytes(const helm_handle* H, int nr) {
  const int m = H->dec.restart;
  size_t b = sizeof(z64) * (size_t)H->n * nr * (3 + (m + 1) + m);
  b += sizeof(z64) * 1024 * (size_t)(m + 1) * (block_chunks(H->n) + 1);  // block FGMRES
  b += level_ws_bytes(H->fine, nr);
  b += KrylovArrays::bytes(m, nr);
  b += sizeof(z64) * RED_BLOCKS * 32 * (size_t)nr + sizeof(double) * RED_BLOCKS * (size_t)nr + 2 * sizeof(double) * nr;
  if (H->two_level()) {
    const int ci = H->dec.coarse_iters;
    const size_t nc = (size_t)H->coarse.n;
    b += sizeof(z64) * (size_t)H->n * nr * 2;
    b += sizeof(z64) * nc * nr * (3 + (ci + 1) + ci);
    b += level_ws_bytes(H->coarse, nr);
    b += KrylovArrays::bytes(ci, nr);
  }
  return b;
}

size_t resident_bytes_planned(const helm_handle* H) {
  size_t b = sizeof(z64) * (size_t)H->n * 3 + level_resident_bytes(H->fine);  // velocity, sigma, row diagonals
  if (H->dec.adaptive) b += sizeof(double) * 8 * (size_t)H->n + sizeof(double) * 7 * ADAPT_N;
  if (H->two_level()) b += level_resident_bytes(H->coarse) + sizeof(z64) * (size_t)H->coarse.n * 27;
  return b;
}

// Fold the sweep times of replayed graphs into the statistics (the stream has
// been synchronised since the replay).
void harvest_graphs(helm_handle* H) {
  for (auto& c : H->captured) {
    if (!c->pending) continue;
    for (int lv = 0; lv < NTIMED; ++lv)
      for (size_t i = 0; i < c->ev[lv].size(); ++i) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, c->ev[lv][i].first, c->ev[lv][i].second);
        H->sweep_stat[lv][0] += 1;
        H->sweep_stat[lv][1] += ms;
        H->sweep_stat[lv][2] += c->fl[lv][i];
        H->sweep_stat[lv][3] += c->by[lv][i];
      }
    c->pending = false;
  }
}

// Forget every captured iteration (their arguments point into workspace that is
// about to move or be released).
void drop_graphs(helm_handle* H) {
  if (H->captured.empty()) return;
  (void)hipStreamSynchronize(H->stream);
  harvest_graphs(H);
  H->captured.clear();
}

// Batch size of the next launches (the arrays hold at least W.nr columns).
void set_batch(helm_handle* H, int nr) {
  H->ws.ko.st.nrhs = nr;
  H->ws.kc.st.nrhs = nr;
}

void ensure_ws(helm_handle* H, int nr) {
  Workspace& W = H->ws;
  if (W.nr >= nr) {
    set_batch(H, nr);
    return;
  }
  drop_graphs(H);
  ++H->ws_gen;
  W.nr = 0;
  const int m = H->dec.restart;
  const size_t vec = sizeof(z64) * (size_t)H->n * nr;
  W.b.alloc(vec);
  W.x.alloc(vec);
  W.w.alloc(vec);
  W.V.alloc(vec * (m + 1));
  W.Zv.alloc(vec * m);
  W.yl_f.alloc((size_t)H->fine.vec_total * nr * elem_size(H->fine.prec));
  W.tb_f.alloc((size_t)sweep_tbuf_elems(H->fine.nsub, H->fine.bpmax, nr) * elem_size(H->fine.prec));
  W.zpart.alloc(sizeof(z64) * RED_BLOCKS * 32 * (size_t)nr);
  W.dpart.alloc(sizeof(double) * RED_BLOCKS * (size_t)nr);
  W.bn2.alloc(sizeof(double) * nr);
  W.beta2.alloc(sizeof(double) * nr);
  W.cols.alloc(sizeof(int) * nr);
  W.bpart.alloc(sizeof(z64) * 1024 * (size_t)(m + 1) * block_chunks(H->n));
  W.bcoef.alloc(sizeof(z64) * 1024 * (size_t)(m + 1));
  W.ko.alloc(m, nr);
  if (H->two_level()) {
    const int ci = H->dec.coarse_iters;
    const size_t cvec = sizeof(z64) * (size_t)H->coarse.n * nr;
    W.q.alloc(vec);
    W.t.alloc(vec);
    W.cc.alloc(cvec);
    W.wc.alloc(cvec);
    W.ec.alloc(cvec);
    W.Vc.alloc(cvec * (ci + 1));
    W.Zc.alloc(cvec * ci);
    W.yl_c.alloc((size_t)H->coarse.vec_total * nr * elem_size(H->coarse.prec));
    W.tb_c.alloc((size_t)sweep_tbuf_elems(H->coarse.nsub, H->coarse.bpmax, nr) * elem_size(H->coarse.prec));
    W.kc.alloc(ci, nr);
  }
  W.nr = nr;
  set_batch(H, nr);
}

// ---------------------------------------------------------------------------
// Building blocks of one preconditioner application.
// ---------------------------------------------------------------------------
void oras_sweep(helm_handle* H, Level& L, int nr, const z64* u, z64* z, const z64* add, void* yl, void* tb);

// Algorithmic work of one batched local-solve launch: every plane product
// Sinv_k T (ez forward + ez-1 backward per box) costs 8 b^2 real flops per
// right-hand side; the bytes count each factor once per application (the
// implementation reads it once per plane product and right-hand-side group:
// that excess is what measured traffic shows) plus the plane vectors (gather,
// scatter, stored planes).
void sweep_work(const helm_handle* H, const Level& L, int nr, double* flops, double* bytes) {
  const int es = (int)elem_size(L.prec);          // plane vectors
  const int fs = L.half ? 4 : es;                 // factor entries
  double f = 0, by = 0;
  for (const Sub& sb : L.subs) {
    const double planes = 2.0 * sb.ez - 1.0;
    const double b = sb.b;
    f += planes * 8.0 * b * b * nr;
    by += (double)sb.ez * b * b * fs;                         // factors, once per application
    by += (double)sb.b * sb.ez * nr * (16.0 + 3.0 * es);      // gather + stored planes (w, r, w)
    by += (double)(sb.hi[0] - sb.lo[0]) * (sb.hi[1] - sb.lo[1]) * (sb.hi[2] - sb.lo[2]) * nr * 16.0;  // scatter
  }
  *flops = f;
  *bytes = by;
}

// Record a timing event on the handle's stream; while the stream is being
// captured, as an event-record node appended to the captured graph.
void record_timing_event(helm_handle* H, hipEvent_t e) {
  if (!H->capturing) {
    HELM_CHECK_HIP(hipEventRecord(e, H->stream));
    return;
  }
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  unsigned long long id = 0;
  hipGraph_t g = nullptr;
  const hipGraphNode_t* deps = nullptr;
  size_t nd = 0;
  HELM_CHECK_HIP(hipStreamGetCaptureInfo_v2(H->stream, &st, &id, &g, &deps, &nd));
  hipGraphNode_t node = nullptr;
  HELM_CHECK_HIP(hipGraphAddEventRecordNode(&node, g, deps, nd, e));
  HELM_CHECK_HIP(hipStreamUpdateCaptureDependencies(H->stream, &node, 1, hipStreamSetCaptureDependencies));
}

void oras_apply(helm_handle* H, Level& L, int nr, const z64* u, z64* z, const z64* add, void* yl, void* tb) {
  const int lv = &L == &H->fine ? 0 : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (H->timing) {
    HELM_CHECK_HIP(locked_event_create(&e0));
    HELM_CHECK_HIP(locked_event_create(&e1));
    record_timing_event(H, e0);
  }
  oras_sweep(H, L, nr, u, z, add, yl, tb);
  if (g_work) {
    double f, by;
    sweep_work(H, L, nr, &f, &by);
    account(by, f, L.half ? FP16_PEAK : (L.prec ? FP32_PEAK : FP64_PEAK));
  }
  if (H->timing) {
    record_timing_event(H, e1);
    double f, by;
    sweep_work(H, L, nr, &f, &by);
    auto& ev = H->capturing ? H->capturing->ev[lv] : H->sweep_ev[lv];
    auto& fl = H->capturing ? H->capturing->fl[lv] : H->sweep_flops[lv];
    auto& bb = H->capturing ? H->capturing->by[lv] : H->sweep_bytes[lv];
    ev.push_back({e0, e1});
    fl.push_back(f);
    bb.push_back(by);
  }
}

// The fine 27-point product y = A x, or y = b - A x when b is given; with
// timing on, bracketed by events like the sweeps (slot 2 or 3) with its
// algorithmic work: x read and y written once, b read once for a residual,
// s k^2 once per node; 27 complex multiply-adds per node and right-hand side.
void fine_product(helm_handle* H, int nr, const z64* b, const z64* x, z64* y) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (H->timing) {
    HELM_CHECK_HIP(locked_event_create(&e0));
    HELM_CHECK_HIP(locked_event_create(&e1));
    record_timing_event(H, e0);
  }
  if (b)
    launch_residual(H->op, nr, b, x, y, H->stream);
  else
    launch_stencil(H->op, nr, x, y, H->stream);
  if (H->timing) {
    record_timing_event(H, e1);
    const int slot = b ? 3 : 2;
    const double n = (double)H->n;
    auto& ev = H->capturing ? H->capturing->ev[slot] : H->sweep_ev[slot];
    auto& fl = H->capturing ? H->capturing->fl[slot] : H->sweep_flops[slot];
    auto& bb = H->capturing ? H->capturing->by[slot] : H->sweep_bytes[slot];
    ev.push_back({e0, e1});
    fl.push_back(216.0 * n * nr);
    bb.push_back(16.0 * n * nr * (b ? 3 : 2) + 16.0 * n);
  }
}

// Fold the recorded sweep events into the statistics (the stream has been synchronised).
void collect_sweep_timing(helm_handle* H) {
  for (int lv = 0; lv < NTIMED; ++lv) {
    for (size_t i = 0; i < H->sweep_ev[lv].size(); ++i) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, H->sweep_ev[lv][i].first, H->sweep_ev[lv][i].second);
      H->sweep_stat[lv][0] += 1;
      H->sweep_stat[lv][1] += ms;
      H->sweep_stat[lv][2] += H->sweep_flops[lv][i];
      H->sweep_stat[lv][3] += H->sweep_bytes[lv][i];
      locked_event_destroy(H->sweep_ev[lv][i].first);
      locked_event_destroy(H->sweep_ev[lv][i].second);
    }
    H->sweep_ev[lv].clear();
    H->sweep_flops[lv].clear();
    H->sweep_bytes[lv].clear();
  }
}

void oras_sweep(helm_handle* H, Level& L, int nr, const z64* u, z64* z, const z64* add, void* yl, void* tb) {
  const Sub* order = L.d_subs.as<Sub>() + L.nsub;  // the boxes in sweep launch order
  if (L.half) {
    if (!oras_half(order, L.nsub, L.bpmax, L.cpl.as<c32>(), L.sinv16.as<uint4>(), L.sexp.as<int>(),
                   L.maxez, nr, u, z, add, L.nx, L.ny, (c32*)yl, H->stream))
      throw HelmError(HELM_EINVAL, "approximate local solves do not fit this plane size");
    return;
  }
  if (L.prec == 1)
    Factor<float>::sweep(order, L.nsub, L.bpmax, L.maxez, L.cpl.as<c32>(), L.sinv.as<c32>(), nr, u, z, add, L.nx, L.ny,
                         (c32*)yl, (c32*)tb, H->stream);
  else
    Factor<double>::sweep(order, L.nsub, L.bpmax, L.maxez, L.cpl.as<z64>(), L.sinv.as<z64>(), nr, u, z, add, L.nx,
                          L.ny, (z64*)yl, (z64*)tb, H->stream);
}

void coarse_spmv(helm_handle* H, int nr, const z64* x, z64* y) {
  launch_coarse_spmv(H->coarse.nx, H->coarse.ny, H->coarse.nz, H->coarse.E.as<z64>(), nr, x, y, H->stream);
}

// One Arnoldi step with CGS2 on vectors of length len: w is orthogonalised
// against V_0..V_j; then the Givens kernel updates the least-squares problem.
void arnoldi_step(helm_handle* H, KrylovArrays& K, int j, const z64* V, z64* w, long long len, int nr, double tol,
                  int maxit, int fixed) {
  Workspace& W = H->ws;
  const long long vs = len * nr;
  // first Gram-Schmidt projections, with ||w||^2 (for the breakdown test) from the same read of w
  launch_dots(V, vs, j + 1, w, len, nr, W.zpart.as<z64>(), K.h.as<z64>(), H->stream, W.dpart.as<double>(),
              K.w0.as<double>());
  // first update w' = w - V h1 with the second projections h2 = V^T w' and ||w'||^2 in the same pass
  if (!launch_axpy_dots(V, vs, j + 1, K.h.as<z64>(), w, len, nr, W.zpart.as<z64>(), K.h2.as<z64>(), H->stream,
                        W.dpart.as<double>(), K.w1.as<double>())) {
    launch_axpy_multi(V, vs, j + 1, K.h.as<z64>(), w, len, nr, W.dpart.as<double>(), K.w1.as<double>(), H->stream);
    launch_dots(V, vs, j + 1, w, len, nr, W.zpart.as<z64>(), K.h2.as<z64>(), H->stream);
  }
  // second update only where it matters (selective reorthogonalisation): skipped for the batch when
  // ||h2|| <= 1e-12 ||w'|| for every right-hand side, decided on the device
  static const double tau2 = std::getenv("HELM_FULL_CGS2") ? -1.0 : 1e-24;
  launch_reorth_check(K.st, j + 1, tau2, 16.0 * (double)len * nr, H->stream);
  launch_axpy_multi(V, vs, j + 1, K.h2.as<z64>(), w, len, nr, W.dpart.as<double>(), K.nrm2.as<double>(), H->stream,
                    K.skip.as<int>());
  launch_givens(K.st, j, tol, maxit, fixed, H->stream);
}

// e = GMRES_{ci}(E, c), right-preconditioned by the coarse one-level ORAS, x0 = 0.
void coarse_solve(helm_handle* H, int nr, const z64* c, z64* e) {
  Workspace& W = H->ws;
  KrylovArrays& K = W.kc;
  const long long nc = H->coarse.n;
  const long long vs = nc * nr;
  const int ci = H->dec.coarse_iters;
  launch_norm2(c, nc, nr, W.dpart.as<double>(), W.beta2.as<double>(), H->stream);
  launch_cycle_start_fixed(K.st, W.beta2.as<double>(), H->stream);
  launch_scale(c, K.fac.as<double>(), W.Vc.as<z64>(), nc, nr, H->stream);
  for (int j = 0; j < ci; ++j) {
    z64* vj = W.Vc.as<z64>() + j * vs;
    z64* zj = W.Zc.as<z64>() + j * vs;
    oras_apply(H, H->coarse, nr, vj, zj, nullptr, W.yl_c.p, W.tb_c.p);
    coarse_spmv(H, nr, zj, W.wc.as<z64>());
    arnoldi_step(H, K, j, W.Vc.as<z64>(), W.wc.as<z64>(), nc, nr, 0.0, 1 << 30, 1);
    if (j + 1 < ci) launch_scale(W.wc.as<z64>(), K.fac.as<double>(), W.Vc.as<z64>() + (j + 1) * vs, nc, nr, H->stream);
  }
  launch_backsolve(K.st, H->stream);
  launch_fill(e, vs, H->stream);
  launch_update(W.Zc.as<z64>(), vs, ci, K.y.as<z64>(), e, nc, nr, H->stream);
}

// q = Z GMRES(E, Z^T r)
void coarse_correction(helm_handle* H, int nr, const z64* r, z64* q) {
  Workspace& W = H->ws;
  launch_restrict(H->nx, H->ny, H->nz, nr, r, W.cc.as<z64>(), H->stream);
  coarse_solve(H, nr, W.cc.as<z64>(), W.ec.as<z64>());
  launch_prolong(H->nx, H->ny, H->nz, nr, W.ec.as<z64>(), q, H->stream);
}

// z = M^{-1} v (eq. oras or eq. 2lvl)
void precond(helm_handle* H, int nr, const z64* v, z64* z) {
  Workspace& W = H->ws;
  if (!H->two_level()) {
    oras_apply(H, H->fine, nr, v, z, nullptr, W.yl_f.p, W.tb_f.p);
    return;
  }
  coarse_correction(H, nr, v, W.q.as<z64>());
  fine_product(H, nr, v, W.q.as<z64>(), W.t.as<z64>());  // t = v - A q
  oras_apply(H, H->fine, nr, W.t.as<z64>(), z, W.q.as<z64>(), W.yl_f.p, W.tb_f.p);
}

int read_counter(helm_handle* H, KrylovArrays& K) {
  int v = 0;
  HELM_CHECK_HIP(hipMemcpyAsync(&v, K.counter.p, sizeof(int), hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  harvest_graphs(H);
  return v;
}
void zero_counter(helm_handle* H, KrylovArrays& K) {
  // a fill kernel rather than a memset, so that the sequence stays capturable
  launch_fill(K.counter.as<z64>(), 1, H->stream);
}

// Outer iteration j: z_j = M^{-1} v_j, w = A z_j, Arnoldi step on w (CGS2,
// Givens, convergence count).  No host synchronisation inside, so it can be
// captured.
void outer_step(helm_handle* H, int nr, int j, double tol, int maxit) {
  Workspace& W = H->ws;
  const long long vs = H->n * nr;
  z64* vj = W.V.as<z64>() + j * vs;
  z64* zj = W.Zv.as<z64>() + j * vs;
  precond(H, nr, vj, zj);
  fine_product(H, nr, nullptr, zj, W.w.as<z64>());
  zero_counter(H, W.ko);
  arnoldi_step(H, W.ko, j, W.V.as<z64>(), W.w.as<z64>(), H->n, nr, tol, maxit, 0);
}

// Whether the next sweep of level L on nr right-hand sides would still run the
// group-size tuner (which synchronises, so it must not be captured).
bool sweep_untuned(const Level& L, int nr) {
  static const bool no_tune = std::getenv("HELM_NO_TUNE") != nullptr || std::getenv("HELM_NO_FUSED") != nullptr;
  if (no_tune) return false;
  return tuned_group(L.half ? 2 : (int)elem_size(L.prec) / 2, L.bpmax, L.nsub, nr, L.nx, L.ny) == 0;
}

// Run outer iteration j from its captured graph, capturing it first if needed.
// Falls back to direct launches while a sweep or a row-tiled product is
// untuned, and for good if the runtime refuses capture.
void run_outer_step(helm_handle* H, int nr, int j, double tol, int maxit) {
  if (!H->graphs || (H->timing && !H->graph_timing) || sweep_untuned(H->fine, nr) ||
      (H->two_level() && sweep_untuned(H->coarse, nr)) || stencil_untuned(H->op, nr) ||
      (H->two_level() && coarse_spmv_untuned(H->coarse.nx, H->coarse.ny, H->coarse.nz, nr))) {
    outer_step(H, nr, j, tol, maxit);
    return;
  }
  Captured* c = nullptr;
  for (auto& e : H->captured)
    if (e->j == j && e->nr == nr && e->maxit == maxit && e->tol == tol && e->gen == H->ws_gen &&
        e->timed == H->timing && e->policy == sweep_policy()) {
      c = e.get();
      break;
    }
  if (!c) {
    auto e = std::make_unique<Captured>();
    e->j = j;
    e->nr = nr;
    e->maxit = maxit;
    e->tol = tol;
    e->gen = H->ws_gen;
    e->timed = H->timing;
    e->policy = sweep_policy();
    std::lock_guard<std::recursive_mutex> cl(capture_lock());
    const hipError_t be = hipStreamBeginCapture(H->stream, hipStreamCaptureModeRelaxed);
    if (be != hipSuccess) {
      (void)hipGetLastError();
      std::fprintf(stderr, "helm: stream capture unavailable (%s); launching directly\n", hipGetErrorString(be));
      H->graphs = false;
      outer_step(H, nr, j, tol, maxit);
      return;
    }
    H->capturing = e.get();
    hipGraph_t g = nullptr;
    WorkBound* const outer_work = g_work;
    g_work = outer_work ? &e->work : nullptr;  // one replay's work; added per launch below
    try {
      outer_step(H, nr, j, tol, maxit);
      g_work = outer_work;
    } catch (const HelmError& err) {
      g_work = outer_work;
      H->capturing = nullptr;
      if (hipStreamEndCapture(H->stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      if (!H->timing) throw;
      // event nodes refused by the runtime: time the sweeps with direct launches
      (void)hipGetLastError();
      std::fprintf(stderr, "helm: no timing events inside graphs (%s); timed iterations launch directly\n", err.what());
      H->graph_timing = false;
      outer_step(H, nr, j, tol, maxit);
      return;
    } catch (...) {
      g_work = outer_work;
      H->capturing = nullptr;
      if (hipStreamEndCapture(H->stream, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
      throw;
    }
    H->capturing = nullptr;
    hipError_t ce = hipStreamEndCapture(H->stream, &g);
    if (ce == hipSuccess && !g) ce = hipErrorInvalidValue;
    if (ce == hipSuccess) ce = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (ce != hipSuccess) {
      // nothing captured has run: do the iteration directly, and stop capturing
      (void)hipGetLastError();
      std::fprintf(stderr, "helm: graph capture failed (%s); launching directly\n", hipGetErrorString(ce));
      H->graphs = false;
      outer_step(H, nr, j, tol, maxit);
      return;
    }
    H->graph_stat[0] += 1;
    c = e.get();
    H->captured.push_back(std::move(e));
  }
  if (c->pending) {  // replayed twice without a sync in between: read the first replay's times
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    harvest_graphs(H);
  }
  HELM_CHECK_HIP(hipGraphLaunch(c->exec, H->stream));
  c->pending = c->timed;
  H->graph_stat[1] += 1;
  if (g_work) g_work->add(c->work);
}

// Batched FGMRES on W.nr right-hand sides held node-major in W.b / W.x.
// Per-RHS results of a batch column, reported under its index in the chunk.
struct ChunkOut {
  std::vector<int> it, conv;
  std::vector<double> est, tru;
};

// Hand finished columns `cols` of the current batch (width nr, column c holds
// the chunk's right-hand side orig[c]) to the caller: per-RHS results into out,
// solutions field-major into X (chunk offset r0).  The basis storage V is free
// here and serves as staging.
void emit_columns(helm_handle* H, int nr, const std::vector<int>& orig, const std::vector<int>& cols, void* X,
                  int r0, ChunkOut& out) {
  Workspace& W = H->ws;
  KrylovArrays& K = W.ko;
  const long long n = H->n;
  const int nc = (int)cols.size();
  if (nc == 0) return;
  std::vector<int> it(nr), conv(nr);
  std::vector<double> est(nr), beta(nr), bn(nr);
  HELM_CHECK_HIP(hipMemcpyAsync(it.data(), K.it.p, sizeof(int) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(conv.data(), K.conv.p, sizeof(int) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(est.data(), K.est.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(beta.data(), K.beta.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(bn.data(), K.bnorm.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  bool identity = nc == nr;
  for (int k = 0; k < nc && identity; ++k) identity = cols[k] == k && orig[k] == k;
  for (int c : cols) {
    const int o = orig[c];
    out.it[o] = it[c];
    out.conv[o] = conv[c];
    out.est[o] = est[c];
    out.tru[o] = bn[c] > 0 ? beta[c] / bn[c] : 0.0;
  }
  if (identity) {  // the whole batch in its original order: one transpose and one copy
    launch_to_field_major(W.x.as<z64>(), W.w.as<z64>(), n, nr, H->stream);
    HELM_CHECK_HIP(hipMemcpyAsync((char*)X + sizeof(z64) * (size_t)n * r0, W.w.p, sizeof(z64) * (size_t)n * nr,
                                  hipMemcpyDefault, H->stream));
    return;
  }
  z64* sel = W.V.as<z64>();
  z64* fm = sel + (long long)n * nc;
  HELM_CHECK_HIP(hipMemcpyAsync(W.cols.p, cols.data(), sizeof(int) * nc, hipMemcpyHostToDevice, H->stream));
  launch_gather_cols(W.x.as<z64>(), nr, W.cols.as<int>(), nc, n, sel, H->stream);
  launch_to_field_major(sel, fm, n, nc, H->stream);
  for (int k = 0; k < nc; ++k)
    HELM_CHECK_HIP(hipMemcpyAsync((char*)X + sizeof(z64) * (size_t)n * (r0 + orig[cols[k]]), fm + (long long)n * k,
                                  sizeof(z64) * (size_t)n, hipMemcpyDefault, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
}

// At a restart some right-hand sides are done: report them and continue with
// a narrower batch of the rest (x, b and the residual w repacked, the per-RHS
// Krylov state of the kept columns moved to the front).  Each column's
// arithmetic is unchanged; only the batch width shrinks.
void compact_batch(helm_handle* H, int& nr, std::vector<int>& orig, void* X, int r0, ChunkOut& out) {
  Workspace& W = H->ws;
  KrylovArrays& K = W.ko;
  const long long n = H->n;
  std::vector<int> act(nr);
  HELM_CHECK_HIP(hipMemcpyAsync(act.data(), K.active.p, sizeof(int) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  std::vector<int> keep, done;
  for (int c = 0; c < nr; ++c) (act[c] ? keep : done).push_back(c);
  emit_columns(H, nr, orig, done, X, r0, out);
  const int nk = (int)keep.size();
  // vectors: gather the kept columns into the (free) basis storage, copy back narrower
  z64* tmp = W.V.as<z64>();
  const long long blk = n * nk;
  HELM_CHECK_HIP(hipMemcpyAsync(W.cols.p, keep.data(), sizeof(int) * nk, hipMemcpyHostToDevice, H->stream));
  launch_gather_cols(W.x.as<z64>(), nr, W.cols.as<int>(), nk, n, tmp, H->stream);
  launch_gather_cols(W.b.as<z64>(), nr, W.cols.as<int>(), nk, n, tmp + blk, H->stream);
  launch_gather_cols(W.w.as<z64>(), nr, W.cols.as<int>(), nk, n, tmp + 2 * blk, H->stream);
  launch_copy(tmp, W.x.as<z64>(), blk, H->stream);
  launch_copy(tmp + blk, W.b.as<z64>(), blk, H->stream);
  launch_copy(tmp + 2 * blk, W.w.as<z64>(), blk, H->stream);
  // per-RHS state of a fresh cycle: bnorm, beta, est, fac, it and g[0] move, the flags are known
  std::vector<double> bn(nr), beta(nr), est(nr), fac(nr);
  std::vector<int> it(nr);
  std::vector<z64> g0(nr);
  HELM_CHECK_HIP(hipMemcpyAsync(bn.data(), K.bnorm.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(beta.data(), K.beta.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(est.data(), K.est.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(fac.data(), K.fac.p, sizeof(double) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(it.data(), K.it.p, sizeof(int) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(g0.data(), K.g.p, sizeof(z64) * nr, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  auto pick = [&](auto& v) {
    std::remove_reference_t<decltype(v)> o(nk);
    for (int k = 0; k < nk; ++k) o[k] = v[keep[k]];
    return o;
  };
  const auto bn2 = pick(bn), beta2 = pick(beta), est2 = pick(est), fac2 = pick(fac);
  const auto it2 = pick(it);
  const auto g02 = pick(g0);
  const std::vector<int> ones(nk, 1), zeros(nk, 0);
  HELM_CHECK_HIP(hipMemcpyAsync(K.bnorm.p, bn2.data(), sizeof(double) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.beta.p, beta2.data(), sizeof(double) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.est.p, est2.data(), sizeof(double) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.fac.p, fac2.data(), sizeof(double) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.it.p, it2.data(), sizeof(int) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.g.p, g02.data(), sizeof(z64) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.active.p, ones.data(), sizeof(int) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.done.p, zeros.data(), sizeof(int) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.conv.p, zeros.data(), sizeof(int) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipMemcpyAsync(K.kc.p, zeros.data(), sizeof(int) * nk, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  std::vector<int> orig2(nk);
  for (int k = 0; k < nk; ++k) orig2[k] = orig[keep[k]];
  orig.swap(orig2);
  nr = nk;
  set_batch(H, nr);
}

// FGMRES on one batch; finished right-hand sides leave the batch at restarts.
// orig0: the chunk index of each batch column (identity when null).
void fgmres_chunk(helm_handle* H, int nr, double tol, int maxit, bool x0, void* X, int r0, ChunkOut& out,
                  const std::vector<int>* orig0 = nullptr) {
  Workspace& W = H->ws;
  KrylovArrays& K = W.ko;
  const long long n = H->n;
  const int m = H->dec.restart;
  std::vector<int> orig(nr);
  for (int c = 0; c < nr; ++c) orig[c] = orig0 ? (*orig0)[c] : c;
  // compaction stages three vectors of the batch in the basis storage
  static const bool no_compact = std::getenv("HELM_NO_COMPACT") != nullptr;
  const bool compact = !no_compact && m + 1 >= 3;
  launch_norm2(W.b.as<z64>(), n, nr, W.dpart.as<double>(), W.bn2.as<double>(), H->stream);
  launch_krylov_init(K.st, W.bn2.as<double>(), H->stream);
  if (x0) {
    fine_product(H, nr, W.b.as<z64>(), W.x.as<z64>(), W.w.as<z64>());
  } else {
    launch_fill(W.x.as<z64>(), n * nr, H->stream);
    launch_copy(W.b.as<z64>(), W.w.as<z64>(), n * nr, H->stream);
  }
  launch_norm2(W.w.as<z64>(), n, nr, W.dpart.as<double>(), W.beta2.as<double>(), H->stream);
  zero_counter(H, K);
  launch_cycle_start(K.st, W.beta2.as<double>(), tol, maxit, 1, H->stream);
  int nact = read_counter(H, K);
  while (nact > 0) {
    if (compact && nact < nr) compact_batch(H, nr, orig, X, r0, out);
    const long long vs = n * nr;
    launch_scale(W.w.as<z64>(), K.fac.as<double>(), W.V.as<z64>(), n, nr, H->stream);
    int steps = 0;  // basis vectors Z_0 .. Z_{steps-1} written in this cycle
    for (int j = 0; j < m; ++j) {
      run_outer_step(H, nr, j, tol, maxit);
      steps = j + 1;
      if (read_counter(H, K) == 0) break;
      launch_scale(W.w.as<z64>(), K.fac.as<double>(), W.V.as<z64>() + (j + 1) * vs, n, nr, H->stream);
    }
    launch_backsolve(K.st, H->stream);
    // only the vectors of this cycle: the rest of Z holds stale (pooled) memory,
    // and 0 * NaN would spoil x even where y is zero
    launch_update(W.Zv.as<z64>(), vs, steps, K.y.as<z64>(), W.x.as<z64>(), n, nr, H->stream);
    fine_product(H, nr, W.b.as<z64>(), W.x.as<z64>(), W.w.as<z64>());
    launch_norm2(W.w.as<z64>(), n, nr, W.dpart.as<double>(), W.beta2.as<double>(), H->stream);
    zero_counter(H, K);
    launch_cycle_start(K.st, W.beta2.as<double>(), tol, maxit, 0, H->stream);
    nact = read_counter(H, K);
  }
  std::vector<int> all(nr);
  for (int c = 0; c < nr; ++c) all[c] = c;
  emit_columns(H, nr, orig, all, X, r0, out);
}

// ---- block FGMRES: one Krylov space shared by the right-hand sides of a batch ----
using cd = std::complex<double>;

// The block least-squares problem min ||E_1 beta - Hbar Y||_F of block FGMRES.
// Hbar is block upper Hessenberg ((m+1)s x ms, s subdiagonals); it is reduced
// to triangular form column by column by Householder reflectors acting on the
// s + 1 rows c .. c + s of column c, applied to G = E_1 beta as they are made.
// After block column j the residual of right-hand side r is the norm of the
// s rows of G below the triangle.
struct BlockLS {
  int s = 0, m = 0;
  std::vector<std::vector<cd>> col;  // transformed columns, each (m+1)s rows
  std::vector<std::vector<cd>> ref;  // reflector vectors, s + 1 entries
  std::vector<double> tau;
  std::vector<cd> G;                 // [(m+1)s][s]
  void reset(int s_, int m_, const std::vector<cd>& beta) {  // beta: s x s, row-major
    s = s_;
    m = m_;
    col.clear();
    ref.clear();
    tau.clear();
    G.assign((size_t)(m + 1) * s * s, cd(0, 0));
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) G[(size_t)a * s + b] = beta[(size_t)a * s + b];
  }
  void apply(int c, cd* y, int stride) const {  // y[r * stride], r = c .. c + s
    const std::vector<cd>& v = ref[c];
    cd d(0, 0);
    for (int i = 0; i <= s; ++i) d += std::conj(v[i]) * y[(size_t)(c + i) * stride];
    d *= tau[c];
    for (int i = 0; i <= s; ++i) y[(size_t)(c + i) * stride] -= v[i] * d;
  }
  // Block column j: hcol[row * s + q], rows 0 .. (j+2)s - 1.
  void add_block(int j, const std::vector<cd>& hcol) {
    const int rows = (m + 1) * s;
    for (int q = 0; q < s; ++q) {
      const int c = j * s + q;
      std::vector<cd> x(rows, cd(0, 0));
      for (int r = 0; r < (j + 2) * s; ++r) x[r] = hcol[(size_t)r * s + q];
      for (int cp = 0; cp < c; ++cp) apply(cp, x.data(), 1);
      // reflector for rows c .. c + s: x -> alpha e_1
      double nrm = 0;
      for (int i = 0; i <= s; ++i) nrm += std::norm(x[c + i]);
      nrm = std::sqrt(nrm);
      std::vector<cd> v(s + 1, cd(0, 0));
      double t = 0;
      cd alpha(0, 0);
      if (nrm > 0) {
        const cd x0 = x[c];
        const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1, 0);
        alpha = -ph * nrm;
        for (int i = 0; i <= s; ++i) v[i] = x[c + i];
        v[0] -= alpha;
        double vv = 0;
        for (int i = 0; i <= s; ++i) vv += std::norm(v[i]);
        t = vv > 0 ? 2.0 / vv : 0.0;
      }
      ref.push_back(v);
      tau.push_back(t);
      x[c] = t > 0 ? alpha : x[c];
      for (int i = 1; i <= s; ++i) x[c + i] = cd(0, 0);
      col.push_back(x);
      for (int b = 0; b < s; ++b) apply(c, G.data() + b, s);
    }
  }
  double residual(int j, int r) const {  // after add_block(j)
    double acc = 0;
    for (int row = (j + 1) * s; row < (j + 2) * s; ++row) acc += std::norm(G[(size_t)row * s + r]);
    return std::sqrt(acc);
  }
  // Y (nb s x s, row-major) from the triangle of the first nb block columns.
  std::vector<cd> solve(int nb) const {
    const int K = nb * s;
    std::vector<cd> Y((size_t)K * s, cd(0, 0));
    for (int b = 0; b < s; ++b)
      for (int i = K - 1; i >= 0; --i) {
        cd acc = G[(size_t)i * s + b];
        for (int k = i + 1; k < K; ++k) acc -= col[k][i] * Y[(size_t)k * s + b];
        Y[(size_t)i * s + b] = acc / col[i][i];
      }
    return Y;
  }
};

// Cholesky factor R (upper, G = R^H R) of an s x s Hermitian block G given as
// [a][32 + b] complex128; false when a pivot is not positive beyond rounding
// (the block is numerically rank deficient).  Rinv = R^{-1}.
bool chol_upper(const std::vector<z64>& Gd, int s, std::vector<cd>& R, std::vector<cd>& Rinv) {
  R.assign((size_t)s * s, cd(0, 0));
  double gmax = 0;
  for (int k = 0; k < s; ++k) gmax = std::max(gmax, Gd[(size_t)k * 32 + k].re);
  for (int k = 0; k < s; ++k) {
    double d = Gd[(size_t)k * 32 + k].re;
    for (int i = 0; i < k; ++i) d -= std::norm(R[(size_t)i * s + k]);
    if (!(d > 1e-28 * gmax) || !std::isfinite(d)) return false;
    const double rk = std::sqrt(d);
    R[(size_t)k * s + k] = rk;
    for (int j = k + 1; j < s; ++j) {
      cd g(Gd[(size_t)k * 32 + j].re, Gd[(size_t)k * 32 + j].im);
      for (int i = 0; i < k; ++i) g -= std::conj(R[(size_t)i * s + k]) * R[(size_t)i * s + j];
      R[(size_t)k * s + j] = g / rk;
    }
  }
  Rinv.assign((size_t)s * s, cd(0, 0));
  for (int j = 0; j < s; ++j) {  // column j of R^{-1}: back substitution on e_j
    Rinv[(size_t)j * s + j] = 1.0 / R[(size_t)j * s + j];
    for (int i = j - 1; i >= 0; --i) {
      cd acc(0, 0);
      for (int k = i + 1; k <= j; ++k) acc += R[(size_t)i * s + k] * Rinv[(size_t)k * s + j];
      Rinv[(size_t)i * s + j] = -acc / R[(size_t)i * s + i];
    }
  }
  return true;
}

std::vector<z64> to_padded(const std::vector<cd>& M, int s) {  // s x s row-major -> [32][32]
  std::vector<z64> P(1024, mk(0.0, 0.0));
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b) P[(size_t)a * 32 + b] = mk(M[(size_t)a * s + b].real(), M[(size_t)a * s + b].imag());
  return P;
}

// Q R = Win (n x s) by two Cholesky-QR passes: Qout = Win R1^{-1} R2^{-1},
// R = R2 R1.  Win is overwritten.  False when the block is rank deficient.
bool cholqr2(helm_handle* H, int s, z64* Win, z64* Qout, std::vector<cd>& R) {
  Workspace& W = H->ws;
  const long long n = H->n;
  std::vector<cd> R1, R2, T;
  std::vector<z64> Gd(1024);
  for (int pass = 0; pass < 2; ++pass) {
    z64* src = pass == 0 ? Win : Qout;
    z64* dst = pass == 0 ? Qout : Win;
    launch_block_dots(src, 0, 1, src, n, s, W.bpart.as<z64>(), W.bcoef.as<z64>(), H->stream);
    HELM_CHECK_HIP(hipMemcpyAsync(Gd.data(), W.bcoef.p, sizeof(z64) * 1024, hipMemcpyDeviceToHost, H->stream));
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    std::vector<cd>& Rp = pass == 0 ? R1 : R2;
    if (!chol_upper(Gd, s, Rp, T)) return false;
    const std::vector<z64> Tp = to_padded(T, s);
    HELM_CHECK_HIP(hipMemcpyAsync(W.bcoef.p, Tp.data(), sizeof(z64) * 1024, hipMemcpyHostToDevice, H->stream));
    launch_block_gemm(src, 0, 1, W.bcoef.as<z64>(), n, s, 1.0, false, dst, H->stream);
  }
  launch_copy(Win, Qout, n * s, H->stream);  // the second pass wrote into Win
  R.assign((size_t)s * s, cd(0, 0));
  for (int a = 0; a < s; ++a)
    for (int b = a; b < s; ++b)
      for (int k = a; k <= b; ++k) R[(size_t)a * s + b] += R2[(size_t)a * s + k] * R1[(size_t)k * s + b];
  return true;
}

std::vector<double> column_norms(helm_handle* H, const z64* v, int s) {
  Workspace& W = H->ws;
  std::vector<double> out(s);
  launch_norm2(v, H->n, s, W.dpart.as<double>(), W.bn2.as<double>(), H->stream);
  HELM_CHECK_HIP(hipMemcpyAsync(out.data(), W.bn2.p, sizeof(double) * s, hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  for (double& x : out) x = std::sqrt(x);
  return out;
}

// Block FGMRES on the s columns of W.b (all nonzero), x in W.x (zero, or the
// initial guess when x0): the oracle's block_fgmres step for step.  Returns
// false, with W.x holding the iterate so far, when a block to orthonormalise at
// a (re)start is rank deficient; iters and the residuals go to the per-column
// vectors.
bool block_fgmres_batch(helm_handle* H, int s, double tol, int maxit, bool x0, std::vector<int>& its,
                        std::vector<double>& est, std::vector<double>& tru, int& k) {
  Workspace& W = H->ws;
  const long long n = H->n, vs = n * s;
  const int m = H->dec.restart;
  const std::vector<double> bn = column_norms(H, W.b.as<z64>(), s);
  if (x0) fine_product(H, s, W.b.as<z64>(), W.x.as<z64>(), W.w.as<z64>());
  else {
    launch_fill(W.x.as<z64>(), vs, H->stream);
    launch_copy(W.b.as<z64>(), W.w.as<z64>(), vs, H->stream);
  }
  std::vector<double> rn = column_norms(H, W.w.as<z64>(), s);
  for (int r = 0; r < s; ++r) est[r] = rn[r] / bn[r];
  BlockLS ls;
  std::vector<z64> Cd((size_t)1024 * (m + 1));
  while (true) {
    bool done = true;
    for (int r = 0; r < s; ++r) done = done && rn[r] <= tol * bn[r];
    if (done || k >= maxit) break;
    std::vector<cd> beta;
    if (!cholqr2(H, s, W.w.as<z64>(), W.V.as<z64>(), beta)) return false;
    ls.reset(s, m, beta);
    int nb = 0;
    for (int j = 0; j < m; ++j) {
      z64* vj = W.V.as<z64>() + j * vs;
      z64* zj = W.Zv.as<z64>() + j * vs;
      precond(H, s, vj, zj);
      fine_product(H, s, nullptr, zj, W.w.as<z64>());
      double w0 = 0;
      for (double x : column_norms(H, W.w.as<z64>(), s)) w0 += x * x;
      w0 = std::sqrt(w0);
      // two classical block Gram-Schmidt passes, coefficients accumulated
      std::vector<cd> hcol((size_t)(j + 2) * s * s, cd(0, 0));
      for (int pass = 0; pass < 2; ++pass) {
        launch_block_dots(W.V.as<z64>(), vs, j + 1, W.w.as<z64>(), n, s, W.bpart.as<z64>(), W.bcoef.as<z64>(),
                          H->stream);
        launch_block_gemm(W.V.as<z64>(), vs, j + 1, W.bcoef.as<z64>(), n, s, -1.0, true, W.w.as<z64>(), H->stream);
        HELM_CHECK_HIP(hipMemcpyAsync(Cd.data(), W.bcoef.p, sizeof(z64) * 1024 * (j + 1), hipMemcpyDeviceToHost,
                                      H->stream));
        HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
        for (int i = 0; i <= j; ++i)
          for (int a = 0; a < s; ++a)
            for (int b = 0; b < s; ++b) {
              const z64 c = Cd[(size_t)i * 1024 + a * 32 + b];
              hcol[(size_t)(i * s + a) * s + b] += cd(c.re, c.im);
            }
      }
      // W = V_{j+1} H_{j+1,j}; a rank-deficient W is a breakdown (its block stays zero)
      std::vector<cd> Rn;
      const bool full = j + 1 <= m && cholqr2(H, s, W.w.as<z64>(), W.V.as<z64>() + (j + 1) * vs, Rn);
      double dmin = 0;
      if (full) {
        dmin = std::abs(Rn[0]);
        for (int a = 0; a < s; ++a) {
          dmin = std::min(dmin, std::abs(Rn[(size_t)a * s + a]));
          for (int b = 0; b < s; ++b) hcol[(size_t)((j + 1) * s + a) * s + b] = Rn[(size_t)a * s + b];
        }
      }
      ls.add_block(j, hcol);
      ++k;
      nb = j + 1;
      bool conv = true;
      for (int r = 0; r < s; ++r) {
        est[r] = ls.residual(j, r) / bn[r];
        conv = conv && est[r] <= tol;
      }
      const bool breakdown = !full || dmin <= 1e-14 * w0;
      if (conv || breakdown || k >= maxit) break;
    }
    // X += sum_i Z_i Y_i, then the true residual
    const std::vector<cd> Y = ls.solve(nb);
    std::vector<z64> Yp((size_t)1024 * nb, mk(0.0, 0.0));
    for (int i = 0; i < nb; ++i)
      for (int a = 0; a < s; ++a)
        for (int b = 0; b < s; ++b) {
          const cd y = Y[(size_t)(i * s + a) * s + b];
          Yp[(size_t)i * 1024 + a * 32 + b] = mk(y.real(), y.imag());
        }
    HELM_CHECK_HIP(hipMemcpyAsync(W.bcoef.p, Yp.data(), sizeof(z64) * Yp.size(), hipMemcpyHostToDevice, H->stream));
    launch_block_gemm(W.Zv.as<z64>(), vs, nb, W.bcoef.as<z64>(), n, s, 1.0, true, W.x.as<z64>(), H->stream);
    fine_product(H, s, W.b.as<z64>(), W.x.as<z64>(), W.w.as<z64>());
    rn = column_norms(H, W.w.as<z64>(), s);
  }
  for (int r = 0; r < s; ++r) {
    its[r] = k;
    tru[r] = rn[r] / bn[r];
  }
  return true;
}

// Block FGMRES on a staged batch (W.b, and W.x when x0), results into out and X
// (chunk offset r0).  Right-hand sides that are zero get X = 0 and no
// iteration and stay out of the block; if a block to orthonormalise is rank
// deficient, the batch continues from the current iterate with one Krylov
// space per right-hand side (fgmres_chunk), its iterations added to the
// block's.
void block_chunk(helm_handle* H, int nr, double tol, int maxit, bool x0, void* X, int r0, ChunkOut& out) {
  Workspace& W = H->ws;
  const long long n = H->n;
  const std::vector<double> bn = column_norms(H, W.b.as<z64>(), nr);
  std::vector<int> keep, zero;
  for (int c = 0; c < nr; ++c) (bn[c] > 0 ? keep : zero).push_back(c);
  if (!zero.empty()) {
    launch_fill(W.w.as<z64>(), n, H->stream);
    for (int c : zero) {
      HELM_CHECK_HIP(hipMemcpyAsync((char*)X + sizeof(z64) * (size_t)n * (r0 + c), W.w.p, sizeof(z64) * (size_t)n,
                                    hipMemcpyDefault, H->stream));
      out.it[c] = 0;
      out.conv[c] = 1;
      out.est[c] = 0;
      out.tru[c] = 0;
    }
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  }
  const int s = (int)keep.size();
  if (s == 0) return;
  if (s < nr) {  // the nonzero columns to the front (the basis storage is free here)
    z64* tmp = W.V.as<z64>();
    HELM_CHECK_HIP(hipMemcpyAsync(W.cols.p, keep.data(), sizeof(int) * s, hipMemcpyHostToDevice, H->stream));
    launch_gather_cols(W.b.as<z64>(), nr, W.cols.as<int>(), s, n, tmp, H->stream);
    launch_gather_cols(W.x.as<z64>(), nr, W.cols.as<int>(), s, n, tmp + n * s, H->stream);
    launch_copy(tmp, W.b.as<z64>(), n * s, H->stream);
    launch_copy(tmp + n * s, W.x.as<z64>(), n * s, H->stream);
  }
  set_batch(H, s);
  std::vector<int> its(s, 0);
  std::vector<double> est(s, 0.0), tru(s, 0.0);
  int k = 0;
  if (!block_fgmres_batch(H, s, tol, maxit, x0, its, est, tru, k)) {
    fgmres_chunk(H, s, tol, std::max(maxit - k, 0), true, X, r0, out, &keep);
    for (int c : keep) out.it[c] += k;
    return;
  }
  // solutions field-major to X at their chunk index
  launch_to_field_major(W.x.as<z64>(), W.w.as<z64>(), n, s, H->stream);
  for (int q = 0; q < s; ++q)
    HELM_CHECK_HIP(hipMemcpyAsync((char*)X + sizeof(z64) * (size_t)n * (r0 + keep[q]), W.w.as<z64>() + n * q,
                                  sizeof(z64) * (size_t)n, hipMemcpyDefault, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  for (int q = 0; q < s; ++q) {
    const int c = keep[q];
    out.it[c] = its[q];
    out.est[c] = est[q];
    out.tru[c] = tru[q];
    out.conv[c] = tru[q] <= tol ? 1 : 0;
  }
}

struct Timer {
  hipEvent_t a, b;
  hipStream_t s;
  explicit Timer(hipStream_t st) : s(st) {
    HELM_CHECK_HIP(locked_event_create(&a));
    HELM_CHECK_HIP(locked_event_create(&b));
    HELM_CHECK_HIP(hipEventRecord(a, s));
  }
  double stop() {
    HELM_CHECK_HIP(hipEventRecord(b, s));
    HELM_CHECK_HIP(hipEventSynchronize(b));
    float ms = 0;
    HELM_CHECK_HIP(hipEventElapsedTime(&ms, a, b));
    return ms * 1e-3;
  }
  ~Timer() {
    locked_event_destroy(a);
    locked_event_destroy(b);
  }
};

// The sweeps need only the plane couplings of the local operators: keep them
// in the factor precision and release the full rows.
void extract_couplings(helm_handle* H, Level& L) {
  L.cpl.alloc(elem_size(L.prec) * 18 * (size_t)L.nodes_total);
  if (L.prec)
    launch_couplings<float>(L.nodes_total, L.aloc.as<z64>(), L.cpl.as<c32>(), H->stream);
  else
    launch_couplings<double>(L.nodes_total, L.aloc.as<z64>(), L.cpl.as<z64>(), H->stream);
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  L.aloc.release();
}

void factor_level(helm_handle* H, Level& L) {
  DevBuf Wt, St, Rb, R64, piv, perm;
  const size_t es = elem_size(L.prec);
  Wt.alloc((size_t)L.nsub * L.bpmax * L.bpmax * es);
  St.alloc((size_t)L.nsub * L.bpmax * L.bpmax * es);
  Rb.alloc((size_t)L.nsub * 16 * L.bpmax * es);
  R64.alloc((size_t)L.nsub * 64 * L.bpmax * es);
  piv.alloc((size_t)L.nsub * L.bpmax * sizeof(int));
  perm.alloc((size_t)L.nsub * L.bpmax * sizeof(int));
  launch_fill(H->err.as<z64>(), 1, H->stream);
  for (int k = 0; k < L.maxez; ++k) {
    if (L.prec == 1)
      Factor<float>::plane(L.d_subs.as<Sub>(), L.nsub, L.bpmax, k, L.aloc.as<z64>(), L.sinv.as<c32>(), Wt.as<c32>(),
                           St.as<c32>(), Rb.as<c32>(), R64.as<c32>(), piv.as<int>(), perm.as<int>(), H->err.as<int>(),
                           H->stream);
    else
      Factor<double>::plane(L.d_subs.as<Sub>(), L.nsub, L.bpmax, k, L.aloc.as<z64>(), L.sinv.as<z64>(), Wt.as<z64>(),
                            St.as<z64>(), Rb.as<z64>(), R64.as<z64>(), piv.as<int>(), perm.as<int>(),
                            H->err.as<int>(), H->stream);
  }
  int e = 0;
  HELM_CHECK_HIP(hipMemcpyAsync(&e, H->err.p, sizeof(int), hipMemcpyDeviceToHost, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  if (e) throw HelmError(HELM_EBREAKDOWN, "numerically singular pivot in a local factorisation");
}

// The boxes in launch order for the batched local solves: by decreasing work
// ((2 ez - 1) b^2 per right-hand side, the plane products), dealt round-robin
// over the eight XCDs' contiguous ranges of logical workgroups
// (xcd_contiguous), so that every XCD starts on its largest boxes and the last
// wave of workgroups holds the smallest.  A sweep's results do not depend on
// the order: every box writes only its own plane vectors and its core nodes.
std::vector<Sub> sweep_order(const std::vector<Sub>& subs) {
  const int n = (int)subs.size();
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  auto work = [&](int i) { return (2.0 * subs[i].ez - 1.0) * (double)subs[i].b * subs[i].b; };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work(a) > work(b); });
  constexpr int NXCD = 8;
  const int per = n / NXCD, rem = n % NXCD;
  std::vector<Sub> out(n);
  for (int i = 0; i < n; ++i) {
    const int c = i % NXCD, li = i / NXCD;
    out[c * per + std::min(c, rem) + li] = subs[idx[i]];
  }
  return out;
}

// Device copies of the boxes: [0, nsub) in box order (set-up kernels, arrays
// indexed by box), [nsub, 2 nsub) in sweep launch order.
void upload_subs(Level& L, hipStream_t stream) {
  const size_t n = L.subs.size();
  const std::vector<Sub> order = sweep_order(L.subs);
  L.d_subs.alloc(sizeof(Sub) * n * 2);
  HELM_CHECK_HIP(hipMemcpyAsync(L.d_subs.p, L.subs.data(), sizeof(Sub) * n, hipMemcpyHostToDevice, stream));
  HELM_CHECK_HIP(hipMemcpyAsync(L.d_subs.as<Sub>() + n, order.data(), sizeof(Sub) * n, hipMemcpyHostToDevice, stream));
  HELM_CHECK_HIP(hipStreamSynchronize(stream));
}

void setup_impl(helm_handle* H, const void* velocity, int vel_kind) {
  HELM_CHECK_HIP(hipGetDevice(&H->device));
  H->own = streams().acquire(H->device);
  H->stream = H->own;
  const long long n = H->n;
  // velocity: copied to the host (a real array widened to complex with zero
  // imaginary parts) and validated there
  std::vector<z64> ch((size_t)n);
  if (vel_kind == HELM_VEL_REAL64) {
    std::vector<double> cr((size_t)n);
    HELM_CHECK_HIP(hipMemcpyAsync(cr.data(), velocity, sizeof(double) * n, hipMemcpyDefault, H->stream));
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    for (long long i = 0; i < n; ++i) ch[i] = mk(cr[i], 0.0);
  } else {
    HELM_CHECK_HIP(hipMemcpyAsync(ch.data(), velocity, sizeof(z64) * n, hipMemcpyDefault, H->stream));
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  }
  for (long long i = 0; i < n; ++i) {
    if (!std::isfinite(ch[i].re) || !std::isfinite(ch[i].im) || !(ch[i].re > 0))
      throw HelmError(HELM_EINVAL, "velocity must be finite with a positive real part");
  }
  plan(H);
  const size_t need = resident_bytes_planned(H) + std::max(level_setup_bytes(H->fine), level_setup_bytes(H->coarse)) +
                      ws_bytes(H, 1);
  if (need > budget_bytes()) throw HelmError(HELM_ENOMEM, "footprint " + std::to_string(need) + " bytes exceeds the device budget");

  Timer tall(H->stream);
  H->c.alloc(sizeof(z64) * n);
  HELM_CHECK_HIP(hipMemcpyAsync(H->c.p, ch.data(), sizeof(z64) * n, hipMemcpyHostToDevice, H->stream));
  HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
  H->sigma.alloc(sizeof(z64) * n);
  const int tot_int = H->nx + H->ny + H->nz;
  H->xi_int.alloc(sizeof(z64) * tot_int);
  H->i2_int.alloc(sizeof(z64) * tot_int);
  H->xi_half.alloc(sizeof(z64) * (tot_int + 3));
  H->i2_half.alloc(sizeof(z64) * (tot_int + 3));
  H->flat.alloc(tot_int);
  H->vmax.alloc(sizeof(double));
  H->err.alloc(64);
  launch_vmax(H->c.as<z64>(), n, H->vmax.as<double>(), H->stream);
  AxisPml ax[3] = {{H->nx, H->pml.npml_x, H->pml.npml_x},
                   {H->ny, H->pml.npml_y, H->pml.npml_y},
                   {H->nz, H->pml.npml_ztop, H->pml.npml_zbot}};
  const double R = H->pml.R > 0 ? H->pml.R : 1e-3;
  launch_pml_tables(ax, H->h, H->omega, R, H->vmax.as<double>(), H->xi_int.as<z64>(), H->xi_half.as<z64>(),
                    H->i2_int.as<z64>(), H->i2_half.as<z64>(), H->flat.as<uint8_t>(), H->stream);
  OpDev& op = H->op;
  op.nx = H->nx;
  op.ny = H->ny;
  op.nz = H->nz;
  op.h2inv = 1.0 / (H->h * H->h);
  op.alpha[0] = H->w.w1 + H->w.w2 / 3.0;
  op.alpha[1] = H->w.w2 / 6.0;
  op.alpha[2] = H->w.w3 / 4.0;
  op.wm[0] = H->w.wm1;
  op.wm[1] = H->w.wm2;
  op.wm[2] = H->w.wm3;
  op.wm[3] = H->w.wm4;
  op.sigma = H->sigma.as<z64>();
  op.xi_int = H->xi_int.as<z64>();
  op.xi_half = H->xi_half.as<z64>();
  op.i2_int = H->i2_int.as<z64>();
  op.i2_half = H->i2_half.as<z64>();
  op.flat = H->flat.as<uint8_t>();
  op.off_int[0] = 0;
  op.off_int[1] = H->nx;
  op.off_int[2] = H->nx + H->ny;
  op.off_half[0] = 0;
  op.off_half[1] = H->nx + 1;
  op.off_half[2] = H->nx + H->ny + 2;
  op.wnode = nullptr;
  if (H->dec.adaptive) {  // per-node weights from the table at each node's points per wavelength
    std::vector<helm_weights_t> tw(ADAPT_N);
    fit_weight_table_host(ADAPT_G0, ADAPT_DG, ADAPT_N, ADAPT_NANG, tw.data());
    std::vector<double> tab((size_t)ADAPT_N * 7);
    for (int j = 0; j < ADAPT_N; ++j) {
      const helm_weights_t& w = tw[j];
      const double v[7] = {w.w1, w.w2, w.w3, w.wm1, w.wm2, w.wm3, w.wm4};
      for (int q = 0; q < 7; ++q) tab[(size_t)j * 7 + q] = v[q];
    }
    H->wtab.alloc(sizeof(double) * tab.size());
    H->wnode.alloc(sizeof(double) * 8 * (size_t)n);
    HELM_CHECK_HIP(hipMemcpyAsync(H->wtab.p, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, H->stream));
    launch_node_weights(H->c.as<z64>(), n, H->freq, H->h, H->wtab.as<double>(), ADAPT_N, ADAPT_G0, ADAPT_DG,
                        H->wnode.as<double>(), H->stream);
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    op.wnode = H->wnode.as<double>();
  }
  launch_sigma(op, H->c.as<z64>(), H->omega, H->stream);
  H->diag.alloc(sizeof(z64) * n);
  op.diag = nullptr;
  launch_row_diag(op, H->diag.as<z64>(), H->stream);
  op.diag = H->diag.as<z64>();

  // fine level: local operators with absorbing interfaces, then factorisation
  Level& F = H->fine;
  upload_subs(F, H->stream);
  F.aloc.alloc(sizeof(z64) * 27 * (size_t)F.nodes_total);
  F.sinv.alloc(elem_size(F.prec) * (size_t)F.mat_total);
  launch_local_fine(op, F.d_subs.as<Sub>(), F.nsub, F.maxnodes, H->c.as<z64>(), H->omega, H->h, H->dec.robin,
                    F.aloc.as<z64>(), H->stream);
  {
    Timer tf(H->stream);
    factor_level(H, F);
    H->t_fact = tf.stop();
  }
  extract_couplings(H, F);
  if (F.half) {  // approximate local solves: the complex FP32 inverses to FP16 with a scale per plane
    F.sinv16.alloc(sizeof(uint4) * (size_t)(F.mat_total / 4));
    F.sexp.alloc(sizeof(int) * (size_t)F.nsub * F.maxez);
    launch_to_half(F.d_subs.as<Sub>(), F.nsub, F.maxez, F.sinv.as<c32>(), F.sinv16.as<uint4>(), F.sexp.as<int>(),
                   H->stream);
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    F.sinv.release();
  }
  if (H->two_level()) {
    Timer tc(H->stream);
    Level& C = H->coarse;
    C.E.alloc(sizeof(z64) * 27 * (size_t)C.n);
    launch_build_E(op, C.nx, C.ny, C.nz, C.E.as<z64>(), H->stream);
    upload_subs(C, H->stream);
    C.aloc.alloc(sizeof(z64) * 27 * (size_t)C.nodes_total);
    C.sinv.alloc(elem_size(C.prec) * (size_t)C.mat_total);
    launch_local_coarse(C.nx, C.ny, C.nz, C.E.as<z64>(), C.d_subs.as<Sub>(), C.nsub, C.maxnodes, H->c.as<z64>(), H->nx,
                        H->ny, H->omega, 2.0 * H->h, H->dec.robin, C.aloc.as<z64>(), H->stream);
    factor_level(H, C);
    extract_couplings(H, C);
    H->t_coarse = tc.stop();
  }
  H->t_setup = tall.stop();
  HELM_CHECK_HIP(hipGetLastError());
}

int choose_chunk(helm_handle* H, int nrhs, bool block) {
  int nr = H->dec.nrhs_chunk > 0 ? H->dec.nrhs_chunk : nrhs;
  nr = std::min(nr, nrhs);
  nr = std::min(nr, block ? 32 : 256);  // a block Krylov space spans at most 32 right-hand sides
  if (H->ws.nr >= nr) return nr;  // already allocated
  const size_t held = H->ws.nr > 0 ? ws_bytes(H, H->ws.nr) : 0;
  const size_t avail = budget_bytes() + held;
  while (nr > 1 && ws_bytes(H, nr) > avail) nr = (nr + 1) / 2;
  if (ws_bytes(H, nr) > avail) throw HelmError(HELM_ENOMEM, "Krylov workspace of one right-hand side exceeds the device budget");
  return nr;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

helm_status helm_fit_weights(double gmin, double gmax, int32_t ng, int32_t nang, helm_weights_t* out) {
  return guarded([&]() {
    if (!out || ng < 1 || nang < 1 || !(gmin > 0) || !(gmax >= gmin))
      throw HelmError(HELM_EINVAL, "bad fit parameters");
    fit_weights_host(gmin, gmax, ng, nang, out);
    return HELM_OK;
  });
}

helm_status helm_fit_weight_table(double g0, double dg, int32_t n, int32_t nang, helm_weights_t* out) {
  return guarded([&]() {
    if (!out || n < 1 || nang < 1 || !(g0 > 0) || !(dg > 0) || !std::isfinite(g0) || !std::isfinite(dg))
      throw HelmError(HELM_EINVAL, "bad table parameters");
    fit_weight_table_host(g0, dg, n, nang, out);
    return HELM_OK;
  });
}

helm_status helm_setup(const helm_grid_t* grid, const void* velocity, int32_t vel_kind, double freq_hz,
                       const helm_pml_t* pml, const helm_weights_t* weights, const helm_decomp_t* dec,
                       helm_handle_t** out) {
  return guarded([&]() {
    if (!out || !velocity) throw HelmError(HELM_EINVAL, "null argument");
    *out = nullptr;
    if (vel_kind != HELM_VEL_COMPLEX128 && vel_kind != HELM_VEL_REAL64)
      throw HelmError(HELM_EINVAL, "vel_kind must be HELM_VEL_COMPLEX128 or HELM_VEL_REAL64");
    validate(grid, pml, dec);
    if (!(freq_hz > 0) || !std::isfinite(freq_hz)) throw HelmError(HELM_EINVAL, "frequency must be positive");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
      (void)hipGetLastError();
      throw HelmError(HELM_EDEVICE, "no HIP device");
    }
    std::unique_ptr<helm_handle> H(new helm_handle());
    H->nx = grid->nx;
    H->ny = grid->ny;
    H->nz = grid->nz;
    H->n = (long long)grid->nx * grid->ny * grid->nz;
    H->h = grid->h;
    H->freq = freq_hz;
    H->omega = 2.0 * 3.14159265358979323846 * freq_hz;
    H->pml = *pml;
    H->dec = *dec;
    if (weights) H->w = *weights;
    else fit_weights_host(4.0, 10.0, 7, 15, &H->w);
    setup_impl(H.get(), velocity, vel_kind);
    *out = H.release();
    return HELM_OK;
  });
}

struct helm_request {
  std::atomic<helm_handle*> H{nullptr};  // null once helm_destroy has joined the solve
  std::thread worker;
  std::atomic<bool> done{false};
  std::atomic<int> status{HELM_PENDING};
  std::string message;
  bool joined = false;  // guarded by H->pending_mu
};

namespace {
bool busy(helm_handle* H) {
  std::lock_guard<std::mutex> lk(H->pending_mu);
  return H->pending != nullptr;
}
// Join the handle's in-flight request (if any) and detach it from the handle.
void finish_pending(helm_handle* H) {
  std::lock_guard<std::mutex> lk(H->pending_mu);
  helm_request* q = H->pending;
  if (!q) return;
  if (!q->joined) {
    q->worker.join();
    q->joined = true;
  }
  q->H.store(nullptr);
  H->pending = nullptr;
}
}  // namespace

namespace {
helm_status solve_impl(helm_handle* H, int32_t nrhs, const void* B, void* X, double tol, int32_t maxit,
                       uint32_t flags, int32_t* iters, double* relres_est, double* relres_true) {
  return guarded([&]() {
    if (!H || !B || !X || nrhs < 0 || !(tol >= 0) || maxit < 0) throw HelmError(HELM_EINVAL, "bad solve arguments");
    if (nrhs == 0) return HELM_OK;
    const long long n = H->n;
    const bool block = (flags & HELM_BLOCK) != 0;
    const int nr_max = choose_chunk(H, nrhs, block);
    ensure_ws(H, nr_max);
    Workspace& W = H->ws;
    H->work_solve = WorkBound{};
    HELM_CHECK_HIP(hipMemsetAsync(W.ko.extra.p, 0, sizeof(double), H->stream));
    if (H->two_level()) HELM_CHECK_HIP(hipMemsetAsync(W.kc.extra.p, 0, sizeof(double), H->stream));
    struct Install {  // this thread's launches count towards the solve's bound until return
      WorkBound* prev;
      explicit Install(WorkBound* w) : prev(g_work) { g_work = w; }
      ~Install() { g_work = prev; }
    } install(&H->work_solve);
    std::vector<int> it_all(nrhs), conv_all(nrhs);
    std::vector<double> est_all(nrhs), tru_all(nrhs);
    bool all_conv = true;
    Timer tt(H->stream);
    for (int r0 = 0; r0 < nrhs; r0 += nr_max) {
      const int nr = std::min(nr_max, nrhs - r0);
      set_batch(H, nr);
      const size_t bytes = sizeof(z64) * (size_t)n * nr;
      // stage B[r0:r0+nr] through W.w (field-major) into W.b (node-major)
      HELM_CHECK_HIP(hipMemcpyAsync(W.w.p, (const char*)B + sizeof(z64) * (size_t)n * r0, bytes, hipMemcpyDefault, H->stream));
      launch_to_node_major(W.w.as<z64>(), W.b.as<z64>(), n, nr, H->stream);
      const bool x0 = (flags & HELM_X0) != 0;
      if (x0) {
        HELM_CHECK_HIP(hipMemcpyAsync(W.w.p, (const char*)X + sizeof(z64) * (size_t)n * r0, bytes, hipMemcpyDefault, H->stream));
        launch_to_node_major(W.w.as<z64>(), W.x.as<z64>(), n, nr, H->stream);
      }
      ChunkOut co;
      co.it.assign(nr, 0);
      co.conv.assign(nr, 0);
      co.est.assign(nr, 0.0);
      co.tru.assign(nr, 0.0);
      if (block) block_chunk(H, nr, tol, maxit, x0, X, r0, co);
      else fgmres_chunk(H, nr, tol, maxit, x0, X, r0, co);
      for (int r = 0; r < nr; ++r) {
        it_all[r0 + r] = co.it[r];
        conv_all[r0 + r] = co.conv[r];
        est_all[r0 + r] = co.est[r];
        tru_all[r0 + r] = co.tru[r];
        all_conv = all_conv && co.conv[r];
      }
    }
    H->t_solve = tt.stop();
    collect_sweep_timing(H);
    {  // the second Gram-Schmidt updates that ran (decided on the device) join the solve's bound
      double ex[2] = {0.0, 0.0};
      HELM_CHECK_HIP(hipMemcpyAsync(&ex[0], W.ko.extra.p, sizeof(double), hipMemcpyDeviceToHost, H->stream));
      if (H->two_level())
        HELM_CHECK_HIP(hipMemcpyAsync(&ex[1], W.kc.extra.p, sizeof(double), hipMemcpyDeviceToHost, H->stream));
      HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
      H->work_solve.bytes += ex[0] + ex[1];
      H->work_solve.seconds += (ex[0] + ex[1]) / HBM_PEAK;
    }
    double its = 0;
    for (int r = 0; r < nrhs; ++r) {
      its += it_all[r];
      if (iters) iters[r] = it_all[r];
      if (relres_est) relres_est[r] = est_all[r];
      if (relres_true) relres_true[r] = tru_all[r];
    }
    H->its = its;
    HELM_CHECK_HIP(hipGetLastError());
    return all_conv ? HELM_OK : HELM_NOT_CONVERGED;
  }, H);
}
}  // namespace

helm_status helm_solve(helm_handle_t* H, int32_t nrhs, const void* B, void* X, double tol, int32_t maxit,
                       uint32_t flags, int32_t* iters, double* relres_est, double* relres_true) {
  if (H && busy(H)) return fail_h(H, HELM_EINVAL, "a solve is already in flight on this handle");
  return solve_impl(H, nrhs, B, X, tol, maxit, flags, iters, relres_est, relres_true);
}

size_t helm_footprint(const helm_grid_t* grid, const helm_decomp_t* dec, int32_t nrhs_chunk) {
  try {
    helm_pml_t pml{0, 0, 0, 0, 0};
    validate(grid, &pml, dec);
    helm_handle H;
    H.nx = grid->nx;
    H.ny = grid->ny;
    H.nz = grid->nz;
    H.n = (long long)grid->nx * grid->ny * grid->nz;
    H.dec = *dec;
    plan(&H);
    return resident_bytes_planned(&H) + std::max(level_setup_bytes(H.fine), level_setup_bytes(H.coarse)) +
           ws_bytes(&H, std::max(1, nrhs_chunk));
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return 0;
  }
}

size_t helm_workspace_bytes(const helm_grid_t* grid, const helm_decomp_t* dec, int32_t nrhs_chunk) {
  try {
    helm_pml_t pml{0, 0, 0, 0, 0};
    validate(grid, &pml, dec);
    if (nrhs_chunk < 1) throw HelmError(HELM_EINVAL, "nrhs_chunk must be at least 1");
    helm_handle H;
    H.nx = grid->nx;
    H.ny = grid->ny;
    H.nz = grid->nz;
    H.n = (long long)grid->nx * grid->ny * grid->nz;
    H.dec = *dec;
    plan(&H);
    return ws_bytes(&H, nrhs_chunk);
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return 0;
  }
}

size_t helm_resident_bytes(const helm_handle_t* H) {
  if (!H) return 0;
  // the blocks actually held: the device cache may hand out a block up to an
  // eighth larger than asked for, so this can exceed the planned bytes
  size_t b = 0;
  for (const DevBuf* d : {&H->c, &H->sigma, &H->xi_int, &H->xi_half, &H->i2_int, &H->i2_half, &H->flat, &H->vmax,
                          &H->err, &H->wtab, &H->wnode})
    b += d->bytes;
  for (const Level* L : {&H->fine, &H->coarse})
    for (const DevBuf* d : {&L->d_subs, &L->aloc, &L->sinv, &L->E, &L->cpl, &L->sinv16, &L->sexp}) b += d->bytes;
  const Workspace& W = H->ws;
  for (const DevBuf* d : {&W.b, &W.x, &W.w, &W.V, &W.Zv, &W.q, &W.t, &W.cc, &W.Vc, &W.Zc, &W.wc, &W.ec, &W.yl_f,
                          &W.tb_f, &W.yl_c, &W.tb_c, &W.zpart, &W.dpart, &W.bn2, &W.beta2, &W.cols, &W.bpart,
                          &W.bcoef})
    b += d->bytes;
  for (const KrylovArrays* k : {&W.ko, &W.kc})
    for (const DevBuf* d : {&k->Rm, &k->g, &k->cs, &k->sn, &k->y, &k->h, &k->h2, &k->nrm2, &k->w0, &k->w1, &k->bnorm,
                            &k->beta, &k->est, &k->fac, &k->it, &k->kc, &k->active, &k->done, &k->conv, &k->counter,
                            &k->skip, &k->extra})
      b += d->bytes;
  return b;
}

helm_status helm_last_timings(const helm_handle_t* H, double out[5]) {
  if (!H || !out) return fail(HELM_EINVAL, "null argument");
  out[0] = H->t_setup;
  out[1] = H->t_solve;
  out[2] = H->t_fact;
  out[3] = H->t_coarse;
  out[4] = H->its;
  return HELM_OK;
}

helm_status helm_solve_async(helm_handle_t* H, int32_t nrhs, const void* B, void* X, double tol, int32_t maxit,
                             uint32_t flags, int32_t* iters, double* relres_est, double* relres_true,
                             void* stream, helm_request_t** req) {
  return guarded([&]() {
    if (!H || !B || !X || !req || nrhs < 0 || !(tol >= 0) || maxit < 0)
      throw HelmError(HELM_EINVAL, "bad solve arguments");
    std::lock_guard<std::mutex> lk(H->pending_mu);
    if (H->pending) throw HelmError(HELM_EINVAL, "a solve is already in flight on this handle");
    auto q = std::make_unique<helm_request>();
    q->H = H;
    helm_request* qp = q.get();
    H->pending = qp;
    const hipStream_t on = stream ? (hipStream_t)stream : nullptr;
    try {
      qp->worker = std::thread([=]() {
        helm_status st;
        if (hipSetDevice(H->device) != hipSuccess) {
          (void)hipGetLastError();
          st = fail_h(H, HELM_EDEVICE, "hipSetDevice failed on the solve thread");
        } else {
          // the solve's device work goes to the caller's stream, if given (the
          // handle is busy meanwhile: no other call uses its stream)
          const hipStream_t keep = H->stream;
          if (on) H->stream = on;
          st = solve_impl(H, nrhs, B, X, tol, maxit, flags, iters, relres_est, relres_true);
          H->stream = keep;
        }
        if (st != HELM_OK && st != HELM_NOT_CONVERGED) qp->message = g_last_error;
        qp->status.store(st);
        qp->done.store(true);
      });
    } catch (...) {
      H->pending = nullptr;
      throw HelmError(HELM_EDEVICE, "could not start the solve thread");
    }
    *req = q.release();
    return HELM_OK;
  }, H);
}

helm_status helm_request_query(const helm_request_t* q) {
  if (!q) return fail(HELM_EINVAL, "null request");
  return q->done.load() ? (helm_status)q->status.load() : HELM_PENDING;
}

helm_status helm_request_wait(helm_request_t* q) {
  if (!q) return fail(HELM_EINVAL, "null request");
  if (helm_handle* H = q->H.load()) {  // else helm_destroy already joined the solve
    std::lock_guard<std::mutex> lk(H->pending_mu);
    if (!q->joined) {
      q->worker.join();
      q->joined = true;
    }
    if (H->pending == q) H->pending = nullptr;
  }
  const helm_status st = (helm_status)q->status.load();
  if (st != HELM_OK && st != HELM_NOT_CONVERGED) g_last_error = q->message;
  delete q;
  return st;
}

void helm_destroy(helm_handle_t* H) {
  if (!H) return;
  finish_pending(H);  // a request still owned by the caller stays valid for helm_request_wait
  // the handle's device work is ordered on its stream
  if (H->stream) (void)hipStreamSynchronize(H->stream);
  collect_sweep_timing(H);
  harvest_graphs(H);
  delete H;
}

size_t helm_trim_cache(void) {
  const size_t b = pool().cached_bytes();
  pool().trim();
  return b;
}

size_t helm_device_headroom(void) { return DevicePool::headroom_bytes(); }

helm_status helm_release_workspace(helm_handle_t* H) {
  return guarded([&]() {
    if (!H) throw HelmError(HELM_EINVAL, "null handle");
    if (busy(H)) throw HelmError(HELM_EINVAL, "a solve is in flight on this handle");
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    drop_graphs(H);
    ++H->ws_gen;
    H->ws.~Workspace();  // buffers go back to the device cache
    new (&H->ws) Workspace();
    return HELM_OK;
  }, H);
}

helm_status helm_set_sweep_timing(helm_handle_t* H, int32_t enable) {
  if (!H) return fail(HELM_EINVAL, "null handle");
  H->timing = enable != 0;
  for (int lv = 0; lv < NTIMED; ++lv)
    for (int i = 0; i < 4; ++i) H->sweep_stat[lv][i] = 0;
  return HELM_OK;
}

helm_status helm_set_graphs(helm_handle_t* H, int32_t enable) {
  if (!H) return fail(HELM_EINVAL, "null handle");
  return guarded([&]() {
    drop_graphs(H);
    H->graphs = enable != 0;
    return HELM_OK;
  }, H);
}

helm_status helm_set_sweep_policy(int32_t policy) {
  if (policy < 0 || policy > 6) return fail(HELM_EINVAL, "sweep policy must be 0, 1, 2, 3, 4, 5 or 6");
  set_sweep_policy(policy);
  return HELM_OK;
}

helm_status helm_set_row_tiling(int32_t nodes_per_thread) {
  if (!set_row_tiling(nodes_per_thread))
    return fail(HELM_EINVAL, "tiling must be 0, 2, 4, 8, HELM_TILE_MARCH | 2 or HELM_TILE_MARCH | 3");
  return HELM_OK;
}

helm_status helm_set_lu_panel(int32_t columns) {
  if (!set_lu_panel(columns)) return fail(HELM_EINVAL, "panel width must be 0, 4, 8 or 16");
  return HELM_OK;
}

helm_status helm_solve_bound(const helm_handle_t* H, double out[3]) {
  if (!H || !out) return fail(HELM_EINVAL, "null argument");
  out[0] = H->work_solve.seconds;
  out[1] = H->work_solve.bytes;
  out[2] = H->work_solve.flops;
  return HELM_OK;
}

helm_status helm_graph_stats(const helm_handle_t* H, double out[2]) {
  if (!H || !out) return fail(HELM_EINVAL, "null argument");
  out[0] = H->graph_stat[0];
  out[1] = H->graph_stat[1];
  return HELM_OK;
}

helm_status helm_sweep_stats(const helm_handle_t* H, int32_t level, double out[4]) {
  if (!H || !out || level < 0 || level > 1) return fail(HELM_EINVAL, "bad arguments");
  for (int i = 0; i < 4; ++i) out[i] = H->sweep_stat[level][i];
  return HELM_OK;
}

helm_status helm_sweep_config(const helm_handle_t* H, int32_t level, int32_t nrhs, int32_t out[4]) {
  if (!H || !out || level < 0 || level > (H->two_level() ? 1 : 0) || nrhs <= 0) return fail(HELM_EINVAL, "bad arguments");
  const Level& L = level == 0 ? H->fine : H->coarse;
  int v[4] = {0, 0, 0, 0};
  if (!tuned_config(L.half ? 2 : (int)elem_size(L.prec) / 2, L.bpmax, L.nsub, nrhs, L.nx, L.ny, v))
    for (int& x : v) x = 0;
  for (int i = 0; i < 4; ++i) out[i] = v[i];
  return HELM_OK;
}

helm_status helm_stencil_stats(const helm_handle_t* H, int32_t kind, double out[4]) {
  if (!H || !out || kind < 0 || kind > 1) return fail(HELM_EINVAL, "bad arguments");
  for (int i = 0; i < 4; ++i) out[i] = H->sweep_stat[2 + kind][i];
  return HELM_OK;
}

const char* helm_last_error(const helm_handle_t* H) {
  if (!H) return g_last_error.c_str();
  thread_local std::string copy;  // stable for the caller while the handle may fail again elsewhere
  std::lock_guard<std::mutex> lk(H->err_mu);
  copy = H->err_msg;
  return copy.c_str();
}

helm_status helm_set_stream(helm_handle_t* H, void* stream) {
  if (!H) return fail(HELM_EINVAL, "null handle");
  H->stream = stream ? (hipStream_t)stream : H->own;
  return HELM_OK;
}

}  // extern "C"

// ---- operator-level entry points -------------------------------------------

namespace {
template <typename F>
helm_status map_fields(helm_handle_t* H, int nrhs, long long len_in, long long len_out, const void* in, void* outp,
                       F&& body) {
  return guarded([&]() {
    if (!H || !in || !outp || nrhs < 1 || nrhs > 256) throw HelmError(HELM_EINVAL, "bad arguments");
    DevBuf fi, ni, no, fo;
    fi.alloc(sizeof(z64) * len_in * nrhs);
    ni.alloc(sizeof(z64) * len_in * nrhs);
    no.alloc(sizeof(z64) * len_out * nrhs);
    fo.alloc(sizeof(z64) * len_out * nrhs);
    HELM_CHECK_HIP(hipMemcpyAsync(fi.p, in, sizeof(z64) * len_in * nrhs, hipMemcpyDefault, H->stream));
    launch_to_node_major(fi.as<z64>(), ni.as<z64>(), len_in, nrhs, H->stream);
    body(ni.as<z64>(), no.as<z64>());
    launch_to_field_major(no.as<z64>(), fo.as<z64>(), len_out, nrhs, H->stream);
    HELM_CHECK_HIP(hipMemcpyAsync(outp, fo.p, sizeof(z64) * len_out * nrhs, hipMemcpyDefault, H->stream));
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    collect_sweep_timing(H);
    HELM_CHECK_HIP(hipGetLastError());
    return HELM_OK;
  }, H);
}
}  // namespace

extern "C" {

helm_status helm_apply_A(helm_handle_t* H, int32_t nrhs, const void* X, void* Y) {
  if (!H) return fail(HELM_EINVAL, "null handle");
  return map_fields(H, nrhs, H->n, H->n, X, Y, [&](const z64* x, z64* y) { launch_stencil(H->op, nrhs, x, y, H->stream); });
}

helm_status helm_apply_M(helm_handle_t* H, int32_t nrhs, const void* R, void* Z) {
  if (!H) return fail(HELM_EINVAL, "null handle");
  return map_fields(H, nrhs, H->n, H->n, R, Z, [&](const z64* r, z64* z) {
    ensure_ws(H, nrhs);
    precond(H, nrhs, r, z);
  });
}

helm_status helm_apply_oras(helm_handle_t* H, int32_t level, int32_t nrhs, const void* R, void* Z) {
  if (!H) return fail(HELM_EINVAL, "null handle");
  if (level != 0 && !(level == 1 && H->two_level())) return fail_h(H, HELM_EINVAL, "no such level");
  Level& L = level == 0 ? H->fine : H->coarse;
  return map_fields(H, nrhs, L.n, L.n, R, Z, [&](const z64* r, z64* z) {
    ensure_ws(H, nrhs);
    if (level == 0) oras_apply(H, L, nrhs, r, z, nullptr, H->ws.yl_f.p, H->ws.tb_f.p);
    else oras_apply(H, L, nrhs, r, z, nullptr, H->ws.yl_c.p, H->ws.tb_c.p);
  });
}

}  // extern "C"

// ---- the allocation-free one-level ORAS application ------------------------

namespace {
// Device scratch of helm_apply_oras_noalloc: node-major staging of R and Z and
// the sweep's plane vectors.  A file-scope device array, so each GPU the
// library runs on holds its own copy until the process ends.  In host code its
// name is not a device address: the address comes from hipGetSymbolAddress,
// once per device, and only that address reaches kernels and copies.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

void* scratch_on_current_device() {
  constexpr int MAXDEV = 64;
  static void* ptr[MAXDEV] = {};
  static std::mutex mu;
  int dev = 0;
  HELM_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAXDEV) throw HelmError(HELM_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw HelmError(HELM_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                        hipGetErrorString(e));
    ptr[dev] = p;
  }
  return ptr[dev];
}

bool on_device(const void* p) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

extern "C" {

helm_status helm_apply_oras_noalloc(helm_handle_t* H, int32_t level, int32_t nrhs, const void* R, void* Z) {
  return guarded([&]() {
    if (!H || !R || !Z || nrhs < 1 || nrhs > 256) throw HelmError(HELM_EINVAL, "bad arguments");
    if (level != 0 && !(level == 1 && H->two_level())) throw HelmError(HELM_EINVAL, "no such level");
    if (busy(H)) throw HelmError(HELM_EINVAL, "a solve is in flight on this handle");
    if (!on_device(R) || !on_device(Z)) throw HelmError(HELM_EINVAL, "R and Z must be device memory");
    Level& L = level == 0 ? H->fine : H->coarse;
    const size_t es = elem_size(L.prec);
    const size_t fld = align256(sizeof(z64) * (size_t)L.n * nrhs);
    const size_t yl = align256((size_t)L.vec_total * nrhs * es);
    const size_t tb = align256((size_t)sweep_tbuf_elems(L.nsub, L.bpmax, nrhs) * es);
    const size_t need = 2 * fld + yl + tb;
    if (need > NOALLOC_SCRATCH_BYTES)
      throw HelmError(HELM_EINVAL, "helm_apply_oras_noalloc needs " + std::to_string(need) +
                                       " bytes of scratch for this level and batch; the limit is " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES) + " (use helm_apply_oras)");
    char* base = static_cast<char*>(scratch_on_current_device());
    z64* ni = reinterpret_cast<z64*>(base);
    z64* no = reinterpret_cast<z64*>(base + fld);
    void* ylp = base + 2 * fld;
    void* tbp = base + 2 * fld + yl;
    launch_to_node_major(static_cast<const z64*>(R), ni, L.n, nrhs, H->stream);
    if (L.half) {
      if (!oras_half(L.d_subs.as<Sub>(), L.nsub, L.bpmax, L.cpl.as<c32>(), L.sinv16.as<uint4>(), L.sexp.as<int>(),
                     L.maxez, nrhs, ni, no, nullptr, L.nx, L.ny, (c32*)ylp, H->stream, false))
        throw HelmError(HELM_EINVAL, "approximate local solves do not fit this plane size");
    } else if (L.prec == 1)
      Factor<float>::sweep(L.d_subs.as<Sub>(), L.nsub, L.bpmax, L.maxez, L.cpl.as<c32>(), L.sinv.as<c32>(), nrhs, ni,
                           no, nullptr, L.nx, L.ny, (c32*)ylp, (c32*)tbp, H->stream, false);
    else
      Factor<double>::sweep(L.d_subs.as<Sub>(), L.nsub, L.bpmax, L.maxez, L.cpl.as<z64>(), L.sinv.as<z64>(), nrhs, ni,
                            no, nullptr, L.nx, L.ny, (z64*)ylp, (z64*)tbp, H->stream, false);
    launch_to_field_major(no, static_cast<z64*>(Z), L.n, nrhs, H->stream);
    HELM_CHECK_HIP(hipGetLastError());
    return HELM_OK;
  }, H);
}

helm_status helm_local_solve(helm_handle_t* H, int32_t level, int32_t s, int32_t nrhs, const void* R, void* X) {
  return guarded([&]() {
    if (!H || !R || !X || nrhs < 1 || nrhs > 256) throw HelmError(HELM_EINVAL, "bad arguments");
    if (level != 0 && !(level == 1 && H->two_level())) throw HelmError(HELM_EINVAL, "no such level");
    Level& L = level == 0 ? H->fine : H->coarse;
    if (s < 0 || s >= L.nsub) throw HelmError(HELM_EINVAL, "no such subdomain");
    const Sub& sb = L.subs[s];
    const long long nloc = (long long)sb.b * sb.ez;
    ensure_ws(H, nrhs);
    DevBuf fi, ni, u, zg, xo, fo;
    fi.alloc(sizeof(z64) * nloc * nrhs);
    ni.alloc(sizeof(z64) * nloc * nrhs);
    xo.alloc(sizeof(z64) * nloc * nrhs);
    fo.alloc(sizeof(z64) * nloc * nrhs);
    u.alloc(sizeof(z64) * L.n * nrhs);
    zg.alloc(sizeof(z64) * L.n * nrhs);
    HELM_CHECK_HIP(hipMemcpyAsync(fi.p, R, sizeof(z64) * nloc * nrhs, hipMemcpyDefault, H->stream));
    launch_to_node_major(fi.as<z64>(), ni.as<z64>(), nloc, nrhs, H->stream);
    launch_fill(u.as<z64>(), L.n * nrhs, H->stream);
    launch_box_scatter(sb, L.nx, L.ny, nrhs, ni.as<z64>(), u.as<z64>(), H->stream);
    void* yl = level == 0 ? H->ws.yl_f.p : H->ws.yl_c.p;
    void* tb = level == 0 ? H->ws.tb_f.p : H->ws.tb_c.p;
    const Sub* one = L.d_subs.as<Sub>() + s;
    if (L.half) {
      if (!oras_half(one, 1, L.bpmax, L.cpl.as<c32>(), L.sinv16.as<uint4>(), L.sexp.as<int>(),  // indexed by Sub::id
                     L.maxez, nrhs, u.as<z64>(), zg.as<z64>(), nullptr, L.nx, L.ny, (c32*)yl, H->stream))
        throw HelmError(HELM_EINVAL, "approximate local solves do not fit this plane size");
      launch_box_gather<float>(sb, nrhs, (const c32*)yl, xo.as<z64>(), H->stream);
    } else if (L.prec == 1) {
      Factor<float>::sweep(one, 1, L.bpmax, sb.ez, L.cpl.as<c32>(), L.sinv.as<c32>(), nrhs, u.as<z64>(), zg.as<z64>(),
                           nullptr, L.nx, L.ny, (c32*)yl, (c32*)tb, H->stream);
      launch_box_gather<float>(sb, nrhs, (const c32*)yl, xo.as<z64>(), H->stream);
    } else {
      Factor<double>::sweep(one, 1, L.bpmax, sb.ez, L.cpl.as<z64>(), L.sinv.as<z64>(), nrhs, u.as<z64>(),
                            zg.as<z64>(), nullptr, L.nx, L.ny, (z64*)yl, (z64*)tb, H->stream);
      launch_box_gather<double>(sb, nrhs, (const z64*)yl, xo.as<z64>(), H->stream);
    }
    launch_to_field_major(xo.as<z64>(), fo.as<z64>(), nloc, nrhs, H->stream);
    HELM_CHECK_HIP(hipMemcpyAsync(X, fo.p, sizeof(z64) * nloc * nrhs, hipMemcpyDefault, H->stream));
    HELM_CHECK_HIP(hipStreamSynchronize(H->stream));
    HELM_CHECK_HIP(hipGetLastError());
    return HELM_OK;
  }, H);
}

helm_status helm_restrict(helm_handle_t* H, int32_t nrhs, const void* R, void* C) {
  if (!H || !H->two_level()) return fail(HELM_EINVAL, "two-level handle required");
  return map_fields(H, nrhs, H->n, H->coarse.n, R, C,
                    [&](const z64* r, z64* c) { launch_restrict(H->nx, H->ny, H->nz, nrhs, r, c, H->stream); });
}

helm_status helm_prolong(helm_handle_t* H, int32_t nrhs, const void* C, void* R) {
  if (!H || !H->two_level()) return fail(HELM_EINVAL, "two-level handle required");
  return map_fields(H, nrhs, H->coarse.n, H->n, C, R,
                    [&](const z64* c, z64* r) { launch_prolong(H->nx, H->ny, H->nz, nrhs, c, r, H->stream); });
}

helm_status helm_apply_E(helm_handle_t* H, int32_t nrhs, const void* X, void* Y) {
  if (!H || !H->two_level()) return fail(HELM_EINVAL, "two-level handle required");
  return map_fields(H, nrhs, H->coarse.n, H->coarse.n, X, Y, [&](const z64* x, z64* y) { coarse_spmv(H, nrhs, x, y); });
}

helm_status helm_apply_Q(helm_handle_t* H, int32_t nrhs, const void* R, void* Q) {
  if (!H || !H->two_level()) return fail(HELM_EINVAL, "two-level handle required");
  return map_fields(H, nrhs, H->n, H->n, R, Q, [&](const z64* r, z64* q) {
    ensure_ws(H, nrhs);
    coarse_correction(H, nrhs, r, q);
  });
}

int32_t helm_num_subdomains(const helm_handle_t* H, int32_t level) {
  if (!H) return 0;
  if (level == 0) return H->fine.nsub;
  if (level == 1 && H->two_level()) return H->coarse.nsub;
  return 0;
}

helm_status helm_subdomain_box(const helm_handle_t* H, int32_t level, int32_t s, int32_t box[12]) {
  if (!H || !box) return fail(HELM_EINVAL, "null argument");
  const Level* L = level == 0 ? &H->fine : (level == 1 && H->two_level() ? &H->coarse : nullptr);
  if (!L || s < 0 || s >= L->nsub) return fail(HELM_EINVAL, "no such subdomain");
  const Sub& b = L->subs[s];
  for (int d = 0; d < 3; ++d) {
    box[d] = b.elo[d];
    box[3 + d] = b.ehi[d];
    box[6 + d] = b.lo[d];
    box[9 + d] = b.hi[d];
  }
  return HELM_OK;
}

}  // extern "C"
