// Fused local solves of the ORAS preconditioner (eq. oras) on matrix cores.
//
// One workgroup owns one subdomain and one group of RG right-hand sides and
// runs the whole block-tridiagonal solve in a single launch:
//   forward   T_k = R_i u (plane k) - L_k y_{k-1};  y_k = Sinv_k T_k
//   backward  T   = U_k x_{k+1};                    x_k = y_k - Sinv_k T
// then scatters the core nodes of x (Boolean partition of unity), optionally
// adding a second field.  The plane vector lives in LDS; the dense products
// Sinv_k T stream Sinv_k from HBM through MFMA 16x16x4 tiles (operand lanes:
// A[l%16][l/16], B[l/16][l%16]; output rows differ between f32 and f64).
//
// Complex products on real MFMA: with Sinv stored interleaved (re, im) it is a
// real bp x 2bp matrix A; the plane vector T (bp x RG complex) is expanded on
// the fly into the real 2bp x 2RG matrix
//   B[2q][2r] = Re T[q][r]    B[2q][2r+1] = Im T[q][r]
//   B[2q+1][2r] = -Im T[q][r] B[2q+1][2r+1] = Re T[q][r]
// so that A B is the interleaved complex product (4 real products, one pass).
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "kernels.h"

namespace {

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output element v of lane group lg (lane / 16) sits in tile row 4 lg + v
  static __device__ __forceinline__ int row(int lg, int v) { return 4 * lg + v; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the f64 variant interleaves its rows: element v of lane group lg is tile row lg + 4 v
  static __device__ __forceinline__ int row(int lg, int v) { return lg + 4 * v; }
};


// Make this workgroup's global stores visible to its other waves.
__device__ __forceinline__ void wg_sync_global() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// First PF chunks of Sinv_k for the wave's first 16-row tile; they do not
// depend on the plane operand, so they are issued before T is built.
template <typename T, int PF>
__device__ __forceinline__ void prefetch_tile(const cpx<T>* __restrict__ Sk, int bp, int wave, int lane,
                                              cpx<T> (&a)[PF][4]) {
  const int nmt = bp >> 4;
  if (wave >= nmt) return;
  const cpx<T>* Arow = Sk + (long long)(wave * 16 + (lane & 15)) * bp + 4 * (lane >> 4);
#pragma unroll
  for (int j = 0; j < PF; ++j)
    if (16 * j < bp)
#pragma unroll
      for (int t = 0; t < 4; ++t) a[j][t] = Arow[16 * j + t];
}

// Rows of the wave's M-tiles of Sinv_k x Bs (Bs = T, [bp][RG] in LDS), one
// 16-row tile at a time, with PF chunks of Sinv in flight per wave (the first
// tile's initial chunks arrive pre-loaded in a); out(p, r, nb, value)
// receives each real output entry.
template <typename T, int RG, int PF, typename Out>
__device__ __forceinline__ void plane_product(const cpx<T>* __restrict__ Sk, int bp, const cpx<T>* Bs, int wave,
                                              int nwaves, int lane, cpx<T> (&a)[PF][4], Out&& out) {
  using V4 = typename Mfma<T>::v4;
  constexpr int NT = RG / 8;  // MFMA column tiles (16 real columns = 8 complex)
  const int lrow = lane & 15, lg = lane >> 4, nb = lane & 1;
  const int nmt = bp >> 4;
  const cpx<T>* Bcol = Bs + 4 * lg * RG + (lrow >> 1);
  for (int mt = wave; mt < nmt; mt += nwaves) {
    V4 acc[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = V4{0, 0, 0, 0};
    const cpx<T>* Arow = Sk + (long long)(mt * 16 + lrow) * bp + 4 * lg;
    if (mt != wave) {
#pragma unroll
      for (int j = 0; j < PF; ++j)
        if (16 * j < bp)
#pragma unroll
          for (int t = 0; t < 4; ++t) a[j][t] = Arow[16 * j + t];
    }
    for (int kc0 = 0; kc0 < bp; kc0 += 16 * PF) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        const int kc = kc0 + 16 * j;
        if (kc < bp) {
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            cpx<T> tv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) tv[t] = Bcol[(kc + t) * RG + nt * 8];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              acc[nt] = Mfma<T>::op(a[j][t].re, nb ? tv[t].im : tv[t].re, acc[nt]);
              acc[nt] = Mfma<T>::op(a[j][t].im, nb ? tv[t].re : -tv[t].im, acc[nt]);
            }
          }
          const int kn = kc + 16 * PF;
          if (kn < bp)
#pragma unroll
            for (int t = 0; t < 4; ++t) a[j][t] = Arow[kn + t];
        }
      }
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) out(mt * 16 + Mfma<T>::row(lg, v), nt * 8 + ((lane & 15) >> 1), nb, acc[nt][v]);
  }
}

// LDS holds only the right operand T of the plane product ([bp][RG]); the
// plane solutions y_k / x_k live in yloc and reach the other waves of the
// workgroup through L2 (workgroup-scope release/acquire around the barrier).
template <typename T, int RG, int PF>
__global__ void __launch_bounds__(1024) k_oras_fused(const Sub* __restrict__ subs, int ngroups, int nrhs,
                                                   const z64* __restrict__ aloc, const cpx<T>* __restrict__ sinv,
                                                   const z64* __restrict__ u, z64* __restrict__ z,
                                                   const z64* __restrict__ add, int gnx, int gny,
                                                   cpx<T>* __restrict__ yloc) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* Bs = reinterpret_cast<cpx<T>*>(smem_raw);
  const int s = blockIdx.x / ngroups, g = blockIdx.x % ngroups;
  const Sub sb = subs[s];
  const int r0 = g * RG;
  const int nrg = min(RG, nrhs - r0);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int FT = blockDim.x, nwaves = FT >> 6;
  const int bp = sb.bp, b = sb.b, ex = sb.ex, ey = sb.ey, ez = sb.ez;
  const int cx0 = sb.lo[0] - sb.elo[0], cx1 = sb.hi[0] - sb.elo[0];
  const int cy0 = sb.lo[1] - sb.elo[1], cy1 = sb.hi[1] - sb.elo[1];
  const int cz0 = sb.lo[2] - sb.elo[2], cz1 = sb.hi[2] - sb.elo[2];
  cpx<T>* yb = yloc + sb.vec_off * (long long)nrhs + r0;  // plane k, row p, column r at (k*bp + p)*nrhs + r
  T* yr = reinterpret_cast<T*>(yb);
  double* zr = reinterpret_cast<double*>(z);
  const double* ar = reinterpret_cast<const double*>(add);

  auto gnode = [&](int k, int p) -> long long {
    const int px = p % ex, py = p / ex;
    return (sb.elo[0] + px) + (long long)gnx * ((sb.elo[1] + py) + (long long)gny * (sb.elo[2] + k));
  };
  // coupling of plane k to plane kn = k + dz (dz = -1: L_k, +1: U_k) applied to the stored plane kn
  auto couple = [&](int k, int p, int r, int dz) -> cpx<T> {
    const int px = p % ex, py = p / ex;
    const z64* row = aloc + (sb.node_off + (long long)k * b + p) * 27 + (dz + 1) * 9;
    const cpx<T>* yn = yb + (long long)(k + dz) * bp * nrhs + r;
    cpx<T> v = mk<T>(0, 0);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int cy = py + dy;
      if (cy < 0 || cy >= ey) continue;
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int cx = px + dx;
        if (cx < 0 || cx >= ex) continue;
        cfma(v, ccast<T>(row[(dy + 1) * 3 + (dx + 1)]), yn[(long long)(cx + ex * cy) * nrhs]);
      }
    }
    return v;
  };
  // core node (k, p) of the box: z = x (+ add), one real component per lane
  auto scatter = [&](int k, int p, int r, int nb, T val) {
    if (k < cz0 || k >= cz1 || p >= b || r >= nrg) return;
    const int px = p % ex, py = p / ex;
    if (px < cx0 || px >= cx1 || py < cy0 || py >= cy1) return;
    const long long gi = (gnode(k, p) * nrhs + r0 + r) * 2 + nb;
    zr[gi] = (double)val + (ar ? ar[gi] : 0.0);
  };

  cpx<T> a[PF][4];
  // ---- forward sweep: y_k = Sinv_k (R_i u - L_k y_{k-1})
  for (int k = 0; k < ez; ++k) {
    const cpx<T>* Sk = sinv + sb.mat_off + (long long)k * bp * bp;
    prefetch_tile<T, PF>(Sk, bp, wave, lane, a);
    auto tf = [&](int e) -> cpx<T> {
      const int p = e / RG, r = e % RG;
      cpx<T> v = mk<T>(0, 0);
      if (p < b && r < nrg) {
        v = ccast<T>(u[gnode(k, p) * nrhs + r0 + r]);
        if (k > 0) v = v - couple(k, p, r, -1);
      }
      return v;
    };
    for (int e = tid; e < bp * RG; e += 2 * FT) {
      const cpx<T> v0 = tf(e);
      const bool two = e + FT < bp * RG;
      const cpx<T> v1 = two ? tf(e + FT) : mk<T>(0, 0);
      Bs[e] = v0;
      if (two) Bs[e + FT] = v1;
    }
    __syncthreads();
    const bool last = k == ez - 1;
    plane_product<T, RG, PF>(Sk, bp, Bs, wave, nwaves, lane, a, [&](int p, int r, int nb, T val) {
      if (r < nrg) yr[(((long long)k * bp + p) * nrhs + r) * 2 + nb] = val;
      if (last) scatter(k, p, r, nb, val);  // x_{ez-1} = y_{ez-1}
    });
    wg_sync_global();
  }
  // ---- backward sweep: x_k = y_k - Sinv_k U_k x_{k+1}, x_k overwrites y_k
  for (int k = ez - 2; k >= 0; --k) {
    const cpx<T>* Sk = sinv + sb.mat_off + (long long)k * bp * bp;
    prefetch_tile<T, PF>(Sk, bp, wave, lane, a);
    auto tb = [&](int e) -> cpx<T> {
      const int p = e / RG, r = e % RG;
      return (p < b && r < nrg) ? couple(k, p, r, +1) : mk<T>(0, 0);
    };
    for (int e = tid; e < bp * RG; e += 2 * FT) {
      const cpx<T> v0 = tb(e);
      const bool two = e + FT < bp * RG;
      const cpx<T> v1 = two ? tb(e + FT) : mk<T>(0, 0);
      Bs[e] = v0;
      if (two) Bs[e + FT] = v1;
    }
    __syncthreads();
    plane_product<T, RG, PF>(Sk, bp, Bs, wave, nwaves, lane, a, [&](int p, int r, int nb, T val) {
      if (r >= nrg) return;
      T* yp = yr + (((long long)k * bp + p) * nrhs + r) * 2 + nb;
      const T x = *yp - val;
      *yp = x;
      scatter(k, p, r, nb, x);
    });
    wg_sync_global();
  }
}

template <typename T, int RG>
void launch_fused_t(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, const z64* aloc,
                    const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc,
                    hipStream_t s) {
  constexpr int PF = sizeof(T) == 4 ? 4 : 2;
  const size_t lds = (size_t)bpmax * RG * sizeof(cpx<T>);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_oras_fused<T, RG, PF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
  }
  // waves per workgroup: as few rounds of 16-row tiles as 16 waves allow, evenly spread
  const int nmt = bpmax / 16;
  const int rounds = (nmt + 15) / 16;
  const int nwaves = (nmt + rounds - 1) / rounds;
  hipLaunchKernelGGL((k_oras_fused<T, RG, PF>), dim3(nsub * ngroups), dim3(64 * nwaves), lds, s, subs, ngroups, nrhs, aloc,
                     sinv, u, z, add, gnx, gny, yloc);
}

}  // namespace

// LDS budget of the fused kernel (one plane operand)
constexpr size_t FUSED_LDS = 150 * 1024;

template <typename T>
int fused_group(int bpmax, int nrhs) {
  int rg = nrhs <= 8 ? 8 : (nrhs <= 16 ? 16 : 32);
  while (rg >= 8 && (size_t)bpmax * rg * sizeof(cpx<T>) > FUSED_LDS) rg /= 2;
  return rg >= 8 ? rg : 0;
}

namespace {

template <typename T>
void launch_rg(int rg, const Sub* subs, int nsub, int nrhs, int bpmax, const z64* aloc, const cpx<T>* sinv,
               const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc, hipStream_t s) {
  const int ngroups = (nrhs + rg - 1) / rg;
  switch (rg) {
    case 8: launch_fused_t<T, 8>(subs, nsub, ngroups, nrhs, bpmax, aloc, sinv, u, z, add, gnx, gny, yloc, s); break;
    case 16: launch_fused_t<T, 16>(subs, nsub, ngroups, nrhs, bpmax, aloc, sinv, u, z, add, gnx, gny, yloc, s); break;
    default: launch_fused_t<T, 32>(subs, nsub, ngroups, nrhs, bpmax, aloc, sinv, u, z, add, gnx, gny, yloc, s); break;
  }
}

// Autotuned right-hand-side group of the fused sweep, per problem shape.
struct TuneKey {
  int es, bpmax, nsub, nrhs, gnx, gny;
  bool operator<(const TuneKey& o) const {
    return std::tie(es, bpmax, nsub, nrhs, gnx, gny) < std::tie(o.es, o.bpmax, o.nsub, o.nrhs, o.gnx, o.gny);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

}  // namespace

int tuned_group(int es, int bpmax, int nsub, int nrhs, int gnx, int gny) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({es, bpmax, nsub, nrhs, gnx, gny});
  return it == g_tune.end() ? 0 : it->second;
}

template <typename T>
bool oras_fused(const Sub* subs, int nsub, int bpmax, const z64* aloc, const cpx<T>* sinv, int nrhs, const z64* u,
                z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc, hipStream_t s) {
  const int rgmax = fused_group<T>(bpmax, nrhs);
  if (rgmax == 0) return false;
  const TuneKey key{(int)sizeof(T), bpmax, nsub, nrhs, gnx, gny};
  int rg = 0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) rg = it->second;
  }
  static const bool no_tune = std::getenv("HELM_NO_TUNE") != nullptr;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  if (rg == 0 && !no_tune && cap == hipStreamCaptureStatusNone && rgmax > 8) {
    // time every admissible group size twice on this very input (the sweep is
    // idempotent: z and the scratch planes are overwritten) and keep the fastest
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    for (int cand = 8; cand <= rgmax; cand *= 2) {
      float tot = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        (void)hipEventRecord(e0, s);
        launch_rg<T>(cand, subs, nsub, nrhs, bpmax, aloc, sinv, u, z, add, gnx, gny, yloc, s);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) tot += ms;
      }
      if (tot < best) {
        best = tot;
        rg = cand;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = rg;
  }
  if (rg == 0) rg = rgmax;
  launch_rg<T>(rg, subs, nsub, nrhs, bpmax, aloc, sinv, u, z, add, gnx, gny, yloc, s);
  return true;
}

template bool oras_fused<float>(const Sub*, int, int, const z64*, const c32*, int, const z64*, z64*, const z64*, int,
                                int, c32*, hipStream_t);
template bool oras_fused<double>(const Sub*, int, int, const z64*, const z64*, int, const z64*, z64*, const z64*, int,
                                 int, z64*, hipStream_t);
template int fused_group<float>(int, int);
template int fused_group<double>(int, int);
