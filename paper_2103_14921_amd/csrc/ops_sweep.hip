// Fused local solves of the ORAS preconditioner (eq. oras) on matrix cores.
//
// One workgroup owns one subdomain and one group of RG right-hand sides and
// runs the whole block-tridiagonal solve in a single launch:
//   forward   T_k = R_i u (plane k) - L_k y_{k-1};  y_k = Sinv_k T_k
//   backward  T   = -U_k x_{k+1};                   x_k = y_k + Sinv_k T
// then scatters the core nodes of x (Boolean partition of unity), optionally
// adding a second field.  The plane vector lives in LDS; the dense products
// Sinv_k T stream Sinv_k from HBM through MFMA 16x16x4 tiles (operand lanes:
// A[l%16][l/16], B[l/16][l%16]; output rows differ between f32 and f64).
//
// Complex products on real MFMA: Sinv is stored interleaved (re, im), so each
// lane's A operand yields Re S and Im S together; the product is formed from
// real 16x16x4 steps as described at plane_product (no complex arithmetic and
// no lane-dependent operand selection inside the MFMA loop).
#include <algorithm>
#include <cstdio>
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

// Row width (in complex elements) of the plane operand in LDS.  RG >= 16 keeps
// T itself ([bp][RG], plus 4 elements of padding in complex FP32 so that the
// four lane groups of a read fall in different bank halves).  RG = 8 keeps the
// lane-ready split form [bp][16] described at plane_product.
template <typename T>
__host__ __device__ constexpr int lds_width(int rg) {
  return rg >= 16 ? rg + (sizeof(T) == 4 ? 4 : 0) : 16;
}

// The chunks of Sinv_k a wave reads, in order: its tiles mt = wave, wave +
// nwaves, ... (16 rows each), each cut into bp / 16 chunks of 16 columns.  The
// stream runs across tile boundaries, so the loads of the next tile's first
// chunks are in flight while the current tile finishes; past the end it
// repeats the last chunk (a harmless, always valid address), so every load is
// unconditional and the compiler can wait on exact counts.
template <typename T>
struct ChunkStream {
  const cpx<T>* base;  // row (wave*16 + lane%16), column 4*(lane/16) of Sk
  long long tile_step;  // elements between the wave's consecutive tiles
  int nct, ntw, tile, chunk;
  __device__ __forceinline__ ChunkStream(const cpx<T>* Sk, int bp, int wave, int nwaves, int lane) {
    const int nmt = bp >> 4;
    nct = nmt;
    ntw = wave < nmt ? (nmt - wave + nwaves - 1) / nwaves : 0;
    base = Sk + (long long)(min(wave, nmt - 1) * 16 + (lane & 15)) * bp + 4 * (lane >> 4);
    tile_step = (long long)nwaves * 16 * bp;
    tile = 0;
    chunk = 0;
  }
  __device__ __forceinline__ void next(cpx<T> (&dst)[4]) {
    const bool past = tile >= ntw;
    const cpx<T>* p = base + (past ? (long long)(ntw > 0 ? ntw - 1 : 0) * tile_step + 16 * (nct - 1)
                                   : (long long)tile * tile_step + 16 * chunk);
#pragma unroll
    for (int t = 0; t < 4; ++t) dst[t] = p[t];
    if (++chunk == nct) {
      chunk = 0;
      ++tile;
    }
  }
};

// Start a wave's chunk stream: the first PF chunks, issued before the barrier
// that publishes the plane operand.
template <typename T, int PF>
__device__ __forceinline__ ChunkStream<T> prefetch_tile(const cpx<T>* __restrict__ Sk, int bp, int wave, int nwaves,
                                                        int lane, cpx<T> (&a)[PF][4]) {
  ChunkStream<T> cs(Sk, bp, wave, nwaves, lane);
#pragma unroll
  for (int j = 0; j < PF; ++j) cs.next(a[j]);
  return cs;
}

// Rows of the wave's M-tiles of Sinv_k x T (T = plane operand in LDS): the
// wave walks its chunk stream with PF chunks in flight.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16] of each 16x16x4 step; chunk c, step t covers
// column 16 c + 4 (l/16) + t of Sinv_k.
//
// RG >= 16 (planar): each 16-column tile of complex right-hand sides keeps a
// real and an imaginary accumulator,
//   Re C += Re S Re T - Im S Im T,   Im C += Re S Im T + Im S Re T,
// four real MFMAs per step whose B operands are read straight from T.
// RG = 8 (split): one accumulator whose columns 0..7 hold Re C and 8..15 Im C;
// with B1 = [Re T | Im T] and B2 = [-Im T | Re T],  C = Re S B1 + Im S B2.  The
// operand pair (B1, B2) of each lane is stored ready in LDS, so no lane selects
// or negates anything inside the loop.
// Each tile's accumulators start from init(p, r); out(p, r, value) receives
// each complex output entry (row p, column r).
template <typename T, int RG, int PF, typename Init, typename Out>
__device__ __forceinline__ void plane_product(ChunkStream<T>& cs, const cpx<T>* Bs, int wave, int nwaves, int lane,
                                              cpx<T> (&a)[PF][4], Init&& init, Out&& out) {
  using V4 = typename Mfma<T>::v4;
  constexpr int W = lds_width<T>(RG);
  constexpr int NT = RG >= 16 ? RG / 16 : 1;  // 16-column MFMA tiles
  constexpr int NACC = RG >= 16 ? 2 : 1;
  const int lrow = lane & 15, lg = lane >> 4;
  const int nct = cs.nct, total = cs.ntw * cs.nct;
  const cpx<T>* Bcol = Bs + 4 * lg * W + lrow;
  V4 acc[NT][NACC];
  int mt = wave, kc = 0;
  for (int c0 = 0; c0 < total; c0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      if (c0 + j < total) {
        if (kc == 0) {  // accumulators start from init(p, r) (zero, or y_k in the backward sweep)
          if constexpr (RG >= 16) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const cpx<T> y0 = init(mt * 16 + Mfma<T>::row(lg, v), nt * 16 + lrow);
                acc[nt][0][v] = y0.re;
                acc[nt][1][v] = y0.im;
              }
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const cpx<T> y0 = init(mt * 16 + Mfma<T>::row(lg, v), lrow & 7);
              acc[0][0][v] = lrow < 8 ? y0.re : y0.im;
            }
          }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const T are = a[j][t].re, aim = a[j][t].im;
          if constexpr (RG >= 16) {
            const T naim = -aim;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
              const cpx<T> tv = Bcol[(kc + t) * W + nt * 16];
              acc[nt][0] = Mfma<T>::op(are, tv.re, acc[nt][0]);
              acc[nt][1] = Mfma<T>::op(are, tv.im, acc[nt][1]);
              acc[nt][0] = Mfma<T>::op(naim, tv.im, acc[nt][0]);
              acc[nt][1] = Mfma<T>::op(aim, tv.re, acc[nt][1]);
            }
          } else {
            const cpx<T> tv = Bcol[(kc + t) * W];  // (B1, B2) of this lane
            acc[0][0] = Mfma<T>::op(are, tv.re, acc[0][0]);
            acc[0][0] = Mfma<T>::op(aim, tv.im, acc[0][0]);
          }
        }
        kc += 16;
        if (kc == 16 * nct) {
          if constexpr (RG >= 16) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                out(mt * 16 + Mfma<T>::row(lg, v), nt * 16 + lrow, mk<T>(acc[nt][0][v], acc[nt][1][v]));
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const T im = __shfl_xor(acc[0][0][v], 8);  // column lrow + 8 holds Im of column lrow
              if (lrow < 8) out(mt * 16 + Mfma<T>::row(lg, v), lrow, mk<T>(acc[0][0][v], im));
            }
          }
          kc = 0;
          mt += nwaves;
        }
      }
      cs.next(a[j]);  // chunk c0 + j + PF (unconditional)
    }
  }
}

// Store entry (p, r) of the plane operand in the layout plane_product reads.
template <typename T, int RG>
__device__ __forceinline__ void put_operand(cpx<T>* Bs, int p, int r, cpx<T> v) {
  constexpr int W = lds_width<T>(RG);
  if constexpr (RG >= 16) {
    Bs[p * W + r] = v;
  } else {
    Bs[p * W + r] = mk<T>(v.re, -v.im);     // lane r:     B1 = Re T, B2 = -Im T
    Bs[p * W + r + 8] = mk<T>(v.im, v.re);  // lane r + 8: B1 = Im T, B2 = Re T
  }
}

// LDS holds only the right operand T of the plane product; the plane solutions
// y_k / x_k live in yloc and reach the other waves of the workgroup through L2
// (workgroup-scope release/acquire around the barrier).
// Waves per workgroup at most: 12 in FP64 (three per SIMD leave 168 registers
// for the operand build and the product), 16 in FP32.
template <typename T>
constexpr int fused_max_waves() {
  return sizeof(T) == 8 ? 12 : 16;
}

template <typename T, int RG, int PF>
__global__ void __launch_bounds__(64 * fused_max_waves<T>()) k_oras_fused(const Sub* __restrict__ subs, int ngroups, int nrhs,
                                                   const cpx<T>* __restrict__ cpl, const cpx<T>* __restrict__ sinv,
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

  auto gnode = [&](int k, int p) -> long long {
    const int px = p % ex, py = p / ex;
    return (sb.elo[0] + px) + (long long)gnx * ((sb.elo[1] + py) + (long long)gny * (sb.elo[2] + k));
  };
  // Operand build: each thread handles NE columns r, r + LP, ... of one node p
  // (LP = RG / NE lanes per node), so the nine coupling coefficients are loaded
  // once for NE entries.  All loads of an entry group are issued before any is
  // used: indices are clamped into the box (and columns into the batch) and
  // the coefficients of clamped taps are zero.  Bases are wave-uniform and
  // offsets 32-bit (plane vectors of a box stay far below 2^31 elements).
  constexpr int NE = sizeof(T) == 8 ? 1 : 2, LP = RG / NE;
  const cpx<T>* __restrict__ cbox = cpl + sb.node_off * 18;
  // v[j] = (u_k - L_k y_{k-1}) (dz = -1, with_u) or U_k x_{k+1} (dz = +1) at (p, r + j LP)
  auto build = [&](int k, int p, int r, int dz, bool with_u, cpx<T> (&v)[NE]) {
#pragma unroll
    for (int j = 0; j < NE; ++j) v[j] = mk<T>(0, 0);
    if (p >= b) return;
    int col[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) col[j] = min(r + j * LP, nrg - 1);
    if (with_u) {
      const long long gu = gnode(k, p) * nrhs + r0;
#pragma unroll
      for (int j = 0; j < NE; ++j) v[j] = ccast<T>(u[gu + col[j]]);
    }
    if (k + dz < 0 || k + dz >= ez) return;
    const int px = p % ex, py = p / ex;
    const int ro = (k * b + p) * 18 + (dz + 1) / 2 * 9;
    const int yo = (k + dz) * bp * nrhs;
    cpx<T> cv[9];
    cpx<T> yv[9][NE];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int cx = px + i % 3 - 1, cy = py + i / 3 - 1;
      const bool in = cx >= 0 && cx < ex && cy >= 0 && cy < ey;  // taps leaving the box have zero coefficients
      const int q = yo + (in ? cx + ex * cy : p) * nrhs;
      cv[i] = cbox[ro + i];
#pragma unroll
      for (int j = 0; j < NE; ++j) yv[i][j] = yb[q + col[j]];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i)
#pragma unroll
      for (int j = 0; j < NE; ++j) cfms(v[j], cv[i], yv[i][j]);
  };
  auto build_plane = [&](int k, int dz, bool with_u) {
#pragma unroll 1
    for (int e = tid; e < bp * LP; e += FT) {
      const int p = e / LP, r = e % LP;
      cpx<T> v[NE];
      build(k, p, r, dz, with_u, v);
#pragma unroll
      for (int j = 0; j < NE; ++j) put_operand<T, RG>(Bs, p, r + j * LP, r + j * LP < nrg ? v[j] : mk<T>(0, 0));
    }
  };
  // core node (k, p) of the box: z = x (+ add)
  auto scatter = [&](int k, int p, int r, cpx<T> val) {
    if (k < cz0 || k >= cz1 || p >= b || r >= nrg) return;
    const int px = p % ex, py = p / ex;
    if (px < cx0 || px >= cx1 || py < cy0 || py >= cy1) return;
    const long long gi = gnode(k, p) * nrhs + r0 + r;
    z64 o = ccast<double>(val);
    if (add) o += add[gi];
    z[gi] = o;
  };

  // ---- forward sweep: y_k = Sinv_k (R_i u - L_k y_{k-1})
  for (int k = 0; k < ez; ++k) {
    const cpx<T>* Sk = sinv + sb.mat_off + (long long)k * bp * bp;
    build_plane(k, -1, true);
    cpx<T> a[PF][4];  // per plane, so nothing stays live across the operand build
    ChunkStream<T> cs = prefetch_tile<T, PF>(Sk, bp, wave, nwaves, lane, a);  // in flight across the barrier
    __syncthreads();
    const bool last = k == ez - 1;
    plane_product<T, RG, PF>(
        cs, Bs, wave, nwaves, lane, a, [](int, int) { return mk<T>(0, 0); },
        [&](int p, int r, cpx<T> val) {
          if (r < nrg) yb[((long long)k * bp + p) * nrhs + r] = val;
          if (last) scatter(k, p, r, val);  // x_{ez-1} = y_{ez-1}
        });
    wg_sync_global();
  }
  // ---- backward sweep: x_k = y_k - Sinv_k U_k x_{k+1}, x_k overwrites y_k
  for (int k = ez - 2; k >= 0; --k) {
    const cpx<T>* Sk = sinv + sb.mat_off + (long long)k * bp * bp;
    build_plane(k, +1, false);
    cpx<T> a[PF][4];
    ChunkStream<T> cs = prefetch_tile<T, PF>(Sk, bp, wave, nwaves, lane, a);  // in flight across the barrier
    __syncthreads();
    // x_k = y_k + Sinv_k T (the operand holds -U_k x_{k+1}): the accumulators
    // start from y_k (column clamped into the group, always a valid address)
    plane_product<T, RG, PF>(
        cs, Bs, wave, nwaves, lane, a,
        [&](int p, int r) { return yb[((long long)k * bp + p) * nrhs + min(r, nrg - 1)]; },
        [&](int p, int r, cpx<T> x) {
          if (r >= nrg) return;
          yb[((long long)k * bp + p) * nrhs + r] = x;
          scatter(k, p, r, x);
        });
    wg_sync_global();
  }
}
// Rounds of 16-row tiles per wave: at least enough for the wave limit; more
// rounds mean fewer waves per workgroup, so that two workgroups (two boxes) can
// share a compute unit and overlap one's operand build with the other's product.
template <typename T>
int min_rounds(int bpmax) {
  constexpr int MW = fused_max_waves<T>();
  return (bpmax / 16 + MW - 1) / MW;
}

template <typename T, int RG>
void launch_fused_t(const Sub* subs, int nsub, int ngroups, int nrhs, int bpmax, int rounds, const cpx<T>* cpl,
                    const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc,
                    hipStream_t s) {
  constexpr int PF = sizeof(T) == 4 ? 4 : 2;
  const size_t lds = (size_t)bpmax * lds_width<T>(RG) * sizeof(cpx<T>);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_oras_fused<T, RG, PF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
  }
  // waves per workgroup: the tiles spread evenly over the given number of rounds
  const int nmt = bpmax / 16;
  rounds = std::max(rounds, min_rounds<T>(bpmax));
  const int nwaves = (nmt + rounds - 1) / rounds;
  hipLaunchKernelGGL((k_oras_fused<T, RG, PF>), dim3(nsub * ngroups), dim3(64 * nwaves), lds, s, subs, ngroups, nrhs, cpl,
                     sinv, u, z, add, gnx, gny, yloc);
}

}  // namespace

// LDS budget of the fused kernel (one plane operand)
constexpr size_t FUSED_LDS = 150 * 1024;

template <typename T>
int fused_group(int bpmax, int nrhs) {
  int rg = nrhs <= 8 ? 8 : (nrhs <= 16 ? 16 : 32);
  while (rg >= 8 && (size_t)bpmax * lds_width<T>(rg) * sizeof(cpx<T>) > FUSED_LDS) rg /= 2;
  return rg >= 8 ? rg : 0;
}

namespace {

template <typename T>
void launch_rg(int rg, int rounds, const Sub* subs, int nsub, int nrhs, int bpmax, const cpx<T>* cpl,
               const cpx<T>* sinv, const z64* u, z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc,
               hipStream_t s) {
  const int ngroups = (nrhs + rg - 1) / rg;
  switch (rg) {
    case 8:
      launch_fused_t<T, 8>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny, yloc, s);
      break;
    case 16:
      launch_fused_t<T, 16>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny, yloc, s);
      break;
    default:
      launch_fused_t<T, 32>(subs, nsub, ngroups, nrhs, bpmax, rounds, cpl, sinv, u, z, add, gnx, gny, yloc, s);
      break;
  }
}

// Autotuned launch shape of the fused sweep (right-hand-side group, tile
// rounds per wave), per problem shape.
struct TuneKey {
  int es, bpmax, nsub, nrhs, gnx, gny;
  bool operator<(const TuneKey& o) const {
    return std::tie(es, bpmax, nsub, nrhs, gnx, gny) < std::tie(o.es, o.bpmax, o.nsub, o.nrhs, o.gnx, o.gny);
  }
};
struct TuneVal {
  int rg, rounds;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tune;

}  // namespace

int tuned_group(int es, int bpmax, int nsub, int nrhs, int gnx, int gny) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({es, bpmax, nsub, nrhs, gnx, gny});
  return it == g_tune.end() ? 0 : it->second.rg;
}

template <typename T>
bool oras_fused(const Sub* subs, int nsub, int bpmax, const cpx<T>* cpl, const cpx<T>* sinv, int nrhs, const z64* u,
                z64* z, const z64* add, int gnx, int gny, cpx<T>* yloc, hipStream_t s) {
  const int rgmax = fused_group<T>(bpmax, nrhs);
  if (rgmax == 0) return false;
  const TuneKey key{(int)sizeof(T), bpmax, nsub, nrhs, gnx, gny};
  TuneVal tv{0, 0};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) tv = it->second;
  }
  static const bool no_tune = std::getenv("HELM_NO_TUNE") != nullptr;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cap);
  const int r0 = min_rounds<T>(bpmax), nmt = bpmax / 16;
  if (tv.rg == 0 && !no_tune && cap == hipStreamCaptureStatusNone) {
    // time every admissible (group, rounds) pair twice on this very input (the
    // sweep is idempotent: z and the scratch planes are overwritten) and keep
    // the fastest
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    for (int cand = 8; cand <= rgmax; cand *= 2) {
      int last_waves = 0;
      for (int rounds = r0; rounds <= r0 + 2; ++rounds) {
        const int waves = (nmt + rounds - 1) / rounds;
        if (waves == last_waves) continue;
        last_waves = waves;
        float tot = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          (void)hipEventRecord(e0, s);
          launch_rg<T>(cand, rounds, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, s);
          (void)hipEventRecord(e1, s);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) tot += ms;
        }
        if (tot < best) {
          best = tot;
          tv = {cand, rounds};
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    static const bool verbose = std::getenv("HELM_TUNE_VERBOSE") != nullptr;
    if (verbose)
      std::fprintf(stderr, "helm: sweep tuned (fp%d, bp %d, %d boxes, %d rhs): group %d, %d waves, %.3f ms\n",
                   (int)sizeof(T) * 8, bpmax, nsub, nrhs, tv.rg, (nmt + tv.rounds - 1) / tv.rounds, best);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = tv;
  }
  if (tv.rg == 0) tv = {rgmax, r0};
  launch_rg<T>(tv.rg, tv.rounds, subs, nsub, nrhs, bpmax, cpl, sinv, u, z, add, gnx, gny, yloc, s);
  return true;
}

template bool oras_fused<float>(const Sub*, int, int, const c32*, const c32*, int, const z64*, z64*, const z64*, int,
                                int, c32*, hipStream_t);
template bool oras_fused<double>(const Sub*, int, int, const z64*, const z64*, int, const z64*, z64*, const z64*, int,
                                 int, z64*, hipStream_t);
template int fused_group<float>(int, int);
template int fused_group<double>(int, int);
