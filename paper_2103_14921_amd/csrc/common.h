// Shared device/host helpers of the HIP library: complex arithmetic, error
// handling and the small structs passed to kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};
using z64 = cpx<double>;
using c32 = cpx<float>;

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T r, T i) {
  cpx<T> z;
  z.re = r;
  z.im = i;
  return z;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) {
  return mk(a.re + b.re, a.im + b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) {
  return mk(a.re - b.re, a.im - b.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a) {
  return mk(-a.re, -a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) {
  return mk(s * a.re, s * a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T>& operator+=(cpx<T>& a, cpx<T> b) {
  a.re += b.re;
  a.im += b.im;
  return a;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T>& operator-=(cpx<T>& a, cpx<T> b) {
  a.re -= b.re;
  a.im -= b.im;
  return a;
}
// a += b*c
template <typename T>
__host__ __device__ __forceinline__ void cfma(cpx<T>& a, cpx<T> b, cpx<T> c) {
  a.re = fma(b.re, c.re, a.re);
  a.re = fma(-b.im, c.im, a.re);
  a.im = fma(b.re, c.im, a.im);
  a.im = fma(b.im, c.re, a.im);
}
// a -= b*c
template <typename T>
__host__ __device__ __forceinline__ void cfms(cpx<T>& a, cpx<T> b, cpx<T> c) {
  a.re = fma(-b.re, c.re, a.re);
  a.re = fma(b.im, c.im, a.re);
  a.im = fma(-b.re, c.im, a.im);
  a.im = fma(-b.im, c.re, a.im);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> conj(cpx<T> a) {
  return mk(a.re, -a.im);
}
// conj(a)*b
template <typename T>
__host__ __device__ __forceinline__ void cdot_acc(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(-a.im, b.re, acc.im);
}
template <typename T>
__host__ __device__ __forceinline__ T abs2(cpx<T> a) {
  return a.re * a.re + a.im * a.im;
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cdiv(cpx<T> a, cpx<T> b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    T r = b.im / b.re, d = b.re + b.im * r;
    return mk((a.re + a.im * r) / d, (a.im - a.re * r) / d);
  } else {
    T r = b.re / b.im, d = b.re * r + b.im;
    return mk((a.re * r + a.im) / d, (a.im * r - a.re) / d);
  }
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cinv(cpx<T> b) {
  return cdiv(mk<T>(1, 0), b);
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cpx<To> ccast(cpx<Ti> a) {
  return mk<To>((To)a.re, (To)a.im);
}

// ---------------------------------------------------------------------------
// Operator description passed by value to kernels.
// ---------------------------------------------------------------------------
struct OpDev {
  int nx, ny, nz;
  double h2inv;        // 1/h^2
  double alpha[3];     // face, edge, corner stiffness weights
  double wm[4];        // wm1 (centre), wm2 (face), wm3 (edge), wm4 (corner)
  const z64* sigma;    // s k^2 per node
  const z64* xi_int;   // [nx | ny | nz] stretch at nodes
  const z64* xi_half;  // [(nx+1) | (ny+1) | (nz+1)] stretch at midpoints (j - 1/2)
  const z64* i2_int;   // 1/xi^2 at nodes
  const z64* i2_half;  // 1/xi^2 at midpoints
  const uint8_t* flat; // per-axis flag: 1 where the 3-point neighbourhood has xi == 1
  int off_int[3];      // offsets of each axis in the int tables
  int off_half[3];     // offsets of each axis in the half tables
  // adaptive coefficients: per node {alpha_face, alpha_edge, alpha_corner, wm1,
  // wm2, wm3, wm4, 0}; nullptr = the single set alpha, wm above
  const double* wnode;
  // row diagonals A[i, i] (set-up, in fine_row's order of terms); the products read them
  const z64* diag;
};

// Per-subdomain description (device and host).
struct Sub {
  int elo[3], ehi[3];  // extended box [elo, ehi)
  int lo[3], hi[3];    // core box
  int ex, ey, ez;      // extended sizes
  int b, bp;           // plane size ex*ey and padded plane size
  int id;              // the box's index in box order (for arrays indexed per box)
  long long node_off;  // offset of the box's nodes in the concatenated local arrays
  long long mat_off;   // offset (elements) of the box's plane matrices [ez][bp][bp]
  long long vec_off;   // offset (elements / nrhs) of the box's local vector [ez][bp]
};

#define HELM_CHECK_HIP(expr)                                                       \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      throw HelmError(HELM_EDEVICE, std::string("HIP error ") + hipGetErrorString(_e) + \
                                        " at " + __FILE__ + ":" + std::to_string(__LINE__)); \
    }                                                                              \
  } while (0)

__host__ __device__ __forceinline__ long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }

// Workgroups are dispatched round-robin over the XCDs (each with its own L2):
// the logical index xcd_contiguous(blockIdx.x, gridDim.x) gives XCD c the
// contiguous range [start_c, start_c + count_c) of logical workgroups, so that
// neighbouring logical workgroups, which share data, meet in the same L2.
__device__ __forceinline__ long long xcd_contiguous(long long b, long long nb) {
  constexpr int NXCD = 8;
  const long long q = nb / NXCD, rem = nb % NXCD;
  const long long c = b % NXCD, k = b / NXCD;
  return c * q + (c < rem ? c : rem) + k;
}
