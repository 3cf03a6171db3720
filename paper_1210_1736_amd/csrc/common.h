// Internal definitions shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/sbx.h"

namespace sbx {

// Global-memory views of pointers held in device records: accesses through
// them compile to global_* instructions instead of flat_* ones (which also
// count against the LDS/scalar wait counter, so every LDS wait would wait
// for them too).
template <typename T>
using gp = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gp<T> glb(T* p) {
  return (gp<T>)p;
}

// ---------------------------------------------------------------- errors ---
void set_error(const std::string& msg);

#define SBX_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::sbx::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      return SBX_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

#define SBX_TRY(call)                                                              \
  do {                                                                             \
    sbx_status s_ = (call);                                                        \
    if (s_ != SBX_OK) return s_;                                                   \
  } while (0)

// ------------------------------------------------------- phase recorder ---
// Optional HIP-event marks between kernel launches on a stream: the time
// between two consecutive marks is charged to the phase of the later mark.
enum Phase {
  PH_START = 0, PH_ZERO, PH_PRE, PH_DEPOSIT, PH_FWD_X, PH_FWD_Y, PH_ZPASS, PH_INV_Y, PH_INV_X,
  PH_FORCE, PH_SORT, PH_COUNT
};

struct Recorder {
  bool on = false;
  int used = 0;
  hipEvent_t* ev = nullptr;
  int* tag = nullptr;
  int cap = 0;
  void mark(int t, hipStream_t s) {
    if (!on || used >= cap) return;
    if (hipEventRecord(ev[used], s) == hipSuccess) tag[used++] = t;
  }
};

// ---------------------------------------------------------------- complex --
template <typename T>
struct alignas(2 * sizeof(T)) C2 {
  T re, im;
};

template <typename T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ C2<T> conjc(C2<T> a) { return {a.re, -a.im}; }

// multiply by exp(-i pi/2) = -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ C2<T> rot90(C2<T> a) {
  return INV ? C2<T>{-a.im, a.re} : C2<T>{a.im, -a.re};
}

// cos and sin of 2 pi m / 16, m = 0..15
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977,
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977, 0.70710678118654752, 0.92387953251128674,
    1.0, 0.92387953251128674, 0.70710678118654752, 0.38268343236508977,
    0.0, -0.38268343236508977, -0.70710678118654752, -0.92387953251128674,
    -1.0, -0.92387953251128674, -0.70710678118654752, -0.38268343236508977};

// a * exp(-+ 2 pi i m / 16) with m a compile-time constant
template <int M, bool INV, typename T>
__device__ __forceinline__ C2<T> tw16(C2<T> a) {
  constexpr int m = M & 15;
  if constexpr (m == 0) return a;
  else if constexpr (m == 4) return rot90<INV>(a);
  else if constexpr (m == 8) return C2<T>{-a.re, -a.im};
  else if constexpr (m == 12) return rot90<!INV>(a);
  else {
    const T c = (T)kCos16[m];
    const T s = INV ? (T)kSin16[m] : -(T)kSin16[m];
    return C2<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

// ---------------------------------------------------------- register DFTs --
// In-place DFT of v[0..R) in natural order: V[k] = sum_n v[n] exp(-+2 pi i nk/R).
template <bool INV, typename T>
__device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4s(C2<T>& x0, C2<T>& x1, C2<T>& x2, C2<T>& x3) {
  C2<T> a = x0 + x2, b = x0 - x2, c = x1 + x3, d = rot90<INV>(x1 - x3);
  x0 = a + c;
  x2 = a - c;
  x1 = b + d;
  x3 = b - d;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(C2<T>* v) {
  dft4s<INV>(v[0], v[1], v[2], v[3]);
}

// 8 = 4 x 2: n = 2 n1 + n2, k = k1 + 4 k2
template <bool INV, typename T>
__device__ __forceinline__ void dft8(C2<T>* v) {
  C2<T> a0 = v[0], a1 = v[2], a2 = v[4], a3 = v[6];
  C2<T> b0 = v[1], b1 = v[3], b2 = v[5], b3 = v[7];
  dft4s<INV>(a0, a1, a2, a3);
  dft4s<INV>(b0, b1, b2, b3);
  b1 = tw16<2, INV>(b1);
  b2 = tw16<4, INV>(b2);
  b3 = tw16<6, INV>(b3);
  v[0] = a0 + b0; v[4] = a0 - b0;
  v[1] = a1 + b1; v[5] = a1 - b1;
  v[2] = a2 + b2; v[6] = a2 - b2;
  v[3] = a3 + b3; v[7] = a3 - b3;
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <bool INV, typename T>
__device__ __forceinline__ void dft16(C2<T>* v) {
  C2<T> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    a[n2][0] = v[n2];
    a[n2][1] = v[4 + n2];
    a[n2][2] = v[8 + n2];
    a[n2][3] = v[12 + n2];
    dft4s<INV>(a[n2][0], a[n2][1], a[n2][2], a[n2][3]);
  }
  a[1][1] = tw16<1, INV>(a[1][1]);
  a[1][2] = tw16<2, INV>(a[1][2]);
  a[1][3] = tw16<3, INV>(a[1][3]);
  a[2][1] = tw16<2, INV>(a[2][1]);
  a[2][2] = tw16<4, INV>(a[2][2]);
  a[2][3] = tw16<6, INV>(a[2][3]);
  a[3][1] = tw16<3, INV>(a[3][1]);
  a[3][2] = tw16<6, INV>(a[3][2]);
  a[3][3] = tw16<9, INV>(a[3][3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C2<T> x0 = a[0][k1], x1 = a[1][k1], x2 = a[2][k1], x3 = a[3][k1];
    dft4s<INV>(x0, x1, x2, x3);
    v[k1] = x0;
    v[k1 + 4] = x1;
    v[k1 + 8] = x2;
    v[k1 + 12] = x3;
  }
}

// cos and sin of 2 pi m / 32, m = 0..15
__device__ constexpr double kCos32[16] = {
    1.0, 0.98078528040323043, 0.92387953251128674, 0.83146961230254524,
    0.70710678118654752, 0.55557023301960218, 0.38268343236508977, 0.19509032201612826,
    0.0, -0.19509032201612826, -0.38268343236508977, -0.55557023301960218,
    -0.70710678118654752, -0.83146961230254524, -0.92387953251128674, -0.98078528040323043};
__device__ constexpr double kSin32[16] = {
    0.0, 0.19509032201612826, 0.38268343236508977, 0.55557023301960218,
    0.70710678118654752, 0.83146961230254524, 0.92387953251128674, 0.98078528040323043,
    1.0, 0.98078528040323043, 0.92387953251128674, 0.83146961230254524,
    0.70710678118654752, 0.55557023301960218, 0.38268343236508977, 0.19509032201612826};

// a * exp(-+ 2 pi i m / 32), m = 0..15 a compile-time constant
template <int M, bool INV, typename T>
__device__ __forceinline__ C2<T> tw32(C2<T> a) {
  if constexpr ((M & 1) == 0) {
    return tw16<M / 2, INV>(a);
  } else {
    const T c = (T)kCos32[M];
    const T s = INV ? (T)kSin32[M] : -(T)kSin32[M];
    return C2<T>{a.re * c - a.im * s, a.re * s + a.im * c};
  }
}

template <int M, bool INV, typename T>
__device__ __forceinline__ void tw32_all(C2<T>* b) {
  b[M] = tw32<M, INV>(b[M]);
  if constexpr (M + 1 < 16) tw32_all<M + 1, INV>(b);
}

// 32 = 16 x 2: n = 2 n1 + n2, k = k1 + 16 k2
template <bool INV, typename T>
__device__ __forceinline__ void dft32(C2<T>* v) {
  C2<T> a[16], b[16];
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) {
    a[n1] = v[2 * n1];
    b[n1] = v[2 * n1 + 1];
  }
  dft16<INV>(a);
  dft16<INV>(b);
  tw32_all<1, INV>(b);
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) {
    v[k1] = a[k1] + b[k1];
    v[k1 + 16] = a[k1] - b[k1];
  }
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dftR(C2<T>* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
  else dft32<INV>(v);
}

}  // namespace sbx
