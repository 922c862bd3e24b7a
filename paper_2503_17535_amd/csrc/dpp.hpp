// Cross-lane argmax helpers on DPP (data-parallel primitives): VALU lane
// exchanges within a 16-lane row, no LDS round trip.
#pragma once
#include <hip/hip_runtime.h>

namespace hps {

// DPP controls (GFX9 encoding)
constexpr int DPP_QUAD_XOR1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_ROR4 = 0x124;  // rotate right by 4 within a 16-lane row
constexpr int DPP_ROW_ROR8 = 0x128;  // rotate right by 8 within a 16-lane row
constexpr int DPP_HALF_MIRROR = 0x141;  // reverse within each 8-lane half row

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v));
  const int hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// |x| as a pivot key: NaN and inf map to +inf so that some unused row is
// always chosen.
__device__ __forceinline__ double pivot_key(double x) {
  double v = fabs(x);
  return (v <= 1.7976931348623157e308) ? v : __builtin_inf();
}

// (key, row, val): keep the larger key; ties go to the lower row.  Written
// with selects, not branches: this sits on the critical path of every
// elimination step.
__device__ __forceinline__ void amax_merge(double& key, int& row, double& val, double ok, int orow, double oval) {
  const bool take = (ok > key) | ((ok == key) & (orow < row));
  key = take ? ok : key;
  row = take ? orow : row;
  val = take ? oval : val;
}

// Local scan step over a thread's own rows, visited in increasing row order:
// an equal key never replaces the earlier (lower) row.  Rows already used as
// pivots carry key -1 and never win.
__device__ __forceinline__ void amax_scan(double& key, int& row, double& val, double x, int xrow, bool used) {
  const double k = used ? -1.0 : pivot_key(x);
  const bool take = k > key;
  key = take ? k : key;
  row = take ? xrow : row;
  val = take ? x : val;
}

// Packed 32-bit pivot key of an unused row: |x| above the row's rank code
// (the B low bits, larger for a lower row, code > 0).  The high word of |x|
// keeps its exponent and leading 21 - B mantissa bits (13 for B = 8).  An
// unsigned max over keys picks the largest |x| up to a relative 2^(B-21),
// ties going to the lower row; NaN and inf keys exceed every finite one.
// Used rows take key 0 and so never win against an unused row.
template <int B = 8>
__device__ __forceinline__ unsigned pivot_key32(double x, int code) {
  static_assert(B >= 8 && B <= 16, "code bits");
  const unsigned hi = (unsigned)__double2hiint(x);
  return ((hi & (0x7fffffffu & ~((1u << (B - 1)) - 1u))) << 1) + (unsigned)code;
}

// The same key for codes below 256 in two instructions (and-or): the high
// word of |x| with its low 8 bits (the lowest mantissa bits) replaced by the
// code, i.e. |x| to 12 mantissa bits.
__device__ __forceinline__ unsigned pivot_key32_c8(double x, int code) {
  return ((unsigned)__double2hiint(x) & 0x7fffff00u) | (unsigned)code;
}

// Unsigned max over each aligned group of G = 8 or 16 lanes; every lane of
// the group ends with it.
template <int G>
__device__ __forceinline__ unsigned group_max(unsigned k) {
  static_assert(G == 8 || G == 16, "group of 8 or 16 lanes");
  if (G == 16) {
    k = max(k, (unsigned)dpp_i<DPP_ROW_ROR8>((int)k));
    k = max(k, (unsigned)dpp_i<DPP_ROW_ROR4>((int)k));
  } else {
    k = max(k, (unsigned)dpp_i<DPP_HALF_MIRROR>((int)k));
  }
  k = max(k, (unsigned)dpp_i<DPP_QUAD_XOR2>((int)k));
  k = max(k, (unsigned)dpp_i<DPP_QUAD_XOR1>((int)k));
  return k;
}

// Unsigned max over the whole wavefront (uniform result).
__device__ __forceinline__ unsigned wave_max(unsigned k) {
  k = group_max<16>(k);
  const unsigned a = max((unsigned)__builtin_amdgcn_readlane((int)k, 0), (unsigned)__builtin_amdgcn_readlane((int)k, 16));
  const unsigned b = max((unsigned)__builtin_amdgcn_readlane((int)k, 32), (unsigned)__builtin_amdgcn_readlane((int)k, 48));
  return max(a, b);
}

// A double from one lane (uniform lane index) to every lane.
__device__ __forceinline__ double readlane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// 1/x from the hardware reciprocal estimate and two Newton steps
// r <- r + r (1 - x r), each taking the relative error e to about e^2.
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

template <int CTRL>
__device__ __forceinline__ void amax_step(double& key, int& row, double& val) {
  const double ok = dpp_d<CTRL>(key);
  const int orow = dpp_i<CTRL>(row);
  const double oval = dpp_d<CTRL>(val);
  amax_merge(key, row, val, ok, orow, oval);
}

// Argmax over groups of G consecutive lanes (G = 8 or 16, aligned); every lane
// of the group ends with the group's result.
template <int G>
__device__ __forceinline__ void group_argmax(double& key, int& row, double& val) {
  static_assert(G == 8 || G == 16, "group of 8 or 16 lanes");
  if (G == 16) {
    amax_step<DPP_ROW_ROR8>(key, row, val);
    amax_step<DPP_ROW_ROR4>(key, row, val);
  } else {
    amax_step<DPP_HALF_MIRROR>(key, row, val);
  }
  amax_step<DPP_QUAD_XOR2>(key, row, val);
  amax_step<DPP_QUAD_XOR1>(key, row, val);
}

// Argmax over the whole 64-lane wavefront; every lane ends with the result.
__device__ __forceinline__ void wave_argmax(double& key, int& row, double& val) {
  group_argmax<16>(key, row, val);
  double k = key, v = val;
  int r = row;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const double ok = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(k), 16 * g),
                                       __builtin_amdgcn_readlane(__double2loint(k), 16 * g));
    const int orow = __builtin_amdgcn_readlane(r, 16 * g);
    const double oval = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * g),
                                         __builtin_amdgcn_readlane(__double2loint(v), 16 * g));
    amax_merge(key, row, val, ok, orow, oval);
  }
}


}  // namespace hps
