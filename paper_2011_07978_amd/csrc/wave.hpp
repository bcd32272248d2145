// Wavefront-level helpers for CDNA (64-lane wavefronts, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chem {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Broadcast a double from a uniform lane index (result in scalar registers).
__device__ __forceinline__ double readlane_d(double v, int l) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Make a value that every lane already agrees on wave-uniform (SGPR).
__device__ __forceinline__ double uniform_d(double v) {
    int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lane `src` (per lane) -> value (ds_bpermute).
__device__ __forceinline__ double shfl_d(double v, int src) {
    int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// DPP lane exchange inside 16-lane rows.
//   0xB1 quad_perm [1,0,3,2] (lane ^ 1), 0x4E quad_perm [2,3,0,1] (lane ^ 2),
//   0x141 row_half_mirror (i -> 7 - i in each 8 lanes), 0x140 row_mirror (i -> 15 - i).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Row broadcasts (GFX9 DPP): 0x142 row_bcast:15 hands lane 15 of each row to
// the next row, 0x143 row_bcast:31 hands lane 31 to rows 2 and 3; rows left
// out by the row mask receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_bcast_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Reductions over the 64 lanes.  Within each 16-lane row the two operands of
// every combine are the same pair of values on both lanes (sum and max
// commute), so every lane of a row holds the same row result; the row results
// are then combined as (r0 + r1) + (r2 + r3) by two row broadcasts, the sum
// read from lane 63.  The bits do not depend on scheduling.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    v += dpp_bcast_d<0x142, 0xa>(v);   // rows 1, 3: r1 + r0, r3 + r2
    v += dpp_bcast_d<0x143, 0xc>(v);   // rows 2, 3: + lane 31 (r1 + r0)
    return readlane_d(v, 63);
}

__device__ __forceinline__ double max2(double a, double b) { return a > b ? a : b; }

// The same reductions when only lanes 0..15 can hold nonzero values (the
// other rows would add zeros or maxima of zero): the row-0 result, the same
// bits as the 64-lane form.
__device__ __forceinline__ double wave_sum_row0(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    return readlane_d(v, 0);
}

// Maximum of values that are not NaN.
__device__ __forceinline__ double wave_max(double v) {
    v = max2(v, dpp_d<0xB1>(v));
    v = max2(v, dpp_d<0x4E>(v));
    v = max2(v, dpp_d<0x141>(v));
    v = max2(v, dpp_d<0x140>(v));
    return max2(max2(readlane_d(v, 0), readlane_d(v, 16)), max2(readlane_d(v, 32), readlane_d(v, 48)));
}

__device__ __forceinline__ double wave_max_row0(double v) {
    v = max2(v, dpp_d<0xB1>(v));
    v = max2(v, dpp_d<0x4E>(v));
    v = max2(v, dpp_d<0x141>(v));
    v = max2(v, dpp_d<0x140>(v));
    return readlane_d(v, 0);
}

// Maximum of unsigned 32-bit keys (every lane returns the same value).
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xf, 0xf, false));
    const unsigned a = max((unsigned)__builtin_amdgcn_readlane((int)v, 0),
                           (unsigned)__builtin_amdgcn_readlane((int)v, 16));
    const unsigned b = max((unsigned)__builtin_amdgcn_readlane((int)v, 32),
                           (unsigned)__builtin_amdgcn_readlane((int)v, 48));
    return max(a, b);
}

// 1/x from the hardware reciprocal estimate refined by two Newton-Raphson
// steps (r <- r + r (1 - x r)); zero, infinite and NaN x give NaN.
__device__ __forceinline__ double recip_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Lane mask of p (the compiler's own mask, with no detour through an integer).
__device__ __forceinline__ unsigned long long ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ bool wave_any(bool p) { return ballot(p) != 0ull; }

}  // namespace chem
