// Wavefront-level helpers (64 lanes).
#pragma once

#include <hip/hip_runtime.h>

namespace pgx {

// Segmented inclusive sums over one wavefront (64 lanes) of runs of equal
// keys in adjacent lanes, for any key order (equal keys that are not adjacent
// stay separate runs).  Lane L starts a run when its key differs from lane
// L - 1's.  A Hillis-Steele scan with run-start flags: row shifts of 1, 2, 4
// and 8 lanes within rows of 16 (DPP), then the carries from lanes 15, 31 and
// 47 across rows; each step adds the shifted partial sum only while no run
// start lies in between, so a lane ends with the sum of its run up to
// itself, and the last lane of each run (`tail`) holds the whole run.  The
// steps taken depend on the keys only and are computed once; all 64 lanes
// must take part.
struct SegRuns {
  uint32_t m;
  bool tail;
  __device__ __forceinline__ void init(int key) {
    const int lane = (int)(threadIdx.x & 63u), lr = lane & 15, row = lane >> 4;
    const int prev = __builtin_amdgcn_ds_bpermute(((lane + 63) & 63) << 2, key);
    const int next = __builtin_amdgcn_ds_bpermute(((lane + 1) & 63) << 2, key);
    int h = (lane == 0 || prev != key) ? 1 : 0;  // a run starts at or after the span's start
    tail = lane == 63 || next != key;
    m = 0u;
    const int hs1 = __builtin_amdgcn_update_dpp(1, h, 0x111, 0xF, 0xF, false);
    if (lr >= 1 && !h) { m |= 1u; h |= hs1; }
    const int hs2 = __builtin_amdgcn_update_dpp(1, h, 0x112, 0xF, 0xF, false);
    if (lr >= 2 && !h) { m |= 2u; h |= hs2; }
    const int hs4 = __builtin_amdgcn_update_dpp(1, h, 0x114, 0xF, 0xF, false);
    if (lr >= 4 && !h) { m |= 4u; h |= hs4; }
    const int hs8 = __builtin_amdgcn_update_dpp(1, h, 0x118, 0xF, 0xF, false);
    if (lr >= 8 && !h) { m |= 8u; h |= hs8; }
    const int c15 = __builtin_amdgcn_readlane(h, 15);
    if (row == 1 && !h) { m |= 16u; h |= c15; }
    const int c31 = __builtin_amdgcn_readlane(h, 31);
    if (row == 2 && !h) { m |= 32u; h |= c31; }
    const int c47 = __builtin_amdgcn_readlane(h, 47);
    if (row == 3 && !h) { m |= 64u; h |= c47; }
  }
  template <int CTRL>
  __device__ __forceinline__ static int shr32(int b) {
    return __builtin_amdgcn_update_dpp(0, b, CTRL, 0xF, 0xF, false);
  }
  // v of the lane D below (row shift, 0x110 + D), any 32- or 64-bit type
  template <int D, typename V>
  __device__ __forceinline__ static V shr(V v) {
    if constexpr (sizeof(V) == 4) {
      return __builtin_bit_cast(V, shr32<0x110 + D>(__builtin_bit_cast(int, v)));
    } else {
      const int2 b = __builtin_bit_cast(int2, v);
      return __builtin_bit_cast(V, make_int2(shr32<0x110 + D>(b.x), shr32<0x110 + D>(b.y)));
    }
  }
  template <int L, typename V>
  __device__ __forceinline__ static V lane_value(V v) {
    if constexpr (sizeof(V) == 4) {
      return __builtin_bit_cast(V, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), L));
    } else {
      const int2 b = __builtin_bit_cast(int2, v);
      return __builtin_bit_cast(V, make_int2(__builtin_amdgcn_readlane(b.x, L),
                                             __builtin_amdgcn_readlane(b.y, L)));
    }
  }
  template <typename V>
  __device__ __forceinline__ V add(V v) const {
    const V z = (V)0;
    V s;
    s = shr<1>(v);
    v += (m & 1u) ? s : z;
    s = shr<2>(v);
    v += (m & 2u) ? s : z;
    s = shr<4>(v);
    v += (m & 4u) ? s : z;
    s = shr<8>(v);
    v += (m & 8u) ? s : z;
    s = lane_value<15>(v);
    v += (m & 16u) ? s : z;
    s = lane_value<31>(v);
    v += (m & 32u) ? s : z;
    s = lane_value<47>(v);
    v += (m & 64u) ? s : z;
    return v;
  }
};

}  // namespace pgx
