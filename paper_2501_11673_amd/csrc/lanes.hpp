// Cross-lane sums within a 64-lane wave (gfx950), shared by the persistent
// step kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace kpp {

// Cross-lane exchange without the LDS crossbar.  Lanes are paired across bit
// o of the lane index: o = 32 and 16 by the permlane swaps, o = 8, 2, 1 by DPP
// moves (xor o), o = 4 by the DPP half-row mirror (xor 7: it flips bit 2 and
// keeps the bits above it, which is all a butterfly stage needs).
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double dpp_partner(double v, int o) {
  const int l = __double2loint(v), h = __double2hiint(v);
  switch (o) {
    case 8: return __hiloint2double(dpp_mov<0x128>(h), dpp_mov<0x128>(l));   // row_ror:8
    case 4: return __hiloint2double(dpp_mov<0x141>(h), dpp_mov<0x141>(l));   // row_half_mirror
    case 2: return __hiloint2double(dpp_mov<0x4E>(h), dpp_mov<0x4E>(l));     // quad_perm [2,3,0,1]
    default: return __hiloint2double(dpp_mov<0xB1>(h), dpp_mov<0xB1>(l));    // quad_perm [1,0,3,2]
  }
}
// One butterfly stage over a pair of row sums: a lane with bit o clear returns
// its lo plus its partner's lo, a lane with bit o set its hi plus the
// partner's hi.  For o = 32 (16) the swap leaves x = [lo of the lower lanes,
// hi of the lower lanes] and y = [lo of the upper lanes, hi of the upper
// lanes] per 64 (32) lanes, so x + y is that sum in every lane.
__device__ __forceinline__ double fold(double lo, double hi, int o, bool up) {
  if (o >= 16) {
    const unsigned xl = __double2loint(lo), xh = __double2hiint(lo);
    const unsigned yl = __double2loint(hi), yh = __double2hiint(hi);
    const auto sl = o == 32 ? __builtin_amdgcn_permlane32_swap(xl, yl, false, false)
                            : __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
    const auto sh = o == 32 ? __builtin_amdgcn_permlane32_swap(xh, yh, false, false)
                            : __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
    return __hiloint2double(static_cast<int>(sh[0]), static_cast<int>(sl[0])) +
           __hiloint2double(static_cast<int>(sh[1]), static_cast<int>(sl[1]));
  }
  // the pair passes through an empty asm statement: otherwise the compiler may
  // fold the two selects into one indexed read of the row array, which it
  // lowers to a chain of compares over the whole array
  asm("" : "+v"(lo), "+v"(hi));
  const double send = up ? lo : hi;
  const double keep = up ? hi : lo;
  return keep + dpp_partner(send, o);
}

// sum over the wave, in every lane
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fold(v, v, o, false);
  return v;
}

}  // namespace kpp
