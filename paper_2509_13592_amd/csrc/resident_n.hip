// Instantiation of the single-scene cooperative solver for one row length,
// selected at compile time with -DRES_N1=<32..512>; every column length of
// 32..512 is instantiated for it.
#include "resident.h"

#ifndef RES_N1
#error "compile with -DRES_N1=<row length>"
#endif

#define BCCB_CAT2(a, b) a##b
#define BCCB_CAT(a, b) BCCB_CAT2(a, b)

namespace bccb {

int BCCB_CAT(resident_launch_, RES_N1)(int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s) {
  switch (L2) {
#if RES_N1 >= 32
    case 32: return resident_launch_nn<RES_N1, 32>(mode, a, check_only, s);
#endif
    case 64: return resident_launch_nn<RES_N1, 64>(mode, a, check_only, s);
    case 128: return resident_launch_nn<RES_N1, 128>(mode, a, check_only, s);
    case 256: return resident_launch_nn<RES_N1, 256>(mode, a, check_only, s);
    case 512: return resident_launch_nn<RES_N1, 512>(mode, a, check_only, s);
    default: return -2;
  }
}

}  // namespace bccb
