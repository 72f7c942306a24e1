// Row-length dispatch of the single-scene cooperative solver (the kernels are
// instantiated per row length in resident_n.hip).
#include "resident_api.h"

namespace bccb {

int launch_resident(int L1, int L2, int mode, const ResidentArgs& a, int check_only, hipStream_t s) {
  switch (L1) {
    case 32: return resident_launch_32(L2, mode, a, check_only, s);
    case 64: return resident_launch_64(L2, mode, a, check_only, s);
    case 128: return resident_launch_128(L2, mode, a, check_only, s);
    case 256: return resident_launch_256(L2, mode, a, check_only, s);
    case 512: return resident_launch_512(L2, mode, a, check_only, s);
    default: return -2;
  }
}

}  // namespace bccb
