// Instantiation of the row/column pass kernels for one transform length,
// selected at compile time with -DPASS_N=<8..1024>; the build compiles this
// file once per length so the eight lengths build in parallel.
#include "lista_passes.h"
#include "passes.h"

#ifndef PASS_N
#error "compile with -DPASS_N=<transform length>"
#endif

#define BCCB_CAT2(a, b) a##b
#define BCCB_CAT(a, b) BCCB_CAT2(a, b)

namespace bccb {

int BCCB_CAT(row_launch_, PASS_N)(int E, int mode, const RowArgs& a, int rpb, hipStream_t s) {
  switch (E) {
    case 4: return row_launch_e<PASS_N, 4>(mode, a, rpb, s);
    case 8: return row_launch_e<PASS_N, 8>(mode, a, rpb, s);
#if PASS_N >= 16
    case 16: return row_launch_e<PASS_N, 16>(mode, a, rpb, s);
#endif
#if PASS_N >= 32
    case 32: return row_launch_e<PASS_N, 32>(mode, a, rpb, s);
#endif
    default: return -2;
  }
}

int BCCB_CAT(col_launch_, PASS_N)(int E, int mode, const ColArgs& a, int W, hipStream_t s) {
  switch (E) {
    case 4: return col_launch_e<PASS_N, 4>(mode, a, W, s);
    case 8: return col_launch_e<PASS_N, 8>(mode, a, W, s);
#if PASS_N >= 16
    case 16: return col_launch_e<PASS_N, 16>(mode, a, W, s);
#endif
#if PASS_N >= 32
    case 32: return col_launch_e<PASS_N, 32>(mode, a, W, s);
#endif
    default: return -2;
  }
}

int BCCB_CAT(lista_launch_, PASS_N)(int which, const void* args, int E, int rpb_or_w, int groups, hipStream_t s) {
  switch (E) {
    case 4: return lista_launch_e<PASS_N, 4>(which, args, rpb_or_w, groups, s);
    case 8: return lista_launch_e<PASS_N, 8>(which, args, rpb_or_w, groups, s);
#if PASS_N >= 16
    case 16: return lista_launch_e<PASS_N, 16>(which, args, rpb_or_w, groups, s);
#endif
    default: return -2;
  }
}

}  // namespace bccb
