// Launch table of the compact register-resident panel kernel (gj_panel_rot_kernel):
// one instantiation per scalar type, panel width, rows per thread and thread count.
// Kept in a translation unit of its own so that it compiles beside the engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>

#include "../../include/hss.h"
#include "common.hpp"
#include "k_gj.hpp"
#include "panel.hpp"

namespace hss {

// Panel shapes held in registers: 16 columns, up to four rows per thread on 128,
// 256 or 512 threads, and for single precision up to eight rows per thread. Complex
// double values take four registers each: 16 columns up to 1024 rows (two rows per
// thread on 512 threads), 8 columns above, where 16 would spill or leave one wave
// per SIMD. The pivot search runs in the matrix's own precision.
template <class X>
bool panel_rot_config(int rows, PanelShape& s) {
  const bool zd = std::is_same<X, cd>::value;
  const int nb = zd && rows > 1024 ? 8 : 16;
  if (rows <= 128) {
    s = {nb, 1, 128};
    return true;
  }
  if (rows <= 256 * (zd ? 2 : 4)) {
    s = {nb, (rows + 255) / 256, 256};
    return true;
  }
  if (rows <= 512 * 4) {
    s = {nb, zd && rows <= 1024 ? 2 : (rows + 511) / 512, 512};
    return true;
  }
  if (std::is_same<X, float>::value && rows <= 512 * 8) {
    const int rpt = (rows + 511) / 512;
    s = {16, rpt <= 6 ? 6 : 8, 512};
    return true;
  }
  return false;
}

// Launches the compact panel of shape s (dd == nullptr: only reports whether that
// shape is compiled); false when it is not.
template <class X>
bool panel_rot_variant(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st) {
#define HSS_ROT(NB_, RPT_, NT_)                                                      \
  if (s.nb == NB_ && s.rpt == RPT_ && s.nt == NT_) {                                 \
    if (dd) gj_panel_rot_kernel<X, NB_, RPT_, NT_><<<nn, NT_, 0, st>>>(dd, j0, nb);  \
    return true;                                                                     \
  }
  if constexpr (std::is_same<X, cd>::value) {
    HSS_ROT(8, 1, 128)
    HSS_ROT(8, 1, 256) HSS_ROT(8, 2, 256) HSS_ROT(8, 3, 256) HSS_ROT(8, 4, 256)
    HSS_ROT(8, 3, 512) HSS_ROT(8, 4, 512)
    HSS_ROT(16, 1, 128) HSS_ROT(16, 1, 256) HSS_ROT(16, 2, 256) HSS_ROT(16, 3, 256) HSS_ROT(16, 4, 256)
    HSS_ROT(16, 5, 256) HSS_ROT(16, 2, 512)
  } else {
    HSS_ROT(16, 1, 128)
    HSS_ROT(16, 1, 256) HSS_ROT(16, 2, 256) HSS_ROT(16, 3, 256) HSS_ROT(16, 4, 256)
    HSS_ROT(16, 3, 512) HSS_ROT(16, 4, 512)
  }
  if constexpr (std::is_same<X, float>::value) {
    HSS_ROT(16, 6, 512) HSS_ROT(16, 8, 512)
  }
#undef HSS_ROT
  return false;
}

template <class X>
void launch_panel_rot(const GjDesc<X>* dd, int nn, int j0, int nb, const PanelShape& s, hipStream_t st) {
  if (!panel_rot_variant<X>(dd, nn, j0, nb, s, st))
    throw Error(HSS_EDEVICE, "no panel variant for nb " + std::to_string(s.nb) + ", rpt " + std::to_string(s.rpt) +
                                 ", threads " + std::to_string(s.nt));
}

template <class X> bool panel_rot_compiled(const PanelShape& s) {
  return panel_rot_variant<X>(nullptr, 0, 0, 0, s, nullptr);
}

template <class X>
void launch_panel_tourn(const GjDesc<X>* dd, int nn, int j0, int nb, int nch, int* cand, hipStream_t st) {
  constexpr int NB = tourn_nb<X>(), RPT = tourn_rpt<X>(), RPTF = tourn_cand<X>() / 256;
  if (nb != NB || nch < 1 || nch * NB > tourn_cand<X>()) throw Error(HSS_EINVAL, "tournament panel shape");
  gj_tourn_local_kernel<X, NB, RPT, 256><<<dim3(nch, nn), 256, 0, st>>>(dd, j0, nb, nch, cand);
  gj_tourn_final_kernel<X, NB, RPTF, 256><<<nn, 256, 0, st>>>(dd, j0, nb, nch, cand);
}

// compiled compact panel shapes of a scalar type (0 float, 1 double, 2 complex
// float, 3 complex double) that hold `rows` rows: (nb, rpt, nt) triples into out
// (at most cap), their count returned
int panel_candidates(int scalar, int rows, int32_t* out, int cap) {
  int n = 0;
  for (int nb : {8, 16})
    for (int nt : {128, 256, 512})
      for (int rpt = 1; rpt <= 8; ++rpt) {
        const PanelShape s{nb, rpt, nt};
        if (rpt * nt < rows) continue;
        const bool ok = scalar == 0   ? panel_rot_compiled<float>(s)
                        : scalar == 1 ? panel_rot_compiled<double>(s)
                        : scalar == 2 ? panel_rot_compiled<cf>(s)
                                      : panel_rot_compiled<cd>(s);
        if (!ok) continue;
        if (out && n < cap) {
          out[3 * n] = nb;
          out[3 * n + 1] = rpt;
          out[3 * n + 2] = nt;
        }
        ++n;
      }
  return n;
}

template bool panel_rot_compiled<float>(const PanelShape&);
template bool panel_rot_compiled<double>(const PanelShape&);
template bool panel_rot_compiled<cf>(const PanelShape&);
template bool panel_rot_compiled<cd>(const PanelShape&);
template bool panel_rot_config<float>(int, PanelShape&);
template bool panel_rot_config<double>(int, PanelShape&);
template bool panel_rot_config<cf>(int, PanelShape&);
template bool panel_rot_config<cd>(int, PanelShape&);
template void launch_panel_rot<float>(const GjDesc<float>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<double>(const GjDesc<double>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<cf>(const GjDesc<cf>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_rot<cd>(const GjDesc<cd>*, int, int, int, const PanelShape&, hipStream_t);
template void launch_panel_tourn<float>(const GjDesc<float>*, int, int, int, int, int*, hipStream_t);
template void launch_panel_tourn<double>(const GjDesc<double>*, int, int, int, int, int*, hipStream_t);
template void launch_panel_tourn<cd>(const GjDesc<cd>*, int, int, int, int, int*, hipStream_t);

}  // namespace hss
