// Four-step line passes: launch code for all extended lengths, full set of
// tuned variants for N_p in {90, 160, 288, 540}.
#include "line4_impl.h"

namespace rte {

// N_p = N1 x N2 with both factors products of 2, 3, 4, 5 (register codelets):
// up to 600 both at most 32 (one pass over the lanes of a two-wave
// workgroup); above, N1 <= 32 and N2 <= 40.
bool fourstep_split(int Np, int* n1, int* n2) {
  switch (Np) {
    case 45: *n1 = 5; *n2 = 9; return true;
    case 48: *n1 = 6; *n2 = 8; return true;
    case 50: *n1 = 5; *n2 = 10; return true;
    case 54: *n1 = 6; *n2 = 9; return true;
    case 60: *n1 = 6; *n2 = 10; return true;
    case 64: *n1 = 8; *n2 = 8; return true;
    case 72: *n1 = 8; *n2 = 9; return true;
    case 75: *n1 = 5; *n2 = 15; return true;
    case 80: *n1 = 8; *n2 = 10; return true;
    case 81: *n1 = 9; *n2 = 9; return true;
    case 90: *n1 = 9; *n2 = 10; return true;
    case 96: *n1 = 8; *n2 = 12; return true;
    case 100: *n1 = 10; *n2 = 10; return true;
    case 108: *n1 = 9; *n2 = 12; return true;
    case 120: *n1 = 10; *n2 = 12; return true;
    case 125: *n1 = 5; *n2 = 25; return true;
    case 128: *n1 = 8; *n2 = 16; return true;
    case 135: *n1 = 9; *n2 = 15; return true;
    case 144: *n1 = 12; *n2 = 12; return true;
    case 150: *n1 = 10; *n2 = 15; return true;
    case 160: *n1 = 16; *n2 = 10; return true;
    case 162: *n1 = 9; *n2 = 18; return true;
    case 180: *n1 = 12; *n2 = 15; return true;
    case 192: *n1 = 12; *n2 = 16; return true;
    case 200: *n1 = 10; *n2 = 20; return true;
    case 216: *n1 = 12; *n2 = 18; return true;
    case 225: *n1 = 15; *n2 = 15; return true;
    case 240: *n1 = 15; *n2 = 16; return true;
    case 243: *n1 = 9; *n2 = 27; return true;
    case 250: *n1 = 10; *n2 = 25; return true;
    case 256: *n1 = 16; *n2 = 16; return true;
    case 270: *n1 = 15; *n2 = 18; return true;
    case 288: *n1 = 16; *n2 = 18; return true;
    case 300: *n1 = 15; *n2 = 20; return true;
    case 320: *n1 = 16; *n2 = 20; return true;
    case 324: *n1 = 18; *n2 = 18; return true;
    case 360: *n1 = 18; *n2 = 20; return true;
    case 375: *n1 = 15; *n2 = 25; return true;
    case 384: *n1 = 16; *n2 = 24; return true;
    case 400: *n1 = 20; *n2 = 20; return true;
    case 405: *n1 = 15; *n2 = 27; return true;
    case 432: *n1 = 18; *n2 = 24; return true;
    case 450: *n1 = 18; *n2 = 25; return true;
    case 480: *n1 = 20; *n2 = 24; return true;
    case 486: *n1 = 18; *n2 = 27; return true;
    case 500: *n1 = 20; *n2 = 25; return true;
    case 512: *n1 = 16; *n2 = 32; return true;
    case 540: *n1 = 20; *n2 = 27; return true;
    case 576: *n1 = 24; *n2 = 24; return true;
    case 600: *n1 = 24; *n2 = 25; return true;
    // above 600: both factors at most 40 (long-line variant)
    case 625: *n1 = 25; *n2 = 25; return true;
    case 640: *n1 = 32; *n2 = 20; return true;
    case 648: *n1 = 27; *n2 = 24; return true;
    case 675: *n1 = 27; *n2 = 25; return true;
    case 720: *n1 = 30; *n2 = 24; return true;
    case 729: *n1 = 27; *n2 = 27; return true;
    case 750: *n1 = 30; *n2 = 25; return true;
    case 768: *n1 = 32; *n2 = 24; return true;
    case 800: *n1 = 32; *n2 = 25; return true;
    case 810: *n1 = 30; *n2 = 27; return true;
    case 864: *n1 = 32; *n2 = 27; return true;
    case 900: *n1 = 30; *n2 = 30; return true;
    case 960: *n1 = 32; *n2 = 30; return true;
    case 972: *n1 = 27; *n2 = 36; return true;
    case 1000: *n1 = 25; *n2 = 40; return true;
    case 1024: *n1 = 32; *n2 = 32; return true;
    case 1080: *n1 = 30; *n2 = 36; return true;
    case 1152: *n1 = 32; *n2 = 36; return true;
    case 1200: *n1 = 30; *n2 = 40; return true;
    default: return false;
  }
}

template <typename T, bool ADJ, int N1, int N2>
static hipError_t go(const Lines4Args<T>& a, int upw, int nw, int tg, hipStream_t s) {
  if (tg) return nw == 2 ? go_nw<T, ADJ, N1, N2, 2, true>(a, upw, s) : go_nw<T, ADJ, N1, N2, 1, true>(a, upw, s);
  return nw == 2 ? go_nw<T, ADJ, N1, N2, 2, false>(a, upw, s) : go_nw<T, ADJ, N1, N2, 1, false>(a, upw, s);
}

template <typename T, bool ADJ>
static hipError_t by_size(const Lines4Args<T>& a, int upw, int nw, int tg, hipStream_t s) {
  switch (a.fc.Np) {
    case 90: return go<T, ADJ, 9, 10>(a, upw, nw, tg, s);
    case 160: return go<T, ADJ, 16, 10>(a, upw, nw, tg, s);
    case 288: return go<T, ADJ, 16, 18>(a, upw, nw, tg, s);
    case 540: return go<T, ADJ, 20, 27>(a, upw, nw, tg, s);
    default: {
      hipError_t e = lines4_extra0(a, ADJ, s);
      if (e == hipErrorNotSupported) e = lines4_extra1(a, ADJ, s);
      if (e == hipErrorNotSupported) e = lines4_extra2(a, ADJ, s);
      if (e == hipErrorNotSupported) e = lines4_extra3(a, ADJ, s);
      if (e == hipErrorNotSupported) e = lines4_long0(a, ADJ, s);
      if (e == hipErrorNotSupported) e = lines4_long1(a, ADJ, s);
      return e;
    }
  }
}

template <typename T>
static hipError_t launch4_t(const Plan& p, const LineLaunch& L, hipStream_t s) {
  Lines4Args<T> a;
  a.in = static_cast<const T*>(L.in);
  a.out[0] = static_cast<T*>(L.out_x);
  a.out[1] = static_cast<T*>(L.out_y);
  a.coef[0] = p.dev.xi;
  a.coef[1] = p.dev.eta;
  a.nlines[0] = (int)p.ny;
  a.nlines[1] = (int)p.nx;
  a.line_stride[0] = p.nxp * kGroup;
  a.pt_stride[0] = kGroup;
  a.line_stride[1] = kGroup;
  a.pt_stride[1] = p.nxp * kGroup;
  for (int k = 0; k < 2; ++k) {
    const int np = (a.nlines[k] + 1) / 2;
    a.npe[k] = np + (np & 1);
  }
  a.grp_stride = p.grp_stride;
  a.inst_stride = p.inst_stride;
  a.G = (int)p.G;
  a.nt_out = p.stream_nt ? 1 : 0;
  const bool dx = (L.dirs & 1) != 0, dy = (L.dirs & 2) != 0;
  a.dir_first = dx ? 0 : 1;
  a.fc = dx ? p.fcx : p.fcy;
  const int64_t per = p.cnq * p.G;
  a.units_first = (int)(per * a.npe[a.dir_first]);
  a.nunits = a.units_first + ((dx && dy) ? (int)(per * a.npe[1]) : 0);
  const int upw = p.sched.line_units_per_wave, nw = p.sched.line_waves_per_unit, tg = p.sched.line_global_tables;
  return L.mode == LINE_ADJ ? by_size<T, true>(a, upw, nw, tg, s) : by_size<T, false>(a, upw, nw, tg, s);
}

hipError_t launch_lines4(const Plan& p, const LineLaunch& L, hipStream_t s) {
  if (p.dtype == RTE_F64) return launch4_t<double>(p, L, s);
  return launch4_t<float>(p, L, s);
}

}  // namespace rte
