// Four-step line passes for extended lengths 625..864 (625, 640, 648, 675, 720, 729, 750, 768, 800, 810, 864).
// Each length above 600 up to 1200 that splits into two factors of at most
// 40 is instantiated once (1125 = 3^2 5^3 has no such split and uses the
// generic kernel): one unit per two-wave workgroup, every table read from
// global memory.
#include "line4_impl.h"

namespace rte {

template <typename T>
static hipError_t longs(const Lines4Args<T>& a, bool adj, hipStream_t s) {
  switch (a.fc.Np) {
    case 625: return adj ? go_long<T, true, 25, 25>(a, s) : go_long<T, false, 25, 25>(a, s);
    case 640: return adj ? go_long<T, true, 32, 20>(a, s) : go_long<T, false, 32, 20>(a, s);
    case 648: return adj ? go_long<T, true, 27, 24>(a, s) : go_long<T, false, 27, 24>(a, s);
    case 675: return adj ? go_long<T, true, 27, 25>(a, s) : go_long<T, false, 27, 25>(a, s);
    case 720: return adj ? go_long<T, true, 30, 24>(a, s) : go_long<T, false, 30, 24>(a, s);
    case 729: return adj ? go_long<T, true, 27, 27>(a, s) : go_long<T, false, 27, 27>(a, s);
    case 750: return adj ? go_long<T, true, 30, 25>(a, s) : go_long<T, false, 30, 25>(a, s);
    case 768: return adj ? go_long<T, true, 32, 24>(a, s) : go_long<T, false, 32, 24>(a, s);
    case 800: return adj ? go_long<T, true, 32, 25>(a, s) : go_long<T, false, 32, 25>(a, s);
    case 810: return adj ? go_long<T, true, 30, 27>(a, s) : go_long<T, false, 30, 27>(a, s);
    case 864: return adj ? go_long<T, true, 32, 27>(a, s) : go_long<T, false, 32, 27>(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t lines4_long0(const Lines4Args<double>& a, bool adj, hipStream_t s) { return longs(a, adj, s); }
hipError_t lines4_long0(const Lines4Args<float>& a, bool adj, hipStream_t s) { return longs(a, adj, s); }

}  // namespace rte
