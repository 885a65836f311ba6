// Four-step line passes for extended lengths 50, 75, 81, 150, 180, 256, 270, 375, 400, 480, 576 (one
// instantiation each: one unit per two-wave workgroup, tables from global).
#include "line4_impl.h"

namespace rte {

template <typename T>
static hipError_t extra(const Lines4Args<T>& a, bool adj, hipStream_t s) {
  switch (a.fc.Np) {
    case 50: return adj ? go_one<T, true, 5, 10>(a, s) : go_one<T, false, 5, 10>(a, s);
    case 75: return adj ? go_one<T, true, 5, 15>(a, s) : go_one<T, false, 5, 15>(a, s);
    case 81: return adj ? go_one<T, true, 9, 9>(a, s) : go_one<T, false, 9, 9>(a, s);
    case 150: return adj ? go_one<T, true, 10, 15>(a, s) : go_one<T, false, 10, 15>(a, s);
    case 180: return adj ? go_one<T, true, 12, 15>(a, s) : go_one<T, false, 12, 15>(a, s);
    case 256: return adj ? go_one<T, true, 16, 16>(a, s) : go_one<T, false, 16, 16>(a, s);
    case 270: return adj ? go_one<T, true, 15, 18>(a, s) : go_one<T, false, 15, 18>(a, s);
    case 375: return adj ? go_one<T, true, 15, 25>(a, s) : go_one<T, false, 15, 25>(a, s);
    case 400: return adj ? go_one<T, true, 20, 20>(a, s) : go_one<T, false, 20, 20>(a, s);
    case 480: return adj ? go_one<T, true, 20, 24>(a, s) : go_one<T, false, 20, 24>(a, s);
    case 576: return adj ? go_one<T, true, 24, 24>(a, s) : go_one<T, false, 24, 24>(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t lines4_extra2(const Lines4Args<double>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }
hipError_t lines4_extra2(const Lines4Args<float>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }

}  // namespace rte
