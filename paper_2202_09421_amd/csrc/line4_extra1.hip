// Four-step line passes for extended lengths 45, 60, 72, 120, 135, 192, 200, 300, 360, 384, 405, 600 (one
// instantiation each: one unit per two-wave workgroup, tables from global).
#include "line4_impl.h"

namespace rte {

template <typename T>
static hipError_t extra(const Lines4Args<T>& a, bool adj, hipStream_t s) {
  switch (a.fc.Np) {
    case 45: return adj ? go_one<T, true, 5, 9>(a, s) : go_one<T, false, 5, 9>(a, s);
    case 60: return adj ? go_one<T, true, 6, 10>(a, s) : go_one<T, false, 6, 10>(a, s);
    case 72: return adj ? go_one<T, true, 8, 9>(a, s) : go_one<T, false, 8, 9>(a, s);
    case 120: return adj ? go_one<T, true, 10, 12>(a, s) : go_one<T, false, 10, 12>(a, s);
    case 135: return adj ? go_one<T, true, 9, 15>(a, s) : go_one<T, false, 9, 15>(a, s);
    case 192: return adj ? go_one<T, true, 12, 16>(a, s) : go_one<T, false, 12, 16>(a, s);
    case 200: return adj ? go_one<T, true, 10, 20>(a, s) : go_one<T, false, 10, 20>(a, s);
    case 300: return adj ? go_one<T, true, 15, 20>(a, s) : go_one<T, false, 15, 20>(a, s);
    case 360: return adj ? go_one<T, true, 18, 20>(a, s) : go_one<T, false, 18, 20>(a, s);
    case 384: return adj ? go_one<T, true, 16, 24>(a, s) : go_one<T, false, 16, 24>(a, s);
    case 405: return adj ? go_one<T, true, 15, 27>(a, s) : go_one<T, false, 15, 27>(a, s);
    case 600: return adj ? go_one<T, true, 24, 25>(a, s) : go_one<T, false, 24, 25>(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t lines4_extra1(const Lines4Args<double>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }
hipError_t lines4_extra1(const Lines4Args<float>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }

}  // namespace rte
