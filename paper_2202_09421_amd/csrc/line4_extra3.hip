// Four-step line passes for extended lengths 54, 96, 100, 144, 216, 225, 250, 324, 432, 486, 500 (one
// instantiation each: one unit per two-wave workgroup, tables from global).
#include "line4_impl.h"

namespace rte {

template <typename T>
static hipError_t extra(const Lines4Args<T>& a, bool adj, hipStream_t s) {
  switch (a.fc.Np) {
    case 54: return adj ? go_one<T, true, 6, 9>(a, s) : go_one<T, false, 6, 9>(a, s);
    case 96: return adj ? go_one<T, true, 8, 12>(a, s) : go_one<T, false, 8, 12>(a, s);
    case 100: return adj ? go_one<T, true, 10, 10>(a, s) : go_one<T, false, 10, 10>(a, s);
    case 144: return adj ? go_one<T, true, 12, 12>(a, s) : go_one<T, false, 12, 12>(a, s);
    case 216: return adj ? go_one<T, true, 12, 18>(a, s) : go_one<T, false, 12, 18>(a, s);
    case 225: return adj ? go_one<T, true, 15, 15>(a, s) : go_one<T, false, 15, 15>(a, s);
    case 250: return adj ? go_one<T, true, 10, 25>(a, s) : go_one<T, false, 10, 25>(a, s);
    case 324: return adj ? go_one<T, true, 18, 18>(a, s) : go_one<T, false, 18, 18>(a, s);
    case 432: return adj ? go_one<T, true, 18, 24>(a, s) : go_one<T, false, 18, 24>(a, s);
    case 486: return adj ? go_one<T, true, 18, 27>(a, s) : go_one<T, false, 18, 27>(a, s);
    case 500: return adj ? go_one<T, true, 20, 25>(a, s) : go_one<T, false, 20, 25>(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t lines4_extra3(const Lines4Args<double>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }
hipError_t lines4_extra3(const Lines4Args<float>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }

}  // namespace rte
