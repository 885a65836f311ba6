// Four-step line passes for extended lengths 48, 64, 80, 108, 125, 128, 162, 240, 243, 320, 450, 512 (one
// instantiation each: one unit per two-wave workgroup, tables from global).
#include "line4_impl.h"

namespace rte {

template <typename T>
static hipError_t extra(const Lines4Args<T>& a, bool adj, hipStream_t s) {
  switch (a.fc.Np) {
    case 48: return adj ? go_one<T, true, 6, 8>(a, s) : go_one<T, false, 6, 8>(a, s);
    case 64: return adj ? go_one<T, true, 8, 8>(a, s) : go_one<T, false, 8, 8>(a, s);
    case 80: return adj ? go_one<T, true, 8, 10>(a, s) : go_one<T, false, 8, 10>(a, s);
    case 108: return adj ? go_one<T, true, 9, 12>(a, s) : go_one<T, false, 9, 12>(a, s);
    case 125: return adj ? go_one<T, true, 5, 25>(a, s) : go_one<T, false, 5, 25>(a, s);
    case 128: return adj ? go_one<T, true, 8, 16>(a, s) : go_one<T, false, 8, 16>(a, s);
    case 162: return adj ? go_one<T, true, 9, 18>(a, s) : go_one<T, false, 9, 18>(a, s);
    case 240: return adj ? go_one<T, true, 15, 16>(a, s) : go_one<T, false, 15, 16>(a, s);
    case 243: return adj ? go_one<T, true, 9, 27>(a, s) : go_one<T, false, 9, 27>(a, s);
    case 320: return adj ? go_one<T, true, 16, 20>(a, s) : go_one<T, false, 16, 20>(a, s);
    case 450: return adj ? go_one<T, true, 18, 25>(a, s) : go_one<T, false, 18, 25>(a, s);
    case 512: return adj ? go_one<T, true, 16, 32>(a, s) : go_one<T, false, 16, 32>(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t lines4_extra0(const Lines4Args<double>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }
hipError_t lines4_extra0(const Lines4Args<float>& a, bool adj, hipStream_t s) { return extra(a, adj, s); }

}  // namespace rte
