// Four-step line passes for extended lengths 900..1200 (900, 960, 972, 1000, 1024, 1080, 1152, 1200).
// Each length above 600 up to 1200 that splits into two factors of at most
// 40 is instantiated once (1125 = 3^2 5^3 has no such split and uses the
// generic kernel): one unit per two-wave workgroup, every table read from
// global memory.
#include "line4_impl.h"

namespace rte {

template <typename T>
static hipError_t longs(const Lines4Args<T>& a, bool adj, hipStream_t s) {
  switch (a.fc.Np) {
    case 900: return adj ? go_long<T, true, 30, 30>(a, s) : go_long<T, false, 30, 30>(a, s);
    case 960: return adj ? go_long<T, true, 32, 30>(a, s) : go_long<T, false, 32, 30>(a, s);
    case 972: return adj ? go_long<T, true, 27, 36>(a, s) : go_long<T, false, 27, 36>(a, s);
    case 1000: return adj ? go_long<T, true, 25, 40>(a, s) : go_long<T, false, 25, 40>(a, s);
    case 1024: return adj ? go_long<T, true, 32, 32>(a, s) : go_long<T, false, 32, 32>(a, s);
    case 1080: return adj ? go_long<T, true, 30, 36>(a, s) : go_long<T, false, 30, 36>(a, s);
    case 1152: return adj ? go_long<T, true, 32, 36>(a, s) : go_long<T, false, 32, 36>(a, s);
    case 1200: return adj ? go_long<T, true, 30, 40>(a, s) : go_long<T, false, 30, 40>(a, s);
    default: return hipErrorNotSupported;
  }
}

hipError_t lines4_long1(const Lines4Args<double>& a, bool adj, hipStream_t s) { return longs(a, adj, s); }
hipError_t lines4_long1(const Lines4Args<float>& a, bool adj, hipStream_t s) { return longs(a, adj, s); }

}  // namespace rte
