// fixed_point.h -- exact, order-independent sums of FP64 values: a value is
// split into a multiple of 2^-30 and the remainder, both held as int64 (the
// remainder in units of 2^-80), and the two integer sums are exact whatever
// the order of the additions.  Used where FP64 sums would otherwise depend on
// the order atomics or unsorted lists deliver their terms: the spread
// coupling force of the FP64 form and the soft-sphere pair forces.
#pragma once

#include "device_common.h"

namespace oif {
namespace dev {

// v = hi 2^-30 + lo 2^-80 + (a rounding below 2^-81); false (and zeros) for
// |v| >= 2^25 or a non-finite v.  The bound keeps |hi| below 2^55, so a sum
// of up to 256 values cannot leave the int64 range (|lo| stays below 2^49).
// v - hi 2^-30 is exact: hi 2^-30 is v rounded to a multiple of 2^-30, so it
// is 0 or within a factor 2 of v.
__device__ __forceinline__ bool fx_split(double v, long long& hi, long long& lo) {
    if (!(fabs(v) < 0x1p25)) {
        hi = lo = 0;
        return false;
    }
    const double h = rint(v * 0x1p30);
    hi = (long long)h;
    lo = __double2ll_rn((v - h * 0x1p-30) * 0x1p80);
    return true;
}

// the value of the sums hi (units of 2^-30) and lo (units of 2^-80)
__device__ __forceinline__ double fx_value(long long hi, long long lo) {
    return (double)hi * 0x1p-30 + (double)lo * 0x1p-80;
}

}  // namespace dev
}  // namespace oif
