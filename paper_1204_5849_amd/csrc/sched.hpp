// sched.hpp -- how the workgroups of a launch walk a Morton-ordered work list.
#pragma once

#include <hip/hip_runtime.h>

namespace mapk {

// Work items of a grid of G workgroups, mapped so that the workgroups that
// run on one XCD (workgroups are dealt to the 8 XCDs round robin) walk one
// contiguous range of the Morton-ordered list: neighbouring blocks then meet
// in that XCD's L2.  Workgroup b, the (b / 8)-th on XCD b % 8, processes the
// items first, first + stride, ... below end.  Every item is covered exactly
// once for any G >= 1.
__device__ __forceinline__ void xcd_range(int nitems, int &first, int &stride, int &end)
{
    const int G = gridDim.x, b = blockIdx.x;
    const int x = b & 7, l = b >> 3;
    const int full = G >> 3, rem = G & 7;
    const int cnt = full + (x < rem ? 1 : 0);             // workgroups on this XCD
    const int before = x * full + (x < rem ? x : rem);    // on the XCDs before it
    const long long lo = (long long)nitems * before / G;
    const long long hi = (long long)nitems * (before + cnt) / G;
    first = (int)lo + l;
    stride = cnt;
    end = (int)hi;
}

}  // namespace mapk
