// Host-side dispatch of runtime (p, precision) onto kernel template
// instantiations.
#pragma once

#include "bfsft_impl.h"

namespace bfsft {

template <int P> struct PTag { static constexpr int value = P; };

// 2D grids: p = 3..12
template <typename F> void dispatch_p(int p, F &&f)
{
    switch (p) {
    case 3: f(PTag<3>{}); break;
    case 4: f(PTag<4>{}); break;
    case 5: f(PTag<5>{}); break;
    case 6: f(PTag<6>{}); break;
    case 7: f(PTag<7>{}); break;
    case 8: f(PTag<8>{}); break;
    case 9: f(PTag<9>{}); break;
    case 10: f(PTag<10>{}); break;
    case 11: f(PTag<11>{}); break;
    case 12: f(PTag<12>{}); break;
    default: throw Error{BFSFT_EINVAL, "unsupported p"};
    }
}

// 3D grids: p = 3..8
template <typename F> void dispatch_p3(int p, F &&f)
{
    switch (p) {
    case 3: f(PTag<3>{}); break;
    case 4: f(PTag<4>{}); break;
    case 5: f(PTag<5>{}); break;
    case 6: f(PTag<6>{}); break;
    case 7: f(PTag<7>{}); break;
    case 8: f(PTag<8>{}); break;
    default: throw Error{BFSFT_EINVAL, "unsupported p in 3D"};
    }
}

// (state scalar, compute scalar) of each precision
template <typename F> void dispatch_prec(int precision, F &&f)
{
    switch (precision) {
    case BFSFT_FP64: f((double *)nullptr, (double *)nullptr); break;
    case BFSFT_MIXED: f((float *)nullptr, (double *)nullptr); break;
    case BFSFT_FP32: f((float *)nullptr, (float *)nullptr); break;
    default: throw Error{BFSFT_EINVAL, "unsupported precision"};
    }
}

}  // namespace bfsft
