// Group shapes of the support classes and the dispatch from run-time
// (class, input type, start rule) to a compiled kernel instance.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "d2_internal.h"
#include "d2_solver.h"

namespace d2 {

// ------------------------------------------------------------------ shapes

template <int CLS> struct Shape;
// G: lanes per pair; GS: column capacity; waves per workgroup; occ: waves per
// SIMD the register allocation is held to (the pivot loop waits on LDS and
// lane exchanges, so more resident waves beat a few spilled registers:
// measured best at 4 / 3 / 2 / 1).
template <> struct Shape<0> { static constexpr int G = 16, GS = 16, waves = 4, occ = 4; static constexpr bool LT = false; };
template <> struct Shape<1> { static constexpr int G = 32, GS = 32, waves = 4, occ = 3; static constexpr bool LT = false; };
template <> struct Shape<2> { static constexpr int G = 64, GS = 32, waves = 2, occ = 2; static constexpr bool LT = false; };
template <> struct Shape<3> { static constexpr int G = 64, GS = 64, waves = 1, occ = 2; static constexpr bool LT = true; };

template <int CLS>
struct ShapeCfg {
    static constexpr int G = Shape<CLS>::G, GS = Shape<CLS>::GS;
    static constexpr bool LT = Shape<CLS>::LT;
    static constexpr int threads = Shape<CLS>::waves * 64;
    static constexpr int occ = Shape<CLS>::occ;
    static constexpr int groups = threads / G;
};

// LDS tile of a shape and start rule: Vogel's start scans columns and keeps
// the whole tile; otherwise only the widest shape keeps its upper columns.
template <int CLS, int START>
using TileOf = typename std::conditional<
    START == kStartVogel, Tile<Shape<CLS>::G, Shape<CLS>::GS>,
    typename std::conditional<Shape<CLS>::LT, TileHalf<Shape<CLS>::G, Shape<CLS>::GS>, NoTile>::type>::type;

__host__ __device__ inline int class_of(int64_t T, int64_t S) {
    if (T <= 16) return 0;
    if (T <= 32) return 1;
    return S <= 32 ? 2 : 3;
}

// Calls f.run<class, input type, start rule>() for a run-time choice.
template <typename F>
inline hipError_t dispatch_class(int cls, bool f32, int start, F &&f) {
#define D2_CASE(C)                                                                      \
    case C:                                                                             \
        if (f32) return start == kStartVogel ? f.template run<C, float, kStartVogel>()             \
                      : start == kStartLCM ? f.template run<C, float, kStartLCM>()                   \
                                           : f.template run<C, float, kStartNWC>();                  \
        return start == kStartVogel ? f.template run<C, double, kStartVogel>()                       \
               : start == kStartLCM ? f.template run<C, double, kStartLCM>()                         \
                                    : f.template run<C, double, kStartNWC>();
    switch (cls) {
        D2_CASE(0)
        D2_CASE(1)
        D2_CASE(2)
        default: D2_CASE(3)
    }
#undef D2_CASE
}

}  // namespace d2
