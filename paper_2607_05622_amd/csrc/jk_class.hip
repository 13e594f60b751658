// One canonical shell-quartet class per translation unit: compiled once per
// class index with -DJK_CLASS_INDEX=n so the generated recurrences build in
// parallel.  Defines launch_eri_tile_c<n> and launch_digest_c<n>.
#include "jk_device.h"

#ifndef JK_CLASS_INDEX
#error "compile with -DJK_CLASS_INDEX=<0..20>"
#endif

namespace jk {

#define JK_PASTE2(a, b) a##b
#define JK_PASTE(a, b) JK_PASTE2(a, b)

#define JK_DEFINE(idx, tag, la, lb, lc, ld)                                                       \
    static_assert(idx >= 0, "");                                                                  \
    hipError_t JK_PASTE(launch_eri_tile_c, idx)(const EriTileArgs& a, hipStream_t s) {            \
        const unsigned g = static_cast<unsigned>((a.nq + 255) / 256);                             \
        if constexpr (Eri##tag<double>::kSplit)                                                   \
            hipLaunchKernelGGL(k_eri_tile_split<Eri##tag<double>>, dim3(g), dim3(256), 0, s, a);  \
        else                                                                                      \
            hipLaunchKernelGGL(k_eri_tile<Eri##tag<double>>, dim3(g), dim3(256), 0, s, a);        \
        return hipGetLastError();                                                                 \
    }                                                                                             \
    hipError_t JK_PASTE(launch_digest_c, idx)(const DigestArgs& a, hipStream_t s) {               \
        constexpr int NA = (la + 1) * (la + 2) / 2, NB = (lb + 1) * (lb + 2) / 2;                  \
        const int W = a.colAw + a.colBw;                                                          \
        const size_t lds = sizeof(double) * ((a.want_k ? 2 * (NA + NB) * a.G * W : 0) +           \
                                             (a.want_j ? NA * NB * a.G : 0));                     \
        const unsigned g = static_cast<unsigned>(8 * ((a.nseg + 7) / 8) * a.ngroups);             \
        hipLaunchKernelGGL((k_digest<la, lb, lc, ld>), dim3(g), dim3(256), lds, s, a);            \
        return hipGetLastError();                                                                 \
    }                                                                                             \
    hipError_t JK_PASTE(digest_prepare_c, idx)(size_t lds_bytes) {                                \
        return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_digest<la, lb, lc, ld>),       \
                                   hipFuncAttributeMaxDynamicSharedMemorySize,                    \
                                   static_cast<int>(lds_bytes));                                  \
    }

#define JK_SELECT(idx, tag, la, lb, lc, ld) JK_SELECT_##idx(idx, tag, la, lb, lc, ld)
#if JK_CLASS_INDEX == 0
#define JK_SELECT_0(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_0(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 1
#define JK_SELECT_1(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_1(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 2
#define JK_SELECT_2(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_2(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 3
#define JK_SELECT_3(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_3(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 4
#define JK_SELECT_4(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_4(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 5
#define JK_SELECT_5(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_5(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 6
#define JK_SELECT_6(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_6(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 7
#define JK_SELECT_7(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_7(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 8
#define JK_SELECT_8(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_8(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 9
#define JK_SELECT_9(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_9(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 10
#define JK_SELECT_10(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_10(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 11
#define JK_SELECT_11(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_11(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 12
#define JK_SELECT_12(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_12(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 13
#define JK_SELECT_13(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_13(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 14
#define JK_SELECT_14(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_14(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 15
#define JK_SELECT_15(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_15(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 16
#define JK_SELECT_16(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_16(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 17
#define JK_SELECT_17(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_17(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 18
#define JK_SELECT_18(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_18(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 19
#define JK_SELECT_19(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_19(idx, tag, la, lb, lc, ld)
#endif
#if JK_CLASS_INDEX == 20
#define JK_SELECT_20(idx, tag, la, lb, lc, ld) JK_DEFINE(idx, tag, la, lb, lc, ld)
#else
#define JK_SELECT_20(idx, tag, la, lb, lc, ld)
#endif

JK_CLASS_LIST(JK_SELECT)

}  // namespace jk
