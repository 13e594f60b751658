// One canonical shell-quartet class per translation unit: compiled once per
// class index with -DJK_CLASS_INDEX=n so the generated recurrences build in
// parallel.  Defines launch_eri_tile_c<n> and launch_digest_c<n>.
#include "jk_digest.h"
#include "jk_digest2.h"

#ifndef JK_CLASS_INDEX
#error "compile with -DJK_CLASS_INDEX=<0..20>"
#endif

namespace jk {

#define JK_PASTE2(a, b) a##b
#define JK_PASTE(a, b) JK_PASTE2(a, b)

// Integral launches are grid-stride: enough blocks to fill the chip, each
// walking the item blocks of the launch.
constexpr long long kEriGridCap = 256 * 8;

template <class C, typename R>
hipError_t launch_eri_tpl(const EriTileArgs& a, hipStream_t s) {
    const int block = (a.block == 64 || a.block == 128) ? a.block : 256;
    const long long cap = kEriGridCap * (256 / block);
    const unsigned g = static_cast<unsigned>(a.nblocks < cap ? a.nblocks : cap);
    hipLaunchKernelGGL((k_eri_tile<C, R>), dim3(g), dim3(block), 0, s, a);
    return hipGetLastError();
}

// Digestion.  kernel 2: wave-private tasks (jk_digest2.h), four per
// workgroup, for classes of at most 408 functions per quartet.  Otherwise
// one workgroup per task; pass C has a J wave and one K wave per density
// form, pass D one K wave per density form; kernel 3 is pass C in its
// one-pass form.
template <int la, int lb, int lc, int ld, typename TT>
hipError_t launch_digest_tpl(const DigestArgs& a, hipStream_t s, int pass, int g16, int kernel) {
    constexpr int nf = ncart(la) * ncart(lb) * ncart(lc) * ncart(ld);
    if constexpr (dig2_class(la, lb, lc, ld, nf) && sizeof(TT) == 8) if (kernel == 2) {
        const dim3 grid(8 * ((a.nblocks / 8 + kDig2Waves - 1) / kDig2Waves));
        const dim3 block(64 * kDig2Waves);
        if (pass == 0) {
            if (g16) hipLaunchKernelGGL((k_digest2_c<la, lb, lc, ld, TT, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_digest2_c<la, lb, lc, ld, TT, false>), grid, block, 0, s, a);
        } else {
            if (g16) hipLaunchKernelGGL((k_digest2_d<la, lb, lc, ld, TT, true>), grid, block, 0, s, a);
            else hipLaunchKernelGGL((k_digest2_d<la, lb, lc, ld, TT, false>), grid, block, 0, s, a);
        }
        return hipGetLastError();
    }
    const dim3 grid(a.nblocks);
    // 16-density groups: the last wave takes the D^T contractions, left out
    // when the densities are symmetric.  kernel 3: pass C alone takes all
    // four K blocks (its plans have no pass D items).
    if (kernel == 3) {
        if (pass != 0) return hipSuccess;
        if (g16) hipLaunchKernelGGL((k_digest_c<la, lb, lc, ld, TT, true, true>), grid, dim3(a.skip_t ? 128 : 192), 0, s, a);
        else hipLaunchKernelGGL((k_digest_c<la, lb, lc, ld, TT, false, true>), grid, dim3(128), 0, s, a);
        return hipGetLastError();
    }
    if (pass == 0) {
        if (g16) hipLaunchKernelGGL((k_digest_c<la, lb, lc, ld, TT, true>), grid, dim3(a.skip_t ? 128 : 192), 0, s, a);
        else hipLaunchKernelGGL((k_digest_c<la, lb, lc, ld, TT, false>), grid, dim3(128), 0, s, a);
    } else if constexpr (sizeof(TT) == 8 && dig_d4(la, lb, lc, ld)) {
        if (g16) hipLaunchKernelGGL((k_digest_d4<la, lb, lc, ld, true>), grid, dim3(a.skip_t ? 64 : 128), 0, s, a);
        else hipLaunchKernelGGL((k_digest_d4<la, lb, lc, ld, false>), grid, dim3(64), 0, s, a);
    } else {
        if (g16) hipLaunchKernelGGL((k_digest_d<la, lb, lc, ld, TT, true>), grid, dim3(a.skip_t ? 64 : 128), 0, s, a);
        else hipLaunchKernelGGL((k_digest_d<la, lb, lc, ld, TT, false>), grid, dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

#define JK_DEFINE(idx, tag, la, lb, lc, ld)                                                        \
    hipError_t JK_PASTE(launch_eri_tile_c, idx)(const EriTileArgs& a, hipStream_t s, int fp32) {   \
        return fp32 ? launch_eri_tpl<Eri##tag<float>, float>(a, s)                                 \
                    : launch_eri_tpl<Eri##tag<double>, double>(a, s);                              \
    }                                                                                              \
    hipError_t JK_PASTE(launch_digest_c, idx)(const DigestArgs& a, hipStream_t s, int fp32, int pass, int g16, \
                                              int kernel) {                                        \
        return fp32 ? launch_digest_tpl<la, lb, lc, ld, float>(a, s, pass, g16, kernel)            \
                    : launch_digest_tpl<la, lb, lc, ld, double>(a, s, pass, g16, kernel);          \
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
