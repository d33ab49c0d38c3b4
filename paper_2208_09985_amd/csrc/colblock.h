// Device helpers of the column-block kernel: lane exchange, the initial
// column and the in-place row update of Algorithm 1 on a lane's columns.
#pragma once
#include "internal.h"

namespace colblock {

constexpr uint32_t kDppWaveShl1 = 0x130;

// Text columns per lane for NG windows of 64 / NG lanes each: enough to cover
// 64 columns, rounded up to whole groups of four (the row update's unit).
__host__ __device__ constexpr int cols_per_lane(int ng) {
    const int l = 64 / ng;
    return ((64 + l - 1) / l + 3) / 4 * 4;
}

__device__ __forceinline__ uint32_t from_upper_lane(uint32_t x) {
    // lane l receives lane l+1's value; lane 63 receives 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppWaveShl1, 0xF, 0xF, true);
}

// Z of the initial column (i = n_w): bit j set iff m_w - j <= d
__device__ __forceinline__ uint64_t z_init(int mw, int d) {
    const int s = mw - d;
    return s <= 0 ? ~0ull : (s >= 64 ? 0ull : (~0ull << s));
}

// One error row of the lane's CB columns: two VGPRs per column.
template <int CB>
struct RowRegs {
    uint32_t lo[CB], hi[CB];
};

// Row d of columns CB*q+CB-1 .. CB*q, in place over row d-1.  (nl, nh) is row d
// and (sl, sh) row d-1 of column CB*q+CB; tm and cin are the bits shifted in
// by the M term and by the I/S terms.  The I, S and D terms need only row
// d-1: with S[t] = Z[t] >> 1 | cin they are S[t] | S[t+1] | Z[t+1], and
// S[t+1] serves columns t and t+1, so a first pass shifts every column once
// and then ORs three terms per word in ascending order (each column still
// finds its right neighbour's old value).  The M term needs row d of the right
// neighbour, so a second pass runs from column CB*q+CB-1 down and ORs it in.
template <int CB>
__device__ __forceinline__ void dc_row(RowRegs<CB>& P, const RowRegs<CB>& eq, uint32_t nl, uint32_t nh, uint32_t sl,
                                       uint32_t sh, uint32_t tm, uint32_t cin) {
    // first pass as register-tied assembly: all shifts, then all ORs, so that
    // no instruction waits on the one just before it.  Left to itself the
    // compiler rotates the whole row through new registers every step.
    uint32_t ul[CB + 1], uh[CB + 1];
#pragma unroll
    for (int t = 0; t <= CB; ++t) {
        const uint32_t zl = t < CB ? P.lo[t] : sl;
        const uint32_t zh = t < CB ? P.hi[t] : sh;
        asm volatile("v_alignbit_b32 %[ul], %[zh], %[zl], 1\n\t"
                     "v_alignbit_b32 %[uh], %[cin], %[zh], 1"
                     : [ul] "=&v"(ul[t]), [uh] "=&v"(uh[t])
                     : [zl] "v"(zl), [zh] "v"(zh), [cin] "v"(cin));
    }
#pragma unroll
    for (int t = 0; t < CB; ++t) {
        const uint32_t xl = t < CB - 1 ? P.lo[t + 1] : sl;
        const uint32_t xh = t < CB - 1 ? P.hi[t + 1] : sh;
        asm volatile("v_or3_b32 %[pl], %[ul0], %[ul1], %[xl]\n\t"
                     "v_or3_b32 %[ph], %[uh0], %[uh1], %[xh]"
                     : [pl] "+v"(P.lo[t]), [ph] "+v"(P.hi[t])
                     : [ul0] "v"(ul[t]), [ul1] "v"(ul[t + 1]), [uh0] "v"(uh[t]), [uh1] "v"(uh[t + 1]), [xl] "v"(xl),
                       [xh] "v"(xh));
    }
    // second pass, also register-tied: ((right neighbour's row d) >> 1 | tm) & EQ,
    // eight (or four) columns per assembly statement: the compiler separates
    // consecutive statements that share registers by a wait state, as it cannot
    // see inside them.  High half first: each column's first instruction then
    // reads a result two instructions old.
#define SCG_MCOL(T, XH, XL)                                              \
    "v_alignbit_b32 %[bh], %[tm], %[" XH "], 1\n\t"                     \
    "v_alignbit_b32 %[bl], %[" XH "], %[" XL "], 1\n\t"                 \
    "v_and_or_b32 %[ph" #T "], %[bh], %[eh" #T "], %[ph" #T "]\n\t"     \
    "v_and_or_b32 %[pl" #T "], %[bl], %[el" #T "], %[pl" #T "]\n\t"
#define SCG_MOUT(T, U) [pl##T] "+v"(P.lo[U]), [ph##T] "+v"(P.hi[U])
#define SCG_MIN(T, U) [el##T] "v"(eq.lo[U]), [eh##T] "v"(eq.hi[U])
    if constexpr (CB % 8 == 0) {
#pragma unroll
        for (int t0 = CB - 8; t0 >= 0; t0 -= 8) {
            const uint32_t xl = t0 + 8 < CB ? P.lo[t0 + 8] : nl;
            const uint32_t xh = t0 + 8 < CB ? P.hi[t0 + 8] : nh;
            uint32_t bl, bh;
            asm volatile(SCG_MCOL(7, "xh", "xl") SCG_MCOL(6, "ph7", "pl7") SCG_MCOL(5, "ph6", "pl6")
                         SCG_MCOL(4, "ph5", "pl5") SCG_MCOL(3, "ph4", "pl4") SCG_MCOL(2, "ph3", "pl3")
                         SCG_MCOL(1, "ph2", "pl2") SCG_MCOL(0, "ph1", "pl1")
                         : SCG_MOUT(0, t0), SCG_MOUT(1, t0 + 1), SCG_MOUT(2, t0 + 2), SCG_MOUT(3, t0 + 3),
                           SCG_MOUT(4, t0 + 4), SCG_MOUT(5, t0 + 5), SCG_MOUT(6, t0 + 6), SCG_MOUT(7, t0 + 7),
                           [bl] "=&v"(bl), [bh] "=&v"(bh)
                         : [xl] "v"(xl), [xh] "v"(xh), [tm] "v"(tm), SCG_MIN(0, t0), SCG_MIN(1, t0 + 1),
                           SCG_MIN(2, t0 + 2), SCG_MIN(3, t0 + 3), SCG_MIN(4, t0 + 4), SCG_MIN(5, t0 + 5),
                           SCG_MIN(6, t0 + 6), SCG_MIN(7, t0 + 7));
        }
    } else {
        static_assert(CB % 4 == 0, "columns per lane come in fours");
#pragma unroll
        for (int t0 = CB - 4; t0 >= 0; t0 -= 4) {
            const uint32_t xl = t0 + 4 < CB ? P.lo[t0 + 4] : nl;
            const uint32_t xh = t0 + 4 < CB ? P.hi[t0 + 4] : nh;
            uint32_t bl, bh;
            asm volatile(SCG_MCOL(3, "xh", "xl") SCG_MCOL(2, "ph3", "pl3") SCG_MCOL(1, "ph2", "pl2")
                         SCG_MCOL(0, "ph1", "pl1")
                         : SCG_MOUT(0, t0), SCG_MOUT(1, t0 + 1), SCG_MOUT(2, t0 + 2), SCG_MOUT(3, t0 + 3),
                           [bl] "=&v"(bl), [bh] "=&v"(bh)
                         : [xl] "v"(xl), [xh] "v"(xh), [tm] "v"(tm), SCG_MIN(0, t0), SCG_MIN(1, t0 + 1),
                           SCG_MIN(2, t0 + 2), SCG_MIN(3, t0 + 3));
        }
    }
#undef SCG_MIN
#undef SCG_MOUT
#undef SCG_MCOL
}

}  // namespace colblock
