// Device helpers of the column-block kernel: lane exchange, the initial
// column, the run-length output and the in-place row update of Algorithm 1
// on a lane's columns.
#pragma once
#include "internal.h"

namespace colblock {

constexpr uint32_t kDppWaveShl1 = 0x130;

__device__ __forceinline__ uint32_t from_upper_lane(uint32_t x) {
    // lane l receives lane l+1's value; lane 63 receives 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppWaveShl1, 0xF, 0xF, true);
}

// Z of the initial column (i = n_w): bit j set iff m_w - j <= d
__device__ __forceinline__ uint64_t z_init(int mw, int d) {
    const int s = mw - d;
    return s <= 0 ? ~0ull : (s >= 64 ? 0ull : (~0ull << s));
}

__device__ __forceinline__ int zbit(uint64_t z, int p) { return p >= 64 ? 1 : (int)((z >> p) & 1ull); }

// Append `len` (>= 0) operations `op` to a pair's run list, merging equal
// neighbours; len == 0 changes nothing.
__device__ __forceinline__ void emit_run(int op, int len, int& cur_op, int& cur_len, int& nruns,
                                         uint32_t* __restrict__ runs, int64_t roff, int64_t rcap) {
    const bool same = cur_op == op;
    const bool flush = !same && cur_len > 0 && len > 0;
    if (flush && nruns < rcap) runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
    nruns += flush ? 1 : 0;
    cur_len = len == 0 ? cur_len : (same ? cur_len + len : len);
    cur_op = len == 0 ? cur_op : op;
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
    // second pass, also register-tied: ((right neighbour's row d) >> 1 | tm) & EQ
#pragma unroll
    for (int t = CB - 1; t >= 0; --t) {
        const uint32_t xl = t < CB - 1 ? P.lo[t + 1] : nl;
        const uint32_t xh = t < CB - 1 ? P.hi[t + 1] : nh;
        uint32_t bl, bh;
        // high half first: the next column's first instruction then reads
        // a result two instructions old
        asm volatile("v_alignbit_b32 %[bh], %[tm], %[xh], 1\n\t"
                     "v_alignbit_b32 %[bl], %[xh], %[xl], 1\n\t"
                     "v_and_or_b32 %[ph], %[bh], %[eh], %[ph]\n\t"
                     "v_and_or_b32 %[pl], %[bl], %[el], %[pl]"
                     : [pl] "+v"(P.lo[t]), [ph] "+v"(P.hi[t]), [bl] "=&v"(bl), [bh] "=&v"(bh)
                     : [xl] "v"(xl), [xh] "v"(xh), [tm] "v"(tm), [el] "v"(eq.lo[t]), [eh] "v"(eq.hi[t]));
    }
}

}  // namespace colblock
