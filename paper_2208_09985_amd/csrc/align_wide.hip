// Fused, persistent windowed GenASM-DC + GenASM-TB kernel for gfx950,
// windows of 65..128 characters, plain mode.
//
// The column-block mapping of align_cols.hip with 128-bit bitvectors:
//   * A wavefront holds NG = 4 or 8 windows of different pairs, one per group
//     of L = 64/NG lanes; lane q owns the CB = 128/L text columns
//     CB*q .. CB*q+CB-1.  A column's entry of the current error row is four
//     VGPRs (word k holds pattern bits 32k..32k+31, stored complemented:
//     Z = ~R, bit j of Z set iff D_w(i, j) <= d), and so is its match mask.
//   * Rows of Algorithm 1 (Section 2.2.1) are computed one per step, the
//     lanes of a group skewed by one step; the row and the previous row of
//     the next lane's first column arrive by DPP, and the last lane makes the
//     initial column itself.  The update is the same two passes as for
//     64-bit entries (I/S/D terms from row d-1 in ascending column order, the
//     M term from row d of the right neighbour in descending order), with
//     each shift by one running across four words.
//   * Early termination (Section 2.4.3) is exact: lane 0 of a group holds
//     column 0, and one ballot per step finds the first row whose entry has
//     the msb of R clear.
//   * Entries of rows 0..127, columns 0..min(W-O, 127) (Sections 2.4.1 and
//     2.4.2) go to a per-group region of global memory, 16 bytes per entry,
//     or 12 (the low 96 bits) when W-O <= 95 and 8 when W-O <= 63, as
//     traceback reads bits 0..W-O only; the traceback of each finished
//     window runs in its group's lane 0.
#include "colblock.h"

namespace {

using namespace colblock;

constexpr int kRowsW = 128;       // rows 0..127 are kept for traceback
constexpr int kTbEventsW = 64;    // traceback events per round
enum : int { W_EMPTY = 0, W_RUN = 1, W_DONE = 2, W_TB = 4 };

// A 128-bit pattern-indexed vector: bit j in lo for j < 64, in hi otherwise.
struct V128 {
    uint64_t lo, hi;
};

__device__ __forceinline__ V128 shr128(V128 v, int s) {   // s >= 0
    if (s >= 128) return V128{0ull, 0ull};
    if (s >= 64) return V128{v.hi >> (s - 64), 0ull};
    if (s == 0) return v;
    return V128{(v.lo >> s) | (v.hi << (64 - s)), v.hi >> s};
}

__device__ __forceinline__ int ctz128(V128 x) {
    return x.lo ? (int)__builtin_ctzll(x.lo) : (x.hi ? 64 + (int)__builtin_ctzll(x.hi) : 128);
}

__device__ __forceinline__ int zbit128(V128 z, int p) {
    if (p >= 128) return 1;
    return (int)(((p < 64) ? (z.lo >> p) : (z.hi >> (p - 64))) & 1ull);
}

// Z of the initial column (i = n_w) at row d: bit j set iff m_w - j <= d
__device__ __forceinline__ V128 z_init128(int mw, int d) {
    const int s = mw - d;
    if (s <= 0) return V128{~0ull, ~0ull};
    if (s >= 128) return V128{0ull, 0ull};
    if (s >= 64) return V128{0ull, ~0ull << (s - 64)};
    return V128{~0ull << s, ~0ull};
}

// 128 bases from position pos of a sequence's planes (three Plane2 words;
// sequences of this layout end with two zero padding words)
__device__ __forceinline__ void load_window128(const Plane2* __restrict__ base, int pos, V128& lo, V128& hi) {
    const int w = pos >> 6, r = pos & 63;
    const Plane2 a = base[w], b = base[w + 1], c = base[w + 2];
    if (r == 0) {
        lo = V128{a.lo, b.lo};
        hi = V128{a.hi, b.hi};
    } else {
        lo = V128{(a.lo >> r) | (b.lo << (64 - r)), (b.lo >> r) | (c.lo << (64 - r))};
        hi = V128{(a.hi >> r) | (b.hi << (64 - r)), (b.hi >> r) | (c.hi << (64 - r))};
    }
}

struct GroupRecW {     // LDS: what the slot lane tells its group at set-up
    V128 plo, phi, tlo, thi;   // window planes (pattern at p0, text at t0)
    int32_t m_w, n_w, full, fresh;
};

// a stored entry's low 96 bits
struct __attribute__((packed, aligned(4))) W3 {
    uint32_t x, y, z;
};

__device__ __forceinline__ uint32_t word_of(V128 v, int k) {
    return (uint32_t)((k < 2 ? v.lo : v.hi) >> (32 * (k & 1)));
}

// Occupancy target: three wavefronts per SIMD with 4 windows each (168
// VGPRs), two with 8 (256), so that 10,000 pairs are resident at once.
// SW: 32-bit words kept per stored entry.  Traceback reads bits 0..W-O only, so
// with W-O <= 95 the entries keep their low 96 bits (SW = 3) and with W-O <= 63
// their low 64 (SW = 2); the other words are never written or read.
template <int NG, int SW>
__global__ __launch_bounds__(64, NG == 4 ? 3 : 2) void wide_kernel(const AlignArgs a) {
    constexpr int L = 64 / NG;      // lanes per window
    constexpr int CB = 128 / L;     // columns per lane
    __shared__ GroupRecW grec[NG];
    const int lane = threadIdx.x;
    const int g = lane / L, q = lane % L;
    const bool slot = q == 0;
    const uint64_t gbit = 1ull << (lane - q);   // the group's slot lane in a ballot
    const int cap = a.cap;
    const int stride = a.dstride;               // stored entries per row (16 or 12 bytes each)
    // the block's stored rows start at a wavefront-uniform address; a lane reaches its
    // group's entries with a 32-bit byte offset (a group holds 128 rows of `stride` entries)
    char* const bdent = reinterpret_cast<char*>(reinterpret_cast<uint4*>(a.dent) + (size_t)blockIdx.x * NG * (size_t)(kRowsW * stride));
    const uint32_t gbyte = (uint32_t)(g * kRowsW * stride) * 16u;
    constexpr uint32_t ESZ = 4u * SW;                          // bytes per stored entry
    const uint32_t qbyte = gbyte + (uint32_t)(CB * q) * ESZ;   // the lane's first column in row 0
    const uint32_t rowbytes = (uint32_t)stride * ESZ;
    const bool storer = CB * q < stride;

    if (lane < NG) grec[lane] = GroupRecW{{0, 0}, {0, 0}, {0, 0}, {0, 0}, 0, 0, 0, 0};

    // ---- slot-lane state ----
    int pair = -1, p0 = 0, t0 = 0, m = 0, n = 0, edits = 0, nruns = 0, cur_op = 0, cur_len = 0;
    int mw = 0, nw = 0, kw = 0;
    int64_t roff = 0, rcap = 0, pending = -1;
    bool exhausted = !slot;
    unsigned long long c_windows = 0, c_ops = 0, c_rows = 0, c_err = 0;
    V128 tb_rc{0ull, 0ull};   // slot lane: the initial column at row tb_d - 1 (Z beyond the text window)
    int tb_i = 0, tb_j = 0, tb_d = 0, tb_e = 0, tb_bad = 0;
    unsigned long long c_lane_steps = 0, c_rounds = 0;

    // ---- lane state: word k of the current row / match mask of column t ----
    uint32_t A[4][CB], E[4][CB];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int t = 0; t < CB; ++t) A[k][t] = E[k][t] = 0;
    uint32_t nbs[4] = {0, 0, 0, 0};   // row d-1 of column CB*q+CB
    uint32_t zr[4] = {0, 0, 0, 0};    // initial column at the lane's next row (used by q == L-1)
    int dl = 0;
    int gst = W_EMPTY;
    int full = 0, dw = -1;

    for (;;) {
        // ---- 1. slot lanes take pairs from the queue ----
        if (!exhausted && pair < 0) {
            if (pending < 0) pending = (int64_t)atomicAdd(&a.qctl[0], 1u);
            if (pending >= a.npairs) {
                exhausted = true;
            } else {
                const int polled = __hip_atomic_load(&a.ring[pending], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (polled != 0) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    const int pid = polled - 1;
                    pending = -1;
                    const int pm = a.plen[pid], pn = a.tlen[pid];
                    if (a.bad[pid] || pm == 0) {
                        const bool bad = a.bad[pid] != 0;
                        a.edits[pid] = bad ? -1 : 0;
                        a.text_end[pid] = bad ? -1 : 0;
                        a.status[pid] = bad ? 2 : 0;
                        a.n_runs[pid] = 0;
                        atomicAdd(&a.qctl[2], 1u);
                    } else {
                        pair = pid;
                        m = pm;
                        n = pn;
                        p0 = 0; t0 = 0; edits = 0; nruns = 0; cur_op = 0; cur_len = 0;
                        roff = a.runs_off[pid];
                        rcap = a.runs_off[pid + 1] - roff;
                    }
                }
            }
        }

        // ---- 2. slot lanes start windows ----
        if (slot) {
            GroupRecW& r = grec[g];
            if (gst == W_EMPTY && pair >= 0) {
                mw = min(a.W, m - p0);
                nw = min(a.W, n - t0);
                kw = min(a.k, mw);
                V128 plo, phi, tlo{0, 0}, thi{0, 0};
                load_window128(a.pplanes + a.pword[pair], p0, plo, phi);
                if (nw > 0) load_window128(a.tplanes + a.tword[pair], t0, tlo, thi);
                r.plo = plo;
                r.phi = phi;
                r.tlo = tlo;
                r.thi = thi;
                r.m_w = mw;
                r.n_w = nw;
                r.full = (kw == mw) ? mw : kw + 1;   // row m_w is implicit: D(0,0) <= m_w
                r.fresh = 1;
            } else {
                r.fresh = 0;
            }
        }
        __syncthreads();

        // ---- 3. every lane of a group with a new window builds its columns ----
        // A pass always runs its windows to the end, so no row survives a
        // round: every lane rebuilds its columns (from the group's current
        // record; only a fresh window's are used), which keeps the row and the
        // match masks out of the registers live across rounds.
        {
            const GroupRecW r = grec[g];
            {
                // bits j >= m_w of every entry and match mask are 1 (the empty pattern suffix)
                const V128 beyond{r.m_w >= 64 ? 0ull : (~0ull << r.m_w),
                                  r.m_w >= 128 ? 0ull : (r.m_w <= 64 ? ~0ull : (~0ull << (r.m_w - 64)))};
                const int ncols = min(max(r.n_w - CB * q, 0), CB);
#pragma unroll
                for (int t = 0; t < CB; ++t) {
                    const int c = CB * q + t;   // text column, < 128
                    const uint64_t tl = c < 64 ? (r.tlo.lo >> c) : (r.tlo.hi >> (c - 64));
                    const uint64_t th = c < 64 ? (r.thi.lo >> c) : (r.thi.hi >> (c - 64));
                    const V128 sl = (tl & 1ull) ? r.plo : V128{~r.plo.lo, ~r.plo.hi};
                    const V128 sh = (th & 1ull) ? r.phi : V128{~r.phi.lo, ~r.phi.hi};
                    const bool in = t < ncols;
                    const V128 e{(in ? (sl.lo & sh.lo) : 0ull) | beyond.lo, (in ? (sl.hi & sh.hi) : 0ull) | beyond.hi};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        E[k][t] = word_of(e, k);
                        A[k][t] = 0;
                    }
                }
                const V128 z = z_init128(r.m_w, 0);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    nbs[k] = 0;
                    zr[k] = word_of(z, k);
                }
                dl = q - (L - 1);
                if (r.fresh) {
                    full = r.full;
                    dw = -1;
                    gst = W_RUN;
                }
            }
        }

        const bool any_run = __ballot(gst == W_RUN) != 0;
        if (!any_run && __ballot(gst == W_TB) == 0) {
            if (__ballot(!exhausted && pair < 0) == 0) break;
            if (__hip_atomic_load(&a.qctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (uint32_t)a.npairs) break;
            __builtin_amdgcn_s_sleep(16);
            continue;
        }

        // ---- 4. DC pass: one row of every running window per step ----
        int steps = 0;
        if (any_run) do {
            const bool computing = gst == W_RUN;
            const uint32_t tm = dl >= 0 ? 1u : 0u;    // the M term shifts in a 1 from the lane's first row on
            const uint32_t cin = dl >= 1 ? 1u : 0u;   // the I/S terms from its second row on
            uint32_t nb[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t v = from_upper_lane(A[k][0]);
                nb[k] = q == L - 1 ? zr[k] : v;
            }
            // I, S and D terms from row d-1: with S[t] = Z[t] >> 1 | cin they are
            // S[t] | S[t+1] | Z[t+1].  Ascending columns (each column still sees its
            // right neighbour's row d-1), S[t+1] carried to the next column; then the
            // M term from row d of the right neighbour, descending columns.  Both are
            // register-tied, four columns per statement: the compiler separates
            // consecutive statements that share registers by a wait state.
#define SCG_W1COL(T, X0, X1, X2, X3, S, N)                                          \
    "v_alignbit_b32 %[" N "0], %[" X1 "], %[" X0 "], 1\n\t"                         \
    "v_alignbit_b32 %[" N "1], %[" X2 "], %[" X1 "], 1\n\t"                         \
    "v_alignbit_b32 %[" N "2], %[" X3 "], %[" X2 "], 1\n\t"                         \
    "v_alignbit_b32 %[" N "3], %[cin], %[" X3 "], 1\n\t"                            \
    "v_or3_b32 %[a" #T "0], %[" S "0], %[" N "0], %[" X0 "]\n\t"                    \
    "v_or3_b32 %[a" #T "1], %[" S "1], %[" N "1], %[" X1 "]\n\t"                    \
    "v_or3_b32 %[a" #T "2], %[" S "2], %[" N "2], %[" X2 "]\n\t"                    \
    "v_or3_b32 %[a" #T "3], %[" S "3], %[" N "3], %[" X3 "]\n\t"
#define SCG_W2COL(T, N0, N1, N2, N3)                                                \
    "v_alignbit_b32 %[b3], %[tm], %[" N3 "], 1\n\t"                                 \
    "v_alignbit_b32 %[b2], %[" N3 "], %[" N2 "], 1\n\t"                             \
    "v_alignbit_b32 %[b1], %[" N2 "], %[" N1 "], 1\n\t"                             \
    "v_alignbit_b32 %[b0], %[" N1 "], %[" N0 "], 1\n\t"                             \
    "v_and_or_b32 %[a" #T "3], %[b3], %[e" #T "3], %[a" #T "3]\n\t"                 \
    "v_and_or_b32 %[a" #T "2], %[b2], %[e" #T "2], %[a" #T "2]\n\t"                 \
    "v_and_or_b32 %[a" #T "1], %[b1], %[e" #T "1], %[a" #T "1]\n\t"                 \
    "v_and_or_b32 %[a" #T "0], %[b0], %[e" #T "0], %[a" #T "0]\n\t"
#define SCG_WA(T, U) [a##T##0] "+v"(A[0][U]), [a##T##1] "+v"(A[1][U]), [a##T##2] "+v"(A[2][U]), [a##T##3] "+v"(A[3][U])
#define SCG_WE(T, U) [e##T##0] "v"(E[0][U]), [e##T##1] "v"(E[1][U]), [e##T##2] "v"(E[2][U]), [e##T##3] "v"(E[3][U])
            static_assert(CB % 4 == 0, "columns per lane come in fours");
            uint32_t s0, s1, s2, s3;   // S[t] of the next column to update
            asm volatile("v_alignbit_b32 %[s0], %[z1], %[z0], 1\n\t"
                         "v_alignbit_b32 %[s1], %[z2], %[z1], 1\n\t"
                         "v_alignbit_b32 %[s2], %[z3], %[z2], 1\n\t"
                         "v_alignbit_b32 %[s3], %[cin], %[z3], 1"
                         : [s0] "=&v"(s0), [s1] "=&v"(s1), [s2] "=&v"(s2), [s3] "=&v"(s3)
                         : [z0] "v"(A[0][0]), [z1] "v"(A[1][0]), [z2] "v"(A[2][0]), [z3] "v"(A[3][0]), [cin] "v"(cin));
#pragma unroll
            for (int t0 = 0; t0 < CB; t0 += 4) {
                const uint32_t x0 = t0 + 4 < CB ? A[0][t0 + 4] : nbs[0];
                const uint32_t x1 = t0 + 4 < CB ? A[1][t0 + 4] : nbs[1];
                const uint32_t x2 = t0 + 4 < CB ? A[2][t0 + 4] : nbs[2];
                const uint32_t x3 = t0 + 4 < CB ? A[3][t0 + 4] : nbs[3];
                uint32_t n0, n1, n2, n3;
                asm volatile(SCG_W1COL(0, "a10", "a11", "a12", "a13", "s", "n")
                             SCG_W1COL(1, "a20", "a21", "a22", "a23", "n", "s")
                             SCG_W1COL(2, "a30", "a31", "a32", "a33", "s", "n")
                             SCG_W1COL(3, "x0", "x1", "x2", "x3", "n", "s")
                             : SCG_WA(0, t0), SCG_WA(1, t0 + 1), SCG_WA(2, t0 + 2), SCG_WA(3, t0 + 3),
                               [s0] "+v"(s0), [s1] "+v"(s1), [s2] "+v"(s2), [s3] "+v"(s3),
                               [n0] "=&v"(n0), [n1] "=&v"(n1), [n2] "=&v"(n2), [n3] "=&v"(n3)
                             : [x0] "v"(x0), [x1] "v"(x1), [x2] "v"(x2), [x3] "v"(x3), [cin] "v"(cin));
            }
#pragma unroll
            for (int t0 = CB - 4; t0 >= 0; t0 -= 4) {
                const uint32_t y0 = t0 + 4 < CB ? A[0][t0 + 4] : nb[0];
                const uint32_t y1 = t0 + 4 < CB ? A[1][t0 + 4] : nb[1];
                const uint32_t y2 = t0 + 4 < CB ? A[2][t0 + 4] : nb[2];
                const uint32_t y3 = t0 + 4 < CB ? A[3][t0 + 4] : nb[3];
                uint32_t b0, b1, b2, b3;
                asm volatile(SCG_W2COL(3, "y0", "y1", "y2", "y3") SCG_W2COL(2, "a30", "a31", "a32", "a33")
                             SCG_W2COL(1, "a20", "a21", "a22", "a23") SCG_W2COL(0, "a10", "a11", "a12", "a13")
                             : SCG_WA(0, t0), SCG_WA(1, t0 + 1), SCG_WA(2, t0 + 2), SCG_WA(3, t0 + 3),
                               [b0] "=&v"(b0), [b1] "=&v"(b1), [b2] "=&v"(b2), [b3] "=&v"(b3)
                             : [y0] "v"(y0), [y1] "v"(y1), [y2] "v"(y2), [y3] "v"(y3), [tm] "v"(tm),
                               SCG_WE(0, t0), SCG_WE(1, t0 + 1), SCG_WE(2, t0 + 2), SCG_WE(3, t0 + 3));
            }
#undef SCG_WE
#undef SCG_WA
#undef SCG_W2COL
#undef SCG_W1COL
#pragma unroll
            for (int k = 0; k < 4; ++k) nbs[k] = nb[k];
            {   // initial column, one row further: z >> 1 with a 1 shifted in at the top
                const uint32_t z0 = __builtin_amdgcn_alignbit(zr[1], zr[0], 1);
                const uint32_t z1 = __builtin_amdgcn_alignbit(zr[2], zr[1], 1);
                const uint32_t z2 = __builtin_amdgcn_alignbit(zr[3], zr[2], 1);
                const uint32_t z3 = __builtin_amdgcn_alignbit(1u, zr[3], 1);
                zr[0] = z0; zr[1] = z1; zr[2] = z2; zr[3] = z3;
            }
            // keep the row for traceback
            if (computing && storer && dl >= 0 && dl < kRowsW) {
                uint4* row = reinterpret_cast<uint4*>(bdent + (qbyte + __umul24((uint32_t)dl, rowbytes)));
                if constexpr (SW == 2) {
                    uint2* const row2 = reinterpret_cast<uint2*>(row);
#pragma unroll
                    for (int t = 0; t < CB; ++t) row2[t] = uint2{A[0][t], A[1][t]};
                } else if constexpr (SW == 3) {
                    W3* const row3 = reinterpret_cast<W3*>(row);
#pragma unroll
                    for (int t = 0; t < CB; ++t) row3[t] = W3{A[0][t], A[1][t], A[2][t]};
                } else {
#pragma unroll
                    for (int t = 0; t < CB; ++t) row[t] = uint4{A[0][t], A[1][t], A[2][t], A[3][t]};
                }
            }
            // early termination: column 0 of row d has the msb of R clear
            const uint64_t hb = __ballot(slot && computing && dl >= 0 && (A[0][0] & 1u));
            {
                const int d0 = dl - q;   // row of column 0 computed at this step
                const bool hit = computing && (hb & gbit) != 0 && dw < 0;
                const bool done = hit || (computing && d0 >= full - 1);   // no hit in rows 0..k_w: dw stays -1
                dw = hit ? d0 : dw;
                gst = done ? W_DONE : gst;
            }
            dl += 1;
            steps += 1;
        } while (__ballot(gst == W_RUN) != 0);
        c_lane_steps += 64ull * (unsigned long long)steps;
        c_rounds += 1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

        // ---- 5. traceback of finished windows, advance, output ----
        if (slot && gst == W_DONE) {
            c_rows += (unsigned long long)(dw < 0 ? full : dw + 1);
            tb_d = dw;
            if (tb_d < 0 && kw == mw) tb_d = mw;   // no hit in rows 0..m_w-1: distance m_w
            // work in 64-bit ops: a 128-bit vector operation counts twice
            if (tb_d < 0) {
                c_windows += 1;
                c_ops += 2ull * ((unsigned long long)(kw + 1) + 2ull * nw + 7ull * nw * kw);
                a.edits[pair] = -1;
                a.text_end[pair] = -1;
                a.status[pair] = 1;
                a.n_runs[pair] = 0;
                pair = -1;
                atomicAdd(&a.qctl[2], 1u);
                gst = W_EMPTY;
            } else {
                c_windows += 1;
                c_ops += 2ull * ((unsigned long long)(tb_d + 1) + 2ull * nw + 7ull * nw * tb_d);
                tb_i = tb_j = tb_e = tb_bad = 0;
                tb_rc = z_init128(mw, tb_d - 1);
            }
        }
        if (gst == W_DONE) gst = W_TB;
        if (__ballot(slot && gst == W_TB) != 0) {
            const bool tracing = slot && gst == W_TB;
            const GroupRecW r = grec[g];
            const int jlim = min(mw, cap);
            const int ilim = min(nw, cap);              // a match run stops at the text window's end and at the cap
            uint32_t* const rout = a.runs + roff;       // the pair's run list (m + n + 1 >= 1 entries)
            const int rlast = (int)rcap - 1;
            // `fin` is an integer so that it lives in a vector register: a boolean
            // carried around a loop with a divergent body is kept as a lane mask
            // that the compiler re-merges with scalar operations at every event
            int fin = tracing ? 0 : 1;
            for (int ev = 0; ev < kTbEventsW; ++ev) {
                if (__ballot(fin == 0) == 0) break;
                if (fin == 0) {
                    // match run at (tb_i, tb_j); characters past n_w never match
                    const V128 ta = shr128(r.tlo, tb_i), tb = shr128(r.thi, tb_i);
                    const V128 pa = shr128(r.plo, tb_j), pb = shr128(r.phi, tb_j);
                    const V128 x{(ta.lo ^ pa.lo) | (tb.lo ^ pb.lo), (ta.hi ^ pa.hi) | (tb.hi ^ pb.hi)};
                    const int L0 = max(min(ctz128(x), min(ilim - tb_i, jlim - tb_j)), 0);
                    const int ti = tb_i + L0, tj = tb_j + L0, td = tb_d;
                    // edit step at (ti, tj, td): bits tj, tj+1 of row td-1 at columns ti and ti+1.
                    // The loads go out first; the run bookkeeping below overlaps them.
                    const uint32_t ro = gbyte + __umul24((uint32_t)(max(td, 1) - 1), rowbytes);
                    const char* const p0e = bdent + (ro + (uint32_t)min(ti, stride - 1) * ESZ);
                    const char* const p1e = bdent + (ro + (uint32_t)min(ti + 1, stride - 1) * ESZ);
                    uint4 e0, e1;
                    if constexpr (SW == 2) {
                        const uint2 a0 = *reinterpret_cast<const uint2*>(p0e), a1 = *reinterpret_cast<const uint2*>(p1e);
                        e0 = uint4{a0.x, a0.y, 0u, 0u};
                        e1 = uint4{a1.x, a1.y, 0u, 0u};
                    } else if constexpr (SW == 3) {
                        const W3 a0 = *reinterpret_cast<const W3*>(p0e), a1 = *reinterpret_cast<const W3*>(p1e);
                        e0 = uint4{a0.x, a0.y, a0.z, 0u};
                        e1 = uint4{a1.x, a1.y, a1.z, 0u};
                    } else {
                        e0 = *reinterpret_cast<const uint4*>(p0e);
                        e1 = *reinterpret_cast<const uint4*>(p1e);
                    }
                    // the run list always holds the open run at index nruns, so
                    // extending or starting a run is one unconditional store
                    {
                        const bool same = cur_op == 0;
                        nruns += (!same && cur_len > 0 && L0 > 0) ? 1 : 0;
                        cur_len = L0 == 0 ? cur_len : (same ? cur_len + L0 : L0);
                        cur_op = L0 == 0 ? cur_op : 0;
                        rout[min(nruns, rlast)] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                    }
                    const bool edit = !(tj >= jlim || ti >= cap);
                    const V128 v0{(uint64_t)e0.x | ((uint64_t)e0.y << 32), (uint64_t)e0.z | ((uint64_t)e0.w << 32)};
                    const V128 v1{(uint64_t)e1.x | ((uint64_t)e1.y << 32), (uint64_t)e1.z | ((uint64_t)e1.w << 32)};
                    const V128 za = ti < nw ? v0 : tb_rc;        // Z[ti][td-1]
                    const V128 zb = ti + 1 < nw ? v1 : tb_rc;    // Z[ti+1][td-1]
                    const int has_t = ti < nw;
                    const int sb = has_t & zbit128(zb, tj + 1);
                    const int ib = zbit128(za, tj + 1);
                    const int db = has_t & zbit128(zb, tj);
                    const int op = sb ? 1 : (ib ? 2 : 3);
                    tb_bad |= edit & ((td <= 0) | !(sb | ib | db));
                    tb_i = ti + (edit && op != 2 ? 1 : 0);
                    tb_j = tj + (edit && op != 3 ? 1 : 0);
                    tb_d = td - (edit ? 1 : 0);
                    tb_e += edit ? 1 : 0;
                    if (edit) tb_rc = V128{tb_rc.lo << 1, (tb_rc.hi << 1) | (tb_rc.lo >> 63)};   // m_w - d grows by one
                    {
                        const bool same = cur_op == op;
                        nruns += (edit && !same && cur_len > 0) ? 1 : 0;
                        cur_len = !edit ? cur_len : (same ? cur_len + 1 : 1);
                        cur_op = !edit ? cur_op : op;
                        rout[min(nruns, rlast)] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                    }
                    fin = (!edit || tb_j >= jlim || tb_i >= cap || tb_bad) ? 1 : 0;
                }
            }
            if (tracing && fin) {
                edits += tb_e;
                p0 += tb_j;
                t0 += tb_i;
                gst = W_EMPTY;
                if (tb_bad || p0 >= m) {
                    nruns += cur_len > 0 ? 1 : 0;   // the open run is already in the list
                    const bool ok = !tb_bad && nruns <= rcap;
                    if (!ok) c_err += 1;
                    a.edits[pair] = ok ? edits : -1;
                    a.text_end[pair] = ok ? t0 : -1;
                    a.status[pair] = ok ? 0 : 3;
                    a.n_runs[pair] = ok ? nruns : 0;
                    pair = -1;
                    atomicAdd(&a.qctl[2], 1u);
                }
            }
        }
        {   // the group's lanes learn that its traceback ended
            const uint64_t tbm = __ballot(slot && gst == W_TB);
            if ((tbm & gbit) == 0 && gst == W_TB) gst = W_EMPTY;
        }
        // traceback's reads of the stored rows finish before the next pass overwrites them
        __syncthreads();
    }

    // ---- counters ----
    if (slot) {
        if (c_windows) atomicAdd(&a.stats[ST_WINDOWS], c_windows);
        if (c_ops) atomicAdd(&a.stats[ST_OPS_ALG], c_ops);
        if (c_rows) atomicAdd(&a.stats[ST_ROWS], c_rows);
        if (c_err) atomicAdd(&a.stats[ST_ERRORS], c_err);
    }
    if (lane == 0) {
        atomicAdd(&a.stats[ST_LANE_STEPS], c_lane_steps);
        atomicAdd(&a.stats[ST_ROUNDS], c_rounds);
    }
}

}  // namespace

int wide_dent_stride(int cap, int ng) {
    const int cb = 2 * ng;                            // columns per lane
    const int cols = cap + 1 < 128 ? cap + 1 : 128;   // stored columns 0..min(cap, 127)
    return (cols + cb - 1) / cb * cb;
}

size_t wide_dent_bytes(int grid, int cap, int ng) {
    return (size_t)grid * ng * kRowsW * (size_t)wide_dent_stride(cap, ng) * 16u;
}

// words kept per stored entry for W - O = cap
static int wide_words(int cap) { return cap <= 63 ? 2 : (cap <= 95 ? 3 : 4); }

static const void* wide_fn(int ng, int sw) {
    if (sw == 2) return ng == 8 ? (const void*)wide_kernel<8, 2> : (const void*)wide_kernel<4, 2>;
    if (sw == 3) return ng == 8 ? (const void*)wide_kernel<8, 3> : (const void*)wide_kernel<4, 3>;
    return ng == 8 ? (const void*)wide_kernel<8, 4> : (const void*)wide_kernel<4, 4>;
}

int wide_max_blocks_per_cu(int ng, int cap) {
    int nb = 0;
    const void* f = wide_fn(ng, wide_words(cap));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64, 0) != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_align_wide(const AlignArgs& a, int grid, int ng, hipStream_t s) {
    const int sw = wide_words(a.cap);
#define SCG_WIDE_LAUNCH(NGV, SWV) hipLaunchKernelGGL((wide_kernel<NGV, SWV>), dim3(grid), dim3(64), 0, s, a)
    if (ng == 8) {
        if (sw == 2) SCG_WIDE_LAUNCH(8, 2);
        else if (sw == 3) SCG_WIDE_LAUNCH(8, 3);
        else SCG_WIDE_LAUNCH(8, 4);
    } else {
        if (sw == 2) SCG_WIDE_LAUNCH(4, 2);
        else if (sw == 3) SCG_WIDE_LAUNCH(4, 3);
        else SCG_WIDE_LAUNCH(4, 4);
    }
#undef SCG_WIDE_LAUNCH
    return hipGetLastError();
}
