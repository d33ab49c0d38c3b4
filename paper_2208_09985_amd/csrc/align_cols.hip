// Fused, persistent windowed GenASM-DC + GenASM-TB kernel for gfx950,
// column-block mapping.
//
// Mapping (one wavefront = one workgroup, 64 lanes):
//   * A wavefront holds NG windows of NG different pairs (NG = 4, 8 or 16;
//     also 32 without a learned budget), one per group of L = 64/NG
//     consecutive lanes.  Lane q of a group owns
//     the CB = NG text columns CB*q .. CB*q+CB-1 of its window and keeps, for
//     each of them, the bitvector of the current error row and the column's
//     pattern-match mask (two VGPRs each).  Fewer windows per wavefront give
//     more wavefronts for the same number of pairs, at the price of a longer
//     skew (L-1 steps per window).
//   * The group computes the rows d = 0, 1, 2, ... of Algorithm 1 one after
//     the other (Section 2.2.1).  Inside a row the dependence runs from the
//     text end toward column 0, so the L lanes are skewed by one step: lane q
//     computes row d at step d + L-1 - q.  The value a lane needs from the
//     columns to its right (row d and row d-1 of column CB*q+CB) arrives from
//     lane q+1 through one DPP wave_shl:1 per 32-bit half; lane L-1 takes the
//     window's initial column (Section 2.2.1) instead.  Text columns at
//     or beyond n_w carry the initial column too, because their match mask is
//     empty, so windows shorter than 64 need no special case.
//   * Bitvectors are kept as the complement Z = ~R in LSB-first order (bit j =
//     pattern position j); the update of Algorithm 1 becomes
//         Z[i][d] = (Z[i][d-1] >> 1 | top) | (Z[i+1][d-1] >> 1 | top) | Z[i+1][d-1]
//                 | ((Z[i+1][d] >> 1 | top) & EQ[text[i]])
//     where the shifted row d-1 of a column serves that column and its left
//     neighbour: eight 32-bit operations per entry.  Before a lane's first
//     row its inputs are zero and both shifted-in bits are off, so ramp steps
//     leave it zero.
//   * Early termination (Section 2.4.3): lane 0 of a group holds column 0;
//     the first row whose entry has the msb of R clear is d_w, found by one
//     ballot per step; the group state is updated once per two steps.  A
//     wavefront's DC pass ends when no group is still computing.
//   * Stored entries (Section 2.4.1, entries not edges; Section 2.4.2, only
//     columns 0..W-O are read by traceback) go to a per-group region of
//     global memory, [row][column] with a row stride that is a multiple of
//     CB; each storing lane writes its CB columns with 16-byte stores.  When
//     W-O <= 31 traceback reads bits 0..W-O only, so plain mode stores
//     entries as their low 32 bits (NARROW; Section 2.4.2's narrower stored
//     bitvectors); when W-O <= 47 it stores their low 48 bits as a 32-bit
//     plane and a 16-bit plane (SPLIT), three quarters of the footprint.
//   * Traceback runs in lane 0 of every finished group, all groups of the
//     wavefront together: match runs are skipped with an XOR of the 2-bit
//     planes and a trailing-zero count, and each edit step reads row d-1 at
//     columns i and i+1.  An event (match run, edit step) is one basic
//     block, and the run list keeps the open run in place so that every
//     update is one store.
//   * Row budgets: a pass ends when every window it waits for has found
//     d_w.  Plain mode waits for every window (rows 0..k_w at most).  Fixed
//     mode waits for a window up to fixed_rows rows, learned mode up to the
//     predicted budget (and not at all for a window predicted to need more
//     than 16 rows).  A window over its budget keeps computing in its lanes,
//     with all rows, through the following passes, and is traced back when
//     its d_w is found; rows <= d never depend on rows > d, so the result is
//     bit-identical.
//   * Pairs are taken from the global queue shared with the row-lane kernel;
//     a pair that has advanced yield_chars pattern characters saves its
//     state and goes back to the queue between windows.
#include "colblock.h"
#include "predictor.h"

namespace {

using namespace colblock;

constexpr int kStoredRows = 64;    // rows 0..63 are kept for traceback

// A group is RUN while the pass waits for it, OVER once it has used its row
// budget without finding d_w (it keeps computing, but the pass no longer
// waits for it), DONE when d_w is known (or no row up to k_w has it), TB
// while its traceback runs (possibly over several rounds).
enum : int { G_EMPTY = 0, G_RUN = 1, G_DONE = 2, G_OVER = 3, G_TB = 4 };
constexpr int kTbEvents = 40;      // traceback events (match run + edit step) per round
constexpr int kWaitRows = 16;      // learned mode: largest predicted budget a pass waits for
enum : int { CMD_NONE = 0, CMD_FRESH = 1, CMD_RESUME = 2 };

struct GroupRec {      // LDS: what the slot lane tells its group at set-up
    uint64_t plo, phi, tlo, thi;   // window planes (pattern at p0, text at t0)
    int32_t m_w, n_w;
    int32_t limit;     // rows 0..limit-1 of column 0 may be computed this pass
    int32_t full;      // rows of the whole window
    int32_t cmd;
    int32_t pad;
};

// ST: the stored entries.  0: whole 64-bit entries.  1 (NARROW): their low 32
// bits, when traceback reads bits 0..31 at most.  2 (SPLIT): their low 48 bits
// as a 32-bit plane and a 16-bit plane, when it reads bits 0..47 at most.
// SM: where the stored rows go.  0: rows 0..63 in the global region.  1: the
// lowest lds_rows rows in LDS, the others global.  2 (DENT extended to rows,
// supplementary Section 1): a ring of ring_rows slots in the global region,
// row d in slot d mod ring_rows.
// OW: the wavefront reserves a whole SIMD.  Each pair's windows form a serial
// chain, so the kernel's time is the time of its slowest wavefront, and a
// wavefront that shares its SIMD with another runs its chain up to 1.5x
// slower; the dispatcher does place two on one SIMD while others stay empty.
// Claiming every accumulation register (this kernel issues no MFMA) makes a
// wavefront's register block the whole of a SIMD's, so the hardware places at
// most one per SIMD.  Used when the batch needs no more wavefronts than SIMDs.
template <bool LEARNED, int NG, int ST, int SM, bool OW = false>
__global__ __launch_bounds__(64) void cols_kernel(const AlignArgs a) {
    constexpr bool LR = SM == 1, RING = SM == 2;
    if constexpr (OW) asm volatile("" ::: "a255");
    constexpr bool NARROW = ST == 1, SPLIT = ST == 2;
    // ST 3 (EDGES, the ablation of storing entries instead of edges): every
    // stored slot holds the three edge bitvectors of Algorithm 1 that the
    // traceback tests (I, S and D of the row above, from this row) and the
    // M edge of this row, four 64-bit words, 32 bytes per entry
    constexpr bool EDGES = ST == 3;
    constexpr uint32_t EW = EDGES ? 4u : 1u;   // 8-byte words per stored entry
    constexpr int L = 64 / NG;             // lanes per window
    constexpr int CB = cols_per_lane(NG);  // text columns per lane (CB * L >= 64)
    // NG * L < 64 (10 windows of 6 lanes): the lanes past the last group hold
    // no window; they read an always-empty record and never take a pair
    __shared__ GroupRec grec[NG + 1];
    const int lane = threadIdx.x;
    const int g = lane / L, q = lane % L;
    const bool live = g < NG;
    const bool slot = live && q == 0;
    const uint64_t gbit = 1ull << (lane - q);   // the group's slot lane in a ballot
    const int cap = a.cap;
    const int stride = a.dstride;
    // The block's stored rows start at a wavefront-uniform address; a lane reaches
    // its group's entries with a 32-bit byte offset (a group holds 64 rows of
    // `stride` entries of at most 8 bytes).
    constexpr uint32_t ESZ = NARROW ? 4u : 8u * EW;   // bytes per stored entry
    // rows per group in the global region: 64, or the ring's slots
    const int NR = RING ? a.ring_rows : kStoredRows;
    const uint32_t NRu = (uint32_t)NR;
    char* const bdent = reinterpret_cast<char*>(a.dent + (size_t)blockIdx.x * NG * (size_t)(NR * stride) * EW);
    const uint32_t gbyte = (uint32_t)(g * NR * stride) * 8u * EW;
    // the slot of stored row r (a ring when RING: rows of one window never need
    // more than ring_rows consecutive slots)
    auto slot_of = [&](uint32_t r) -> uint32_t {
        if (!RING) return r;
        uint32_t sl = r >= NRu ? r - NRu : r;
        return sl >= NRu ? r % NRu : sl;
    };
    const uint32_t qbyte = gbyte + (uint32_t)(CB * q) * ESZ;   // the lane's first column in row 0
    const uint32_t rowbytes = (uint32_t)stride * ESZ;
    // SPLIT: rows of the 32-bit plane (stride*4 bytes) for rows 0..63, then rows
    // of the 16-bit plane (stride*2 bytes)
    const uint32_t lobytes = (uint32_t)stride * 4u, hibytes = (uint32_t)stride * 2u;
    const uint32_t hiplane = gbyte + NRu * lobytes;
    const bool storer = CB * q < stride;
    // Rows 0..R-1 of every group's stored region live in LDS (dynamic shared
    // memory, R chosen by the host from the occupancy the batch needs): the
    // same layout as the global region with R rows per group.  Rows R..63 stay
    // in the global region.
    extern __shared__ __align__(16) char lrows[];
    const int R = LR ? a.lds_rows : 0;
    const uint32_t lrowb = SPLIT ? (uint32_t)stride * 6u : rowbytes;   // bytes of one stored row
    const uint32_t lgbyte = (uint32_t)(live ? g : 0) * (uint32_t)R * lrowb;
    const uint32_t lhiplane = lgbyte + (uint32_t)R * lobytes;

    if (lane <= NG) grec[lane] = GroupRec{0, 0, 0, 0, 0, 0, 0, 0, CMD_NONE, 0};

    // ---- slot-lane state (lanes with q == 0) ----
    int pair = -1, p0 = 0, t0 = 0, m = 0, n = 0, edits = 0, nruns = 0, cur_op = 0, cur_len = 0, p0_take = 0;
    int mw = 0, nw = 0, kw = 0;
    int64_t roff = 0, rcap = 0, pending = -1;
    int polled = 0;
    int deep_run = 0;   // slot lane: consecutive windows of the pair with d_w >= mig_d
    // slot lane, one-per-SIMD form: planes words cpq..cpq+2 of the pair's pattern and
    // ctq..ctq+2 of its text (pair cpair)
    Plane2 cpw0{0, 0}, cpw1{0, 0}, cpw2{0, 0}, ctw0{0, 0}, ctw1{0, 0}, ctw2{0, 0};
    int cpair = -1, cpq = 0, ctq = 0;
    const Plane2* cpb = a.pplanes;
    const Plane2* ctb = a.tplanes;
    bool exhausted = !slot;
    // the queue this launch takes pairs from: the main ring, or (helper) hring
    uint32_t* const qhead = a.helper ? &a.qctl[kQcHHead] : &a.qctl[0];
    const int32_t* const qring = a.helper ? a.hring : a.ring;
    const int64_t qcapv = a.helper ? (int64_t)a.npairs : a.qcap;
    uint32_t idle = 0, beat = 0;
    unsigned long long c_windows = 0, c_ops = 0, c_fallback = 0, c_rows = 0, c_err = 0, c_yield = 0;
    int tb_i = 0, tb_j = 0, tb_d = 0, tb_e = 0, tb_bad = 0;   // slot lane: traceback position and edits
    uint64_t tb_rc = 0;   // slot lane: the initial column at row tb_d - 1 (Z beyond the text window)

    unsigned long long c_lane_steps = 0, c_rounds = 0;

    // ---- lane state: current row of the lane's 16 columns, their match masks ----
    RowRegs<CB> A, E;
    for (int t = 0; t < CB; ++t) A.lo[t] = A.hi[t] = E.lo[t] = E.hi[t] = 0;
    uint32_t nbslo = 0, nbshi = 0;     // row d-1 of column CB*q+CB
    uint32_t zrlo = 0, zrhi = 0;       // initial column at the lane's next row (used by q == L-1)
    int dl = 0;                        // row this lane computes at the next step
    int gst = G_EMPTY;                 // group state, identical in the group's L lanes
    int limit = 0, full = 0, dw = -1;
    uint32_t over_events = 0;

    for (;;) {
        // ---- 1. slot lanes take pairs from the queue ----
        if (!exhausted && pair < 0) {
            if (pending < 0) pending = (int64_t)atomicAdd(qhead, 1u);
            if (pending >= qcapv) {
                exhausted = true;
            } else {
                polled = __hip_atomic_load(&qring[pending], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (polled != 0) {
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    const bool fresh = !a.helper && pending < a.npairs;   // hring holds handed-over pairs only
                    const int pid = polled - 1;
                    pending = -1;
                    polled = 0;
                    const int pm = a.plen[pid], pn = a.tlen[pid];
                    // (a helper sees such pairs only among the long pairs it holds from the start)
                    if ((fresh || a.helper) && (a.bad[pid] || pm == 0)) {
                        const bool bad = a.bad[pid] != 0;
                        a.edits[pid] = bad ? -1 : 0;
                        a.text_end[pid] = bad ? -1 : 0;
                        a.status[pid] = bad ? 2 : 0;
                        a.n_runs[pid] = 0;
                        atomicAdd(&a.qctl[2], 1u);
                        if (a.helper) atomicSub(&a.qctl[kQcHInFlight], 1u);
                    } else {
                        pair = pid;
                        m = pm;
                        n = pn;
                        if (fresh) {
                            p0 = 0; t0 = 0; edits = 0; nruns = 0; cur_op = 0; cur_len = 0;
                        } else {
                            const int32_t* st = a.pstate + 8 * (int64_t)pid;
                            p0 = st[0]; t0 = st[1]; edits = st[2]; nruns = st[3]; cur_op = st[4]; cur_len = st[5];
                        }
                        p0_take = p0;
                        deep_run = 0;
                        roff = a.runs_off[pid];
                        rcap = a.runs_off[pid + 1] - roff;
                    }
                }
            }
        }

        // ---- 2. slot lanes start windows (or resume paused ones) ----
        if (slot) {
            GroupRec& r = grec[g];
            if (gst == G_EMPTY && pair >= 0) {
                mw = min(a.W, m - p0);
                nw = min(a.W, n - t0);
                kw = min(a.k, mw);
                const int rows_full = (kw == mw) ? mw : kw + 1;   // row m_w is implicit: D(0,0) <= m_w
                uint64_t plo, phi, tlo = 0, thi = 0;
                if constexpr (OW) {
                    // the slot keeps planes words q and q+1 of both sequences from the window's
                    // start q, and word q+2, loaded a whole pass before it is read: the next
                    // window starts at most 63 characters further, in word q or q+1 (a reload
                    // only for a new or moved pair).  One load site per sequence, so that the
                    // loaded registers are the kept ones and nothing waits for them here
                    const int pq = p0 >> 6, tq = t0 >> 6;
                    const int plast = (m + 63) >> 6, tlast = (n + 63) >> 6;   // the sequence's last (padding) word
                    if (pair != cpair || pq < cpq || pq > cpq + 1 || tq < ctq || tq > ctq + 1) {
                        cpb = a.pplanes + a.pword[pair];
                        ctb = a.tplanes + a.tword[pair];
                        cpair = pair;
                        cpq = pq;
                        ctq = tq;
                        cpw0 = cpb[pq];
                        cpw1 = cpb[pq + 1];
                        ctw0 = ctb[min(tq, tlast)];
                        ctw1 = ctb[min(tq + 1, tlast)];
                    } else {
                        if (pq == cpq + 1) {
                            cpw0 = cpw1;
                            cpw1 = cpw2;
                            cpq = pq;
                        }
                        if (tq == ctq + 1) {
                            ctw0 = ctw1;
                            ctw1 = ctw2;
                            ctq = tq;
                        }
                    }
                    cpw2 = cpb[min(cpq + 2, plast)];
                    ctw2 = ctb[min(ctq + 2, tlast)];
                    const uint32_t pr = (uint32_t)(p0 & 63), tr = (uint32_t)(t0 & 63);
                    plo = pr ? (cpw0.lo >> pr) | (cpw1.lo << (64u - pr)) : cpw0.lo;
                    phi = pr ? (cpw0.hi >> pr) | (cpw1.hi << (64u - pr)) : cpw0.hi;
                    if (nw > 0) {
                        tlo = tr ? (ctw0.lo >> tr) | (ctw1.lo << (64u - tr)) : ctw0.lo;
                        thi = tr ? (ctw0.hi >> tr) | (ctw1.hi << (64u - tr)) : ctw0.hi;
                    }
                } else {
                    load_window(a.pplanes + a.pword[pair], p0, plo, phi);
                    if (nw > 0) load_window(a.tplanes + a.tword[pair], t0, tlo, thi);
                }
                r.plo = plo;
                r.phi = phi;
                r.tlo = tlo;
                r.thi = thi;
                r.m_w = mw;
                r.n_w = nw;
                r.full = rows_full;
                r.limit = a.mode == 2 ? min(a.fixed_rows, rows_full) : rows_full;
                r.cmd = CMD_FRESH;
            } else {
                r.cmd = CMD_NONE;
            }
        }
        __syncthreads();

        // ---- 3. learned row budget of fresh windows: features -> MLP (MFMA) ----
        if constexpr (LEARNED) {
            MlpRegs mlp;
            mlp_load_packed(mlp, a.model.operands, lane);
            const int s = lane & 15, fg = lane >> 4;
            const GroupRec rs = grec[s < NG ? s : 0];
            const WinPlanes o{rs.plo, rs.phi, rs.tlo, rs.thi, rs.m_w, rs.n_w};
            half4_t x4;
            for (int e = 0; e < 4; ++e) x4[e] = feature_to_input(window_feature(o, 4 * fg + e));
            half4_t hid[4];
            const float4_t logit = mlp_tile_forward(mlp, x4, hid);
            __syncthreads();
            if (lane < NG && rs.cmd == CMD_FRESH) {
                // lane s < 16 holds classes 0..3 of group s
                const int C = a.model.C;
                float mx = logit[0];
                for (int c = 1; c < C; ++c) mx = fmaxf(mx, logit[c]);
                float p[4], tot = 0.f;
                for (int c = 0; c < C; ++c) {
                    p[c] = __expf(logit[c] - mx);
                    tot += p[c];
                }
                int cls = C - 1;
                float cum = 0.f;
                for (int c = 0; c < C; ++c) {
                    cum += p[c];
                    if (cum >= a.model.tau * tot) {
                        cls = c;
                        break;
                    }
                }
                // the pass waits for a window only up to its predicted budget, and
                // not at all for one predicted to need many rows
                const int br = a.model.budget_rows[cls];
                grec[lane].limit = br <= kWaitRows ? max(1, min(br, rs.full)) : 1;
            }
            __syncthreads();
        }

        // ---- 4. every lane applies its group's command ----
        {
            const GroupRec r = grec[g];
            if (r.cmd == CMD_FRESH) {
                const uint64_t beyond = r.m_w >= 64 ? 0ull : (~0ull << r.m_w);
                const uint32_t tql = CB * q < 64 ? (uint32_t)(r.tlo >> (CB * q)) : 0u;
                const uint32_t tqh = CB * q < 64 ? (uint32_t)(r.thi >> (CB * q)) : 0u;
                const int ncols = min(max(r.n_w - CB * q, 0), CB);   // this lane's columns inside the text window
                // match mask of column t: the pattern positions whose base equals text base t,
                // i.e. whose bits in both planes equal the text base's.  With m_lo and m_hi all
                // ones where the text base's low or high plane bit is set (a one-bit field,
                // sign-extended), that is ~((p_lo ^ m_lo) | (p_hi ^ m_hi)) on each 32-bit half;
                // zero past the text window's end, and set beyond m_w
                const uint32_t vmask = ncols >= 32 ? ~0u : (1u << ncols) - 1u;   // ncols <= CB <= 32
                const uint32_t pl0 = (uint32_t)r.plo, pl1 = (uint32_t)(r.plo >> 32);
                const uint32_t ph0 = (uint32_t)r.phi, ph1 = (uint32_t)(r.phi >> 32);
                const uint32_t by0 = (uint32_t)beyond, by1 = (uint32_t)(beyond >> 32);
#pragma unroll
                for (int t = 0; t < CB; ++t) {
                    const uint32_t ml = (uint32_t)__builtin_amdgcn_sbfe((int)tql, (uint32_t)t, 1u);
                    const uint32_t mh = (uint32_t)__builtin_amdgcn_sbfe((int)tqh, (uint32_t)t, 1u);
                    const uint32_t vm = (uint32_t)__builtin_amdgcn_sbfe((int)vmask, (uint32_t)t, 1u);
                    E.lo[t] = (~((pl0 ^ ml) | (ph0 ^ mh)) & vm) | by0;
                    E.hi[t] = (~((pl1 ^ ml) | (ph1 ^ mh)) & vm) | by1;
                    A.lo[t] = 0;
                    A.hi[t] = 0;
                }
                nbslo = nbshi = 0;
                const uint64_t zr = z_init(r.m_w, 0);
                zrlo = (uint32_t)zr;
                zrhi = (uint32_t)(zr >> 32);
                dl = q - (L - 1);
                limit = r.limit;
                full = r.full;
                dw = -1;
                gst = G_RUN;
            }
        }
        // with no window to wait for, wait for the ones over budget
        if (__ballot(gst == G_RUN) == 0 && gst == G_OVER) gst = G_RUN;

        const bool any_run = __ballot(gst == G_RUN) != 0;
        if (!any_run && __ballot(gst == G_TB) == 0) {
            // nothing to compute: leave once every pair is finished or no slot
            // can ever receive one; otherwise wait for yielded pairs
            const bool waiting = !exhausted && pair < 0;
            if (__ballot(waiting) == 0) break;
            if (a.helper) {
                // a helper waits for handed-over pairs while the main launch runs: its
                // slots poll their own hring entries; the shared counters are read once
                // every 16 sleeps.  After idle_limit such reads in which the main launch
                // showed no beat (it has not started, or has ended) the helper closes the
                // hand-over gate, so no pair can be handed over later, and leaves once
                // every pair handed over before that is finished (until then a slot
                // that holds a reserved hring entry may still receive one)
                idle += 1u;
                if ((idle & 15u) != 0u) {
                    __builtin_amdgcn_s_sleep(32);
                    continue;
                }
                if (__hip_atomic_load(&a.qctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (uint32_t)a.npairs)
                    break;
                const uint32_t b = __hip_atomic_load(&a.qctl[kQcBeat], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (b != beat) {
                    beat = b;
                    idle = 0u;
                } else if ((idle >> 4) > (uint32_t)a.idle_limit) {
                    uint32_t v = 0u;
                    if (lane == 0) v = atomicOr(&a.qctl[kQcHInFlight], kQcGateClosed);
                    v = __builtin_amdgcn_readfirstlane(v);
                    if ((v & ~kQcGateClosed) == 0u) break;
                }
                __builtin_amdgcn_s_sleep(32);
                continue;
            }
            if (__hip_atomic_load(&a.qctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (uint32_t)a.npairs) break;
            __builtin_amdgcn_s_sleep(16);
            continue;
        }

        // ---- 5. DC pass: one row of every running window per step ----
        int steps = 0;
        // the lane's row at which column 0 reaches the window's last row / its budget
        const int dstop = full - 1 + q, dover = limit - 1 + q;
        const int et = a.no_et ? 0 : 1;
        uint32_t soff = qbyte + (uint32_t)dl * rowbytes;   // byte offset of the lane's row dl (used once dl >= 0)
        if (any_run) do {
            // Two steps per iteration, the state update once per two: every lane
            // computes; only lanes of running windows store and count.  A window
            // that ends at the first step computes one row more, which nothing reads.
            const int computing = gst & 1;   // G_RUN or G_OVER
            uint64_t hb[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int dh = dl + h;                    // the row this lane computes at this step
                const uint32_t tm = dh >= 0 ? 1u : 0u;    // the M term shifts in a 1 from the lane's first row on
                const uint32_t cin = dh >= 1 ? 1u : 0u;   // the I/S terms from its second row on
                uint32_t nlo = from_upper_lane(A.lo[0]);
                uint32_t nhi = from_upper_lane(A.hi[0]);
                if (q == L - 1) {
                    nlo = zrlo;
                    nhi = zrhi;
                }
                dc_row(A, E, nlo, nhi, nbslo, nbshi, tm, cin);
                nbslo = nlo;
                nbshi = nhi;
                {   // initial column, one row further
                    const uint32_t zl = __builtin_amdgcn_alignbit(zrhi, zrlo, 1);
                    const uint32_t zh = __builtin_amdgcn_alignbit(1u, zrhi, 1);
                    zrlo = zl;
                    zrhi = zh;
                }
                // keep the row for traceback: rows below lds_rows in LDS, the others in
                // the global region (same layout, other base and row count)
                if (computing && storer && (uint32_t)dh < (uint32_t)kStoredRows) {
                    auto put = [&](char* const base, uint32_t lo_off, uint32_t hi_off) {
                        if (NARROW) {
                            uint4* row = reinterpret_cast<uint4*>(base + lo_off);
#pragma unroll
                            for (int t = 0; t < CB; t += 4) row[t >> 2] = uint4{A.lo[t], A.lo[t + 1], A.lo[t + 2], A.lo[t + 3]};
                        } else if (SPLIT) {
                            // low words as they are; bits 32..47 two columns to a word
                            uint4* lo = reinterpret_cast<uint4*>(base + lo_off);
#pragma unroll
                            for (int t = 0; t < CB; t += 4) lo[t >> 2] = uint4{A.lo[t], A.lo[t + 1], A.lo[t + 2], A.lo[t + 3]};
                            char* const hp = base + hi_off;
                            uint32_t hw[CB / 2];
#pragma unroll
                            for (int t = 0; t < CB; t += 2) hw[t >> 1] = __builtin_amdgcn_perm(A.hi[t + 1], A.hi[t], 0x05040100u);
                            if constexpr (CB % 8 != 0) {
                                // 8-byte stores: a lane's high words start on an 8-byte boundary
#pragma unroll
                                for (int t = 0; t < CB / 2; t += 2) reinterpret_cast<uint2*>(hp)[t >> 1] = uint2{hw[t], hw[t + 1]};
                            } else {
#pragma unroll
                                for (int t = 0; t < CB / 2; t += 4)
                                    reinterpret_cast<uint4*>(hp)[t >> 2] = uint4{hw[t], hw[t + 1], hw[t + 2], hw[t + 3]};
                            }
                        } else if (EDGES) {
                            // slot d: I, S, D of row d+1 (from row d) and M of row d, per column
                            uint4* row = reinterpret_cast<uint4*>(base + lo_off);
#pragma unroll
                            for (int t = 0; t < CB; ++t) {
                                const uint32_t xl = t + 1 < CB ? A.lo[t + 1] : nlo;   // row d of the next column
                                const uint32_t xh = t + 1 < CB ? A.hi[t + 1] : nhi;
                                const uint32_t il = __builtin_amdgcn_alignbit(A.hi[t], A.lo[t], 1);
                                const uint32_t ih = __builtin_amdgcn_alignbit(1u, A.hi[t], 1);
                                const uint32_t sl = __builtin_amdgcn_alignbit(xh, xl, 1);
                                const uint32_t sh = __builtin_amdgcn_alignbit(1u, xh, 1);
                                const uint32_t ml = sl & E.lo[t];
                                const uint32_t mh = __builtin_amdgcn_alignbit(tm, xh, 1) & E.hi[t];
                                row[2 * t] = uint4{il, ih, sl, sh};
                                row[2 * t + 1] = uint4{xl, xh, ml, mh};
                            }
                        } else {
                            uint4* row = reinterpret_cast<uint4*>(base + lo_off);
#pragma unroll
                            for (int t = 0; t < CB; t += 2) row[t >> 1] = uint4{A.lo[t], A.hi[t], A.lo[t + 1], A.hi[t + 1]};
                        }
                    };
                    const uint32_t udh = (uint32_t)dh;
                    if (LR && R >= kStoredRows) {
                        // every stored row in LDS (a wavefront-uniform test, so no divergent branch)
                        put(lrows, lgbyte + udh * (SPLIT ? lobytes : rowbytes) + (uint32_t)(CB * q) * (SPLIT ? 4u : ESZ),
                            lhiplane + udh * hibytes + (uint32_t)(CB * q) * 2u);
                    } else if (LR && udh < (uint32_t)R) {
                        put(lrows, lgbyte + udh * (SPLIT ? lobytes : rowbytes) + (uint32_t)(CB * q) * (SPLIT ? 4u : ESZ),
                            lhiplane + udh * hibytes + (uint32_t)(CB * q) * 2u);
                    } else {
                        const uint32_t sl = slot_of(udh);
                        put(bdent,
                            SPLIT ? gbyte + __umul24(sl, lobytes) + (uint32_t)(CB * q) * 4u
                                  : (RING ? qbyte + __umul24(sl, rowbytes) : soff + (h ? rowbytes : 0u)),
                            hiplane + __umul24(sl, hibytes) + (uint32_t)(CB * q) * 2u);
                    }
                }
                // early termination: column 0 of row d has the msb of R clear.  Lane 0 of
                // a group holds column 0; a lane's rows stay zero until its first row, so
                // the ballot needs no row test, and each lane reads its slot lane's bit.
                hb[h] = __ballot(A.lo[0] & 1u);
            }
            {   // state update without branches, for rows dl - q and dl + 1 - q of column 0
                const int b0 = (int)(hb[0] >> (lane - q)) & 1;
                const int b1 = (int)(hb[1] >> (lane - q)) & 1;
                const int fresh = computing & (dw < 0 ? 1 : 0);
                const int hit0 = fresh & b0;                                        // first row with a hit
                const int hit1 = fresh & (b0 ^ 1) & b1 & (dl + 1 <= dstop ? 1 : 0);  // (not past the last row)
                const int done = ((hit0 | hit1) & et) | (computing & (dl + 1 >= dstop ? 1 : 0));  // no hit: dw stays -1
                const int over = (done ^ 1) & (gst == G_RUN ? 1 : 0) & (dl + 1 >= dover ? 1 : 0);   // over budget
                dw = hit0 ? dl - q : (hit1 ? dl + 1 - q : dw);
                gst = done ? G_DONE : (over ? G_OVER : gst);
                over_events += over;
            }
            dl += 2;
            soff += 2 * rowbytes;
            steps += 2;
        } while (__ballot(gst == G_RUN) != 0);
        c_lane_steps += 64ull * (unsigned long long)steps;
        c_rounds += 1;
        // the main launch's beat for the helpers, every 32 passes of a wavefront
        if (a.mig_k > 0 && lane == 0 && (c_rounds & 31u) == 0u) atomicAdd(&a.qctl[kQcBeat], 1u);
        // the group's stored rows are read by its slot lane
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

        // ---- 6. traceback of finished windows, advance, output ----
        // Finished windows start their traceback; every traceback in the
        // wavefront then runs at most kTbEvents (match run, edit step)
        // events in this round and continues in the next one, so one very
        // long path does not hold the whole wavefront.
        if (slot && gst == G_DONE) {
            c_rows += (unsigned long long)(dw < 0 || a.no_et ? full : dw + 1);
            tb_d = dw;
            if (tb_d < 0 && kw == mw) tb_d = mw;   // no hit in rows 0..m_w-1: distance m_w
            if (tb_d < 0) {
                // no distance within k: the pair is not aligned
                c_windows += 1;
                c_ops += (unsigned long long)(kw + 1) + 2ull * nw + 7ull * nw * kw;
                a.edits[pair] = -1;
                a.text_end[pair] = -1;
                a.status[pair] = 1;
                a.n_runs[pair] = 0;
                pair = -1;
                atomicAdd(&a.qctl[2], 1u);
                if (a.helper) atomicSub(&a.qctl[kQcHInFlight], 1u);
                gst = G_EMPTY;
            } else {
                c_windows += 1;
                c_ops += (unsigned long long)(tb_d + 1) + 2ull * nw + 7ull * nw * tb_d;
                deep_run = tb_d >= a.mig_d ? deep_run + 1 : 0;
                tb_i = tb_j = tb_e = tb_bad = 0;
                tb_rc = z_init(mw, tb_d - 1);
            }
        }
        if (gst == G_DONE) gst = G_TB;
        if (__ballot(slot && gst == G_TB) != 0) {
            const bool tracing = slot && gst == G_TB;
            const GroupRec r = grec[g];
            const int jlim = min(mw, cap);
            const int ilim = min(nw, cap);              // a match run stops at the text window's end and at the cap
            uint32_t* const rout = a.runs + roff;       // the pair's run list (m + n + 1 >= 1 entries)
            const int rlast = (int)rcap - 1;
            // `fin` is an integer so that it lives in a vector register: a boolean
            // carried around a loop with a divergent body is kept as a lane mask
            // that the compiler re-merges with scalar operations at every event
            int fin = tracing ? 0 : 1;
            for (int ev = 0; ev < kTbEvents; ++ev) {
                if (__ballot(fin == 0) == 0) break;
                if (fin == 0) {
                    // match run at (tb_i, tb_j); characters past n_w never match
                    const uint64_t x = ((r.thi >> tb_i) ^ (r.phi >> tb_j)) | ((r.tlo >> tb_i) ^ (r.plo >> tb_j));
                    int L = x ? (int)__builtin_ctzll(x) : 64;
                    L = max(min(L, min(ilim - tb_i, jlim - tb_j)), 0);
                    const int ti = tb_i + L, tj = tb_j + L, td = tb_d;
                    // edit step at (ti, tj, td): bits tj, tj+1 of row td-1 at columns ti and ti+1.
                    // The loads go out first; the run bookkeeping below overlaps them.
                    uint64_t v0 = 0, v1 = 0, tb_de = 0;
                    // 32- and 48-bit forms: the loaded words as they are (low planes of
                    // columns ti and ti+1; for 48 bits, their two high halves in one word)
                    uint32_t w0 = 0, w1 = 0, wh = 0;
                    if constexpr (LR && (NARROW || SPLIT)) {
                        // as the global form below, from LDS for rows below R (every lane
                        // reads, at a clamped row) and from the global region under a
                        // branch taken only when some group needs a deeper row; the global
                        // words are consumed inside their branch
                        struct __attribute__((packed, aligned(4))) W2 { uint2 v; };
                        const uint32_t rr = (uint32_t)(max(td, 1) - 1);
                        const uint32_t c0 = (uint32_t)min(ti, stride - 1), c1 = (uint32_t)min(ti + 1, stride - 1);
                        const bool in_lds = rr < (uint32_t)R;
                        const uint32_t rl = min(rr, (uint32_t)max(R, 1) - 1u);
                        uint2 hv = uint2{0u, 0u};
                        if (NARROW) {
                            const uint32_t lo_row = lgbyte + rl * rowbytes;
                            w0 = *reinterpret_cast<const uint32_t*>(lrows + (lo_row + c0 * 4u));
                            w1 = *reinterpret_cast<const uint32_t*>(lrows + (lo_row + c1 * 4u));
                        } else {
                            const uint2 lv = reinterpret_cast<const W2*>(lrows + (lgbyte + rl * lobytes + c0 * 4u))->v;
                            hv = reinterpret_cast<const W2*>(lrows + (lhiplane + rl * hibytes + (c0 & ~1u) * 2u))->v;
                            w0 = lv.x;
                            w1 = lv.y;
                        }
                        if (__ballot(!in_lds) != 0) {
                            if (NARROW) {
                                const uint32_t lo_row = gbyte + __umul24(rr, rowbytes);
                                const uint32_t g0 = *reinterpret_cast<const uint32_t*>(bdent + (lo_row + c0 * 4u));
                                const uint32_t g1 = *reinterpret_cast<const uint32_t*>(bdent + (lo_row + c1 * 4u));
                                w0 = in_lds ? w0 : g0;
                                w1 = in_lds ? w1 : g1;
                            } else {
                                const uint2 gl = reinterpret_cast<const W2*>(bdent + (gbyte + __umul24(rr, lobytes) + c0 * 4u))->v;
                                const uint2 gh = reinterpret_cast<const W2*>(bdent + (hiplane + __umul24(rr, hibytes) + (c0 & ~1u) * 2u))->v;
                                w0 = in_lds ? w0 : gl.x;
                                w1 = in_lds ? w1 : gl.y;
                                hv = in_lds ? hv : gh;
                            }
                        }
                        if (SPLIT) wh = __builtin_amdgcn_alignbit(hv.y, hv.x, (c0 & 1u) * 16u);
                    } else if constexpr (LR) {
                        const uint32_t rr = (uint32_t)(max(td, 1) - 1);
                        const uint32_t c0 = (uint32_t)min(ti, stride - 1), c1 = (uint32_t)min(ti + 1, stride - 1);
                        const bool in_lds = rr < (uint32_t)R;
                        struct __attribute__((packed, aligned(4))) W2 { uint64_t v; };
                        uint64_t lw = 0, hw = 0;
                        // rows below R from LDS (every lane reads, at a clamped row); the
                        // others from the global region, skipped when no lane needs one.
                        // The global words are consumed inside their branch, so an event
                        // that reads only LDS waits for no vector-memory operation (the
                        // counter it shares with the run-list stores)
                        if (R > 0) {
                            const uint32_t rl = min(rr, (uint32_t)R - 1u);
                            const uint32_t lo_row = lgbyte + rl * (SPLIT ? lobytes : rowbytes);
                            if (NARROW) {
                                lw = *reinterpret_cast<const uint32_t*>(lrows + (lo_row + c0 * ESZ));
                                hw = *reinterpret_cast<const uint32_t*>(lrows + (lo_row + c1 * ESZ));
                            } else if (SPLIT) {
                                lw = reinterpret_cast<const W2*>(lrows + (lo_row + c0 * 4u))->v;
                                hw = reinterpret_cast<const W2*>(lrows + (lhiplane + rl * hibytes + (c0 & ~1u) * 2u))->v;
                            } else {
                                lw = *reinterpret_cast<const uint64_t*>(lrows + (lo_row + c0 * ESZ));
                                hw = *reinterpret_cast<const uint64_t*>(lrows + (lo_row + c1 * ESZ));
                            }
                        }
                        if (__ballot(!in_lds) != 0) {
                            const uint32_t lo_row = gbyte + __umul24(rr, SPLIT ? lobytes : rowbytes);
                            uint64_t glw, ghw;
                            if (NARROW) {
                                glw = *reinterpret_cast<const uint32_t*>(bdent + (lo_row + c0 * ESZ));
                                ghw = *reinterpret_cast<const uint32_t*>(bdent + (lo_row + c1 * ESZ));
                            } else if (SPLIT) {
                                glw = reinterpret_cast<const W2*>(bdent + (lo_row + c0 * 4u))->v;
                                ghw = reinterpret_cast<const W2*>(bdent + (hiplane + __umul24(rr, hibytes) + (c0 & ~1u) * 2u))->v;
                            } else {
                                glw = *reinterpret_cast<const uint64_t*>(bdent + (lo_row + c0 * ESZ));
                                ghw = *reinterpret_cast<const uint64_t*>(bdent + (lo_row + c1 * ESZ));
                            }
                            lw = in_lds ? lw : glw;
                            hw = in_lds ? hw : ghw;
                        }
                        if (SPLIT) {
                            // columns ti and ti+1 of both planes, as one 8-byte word each (the
                            // 16-bit word from the 4-byte boundary at or below column ti)
                            const uint64_t hs = hw >> ((c0 & 1u) * 16u);
                            v0 = (uint64_t)(uint32_t)lw | (uint64_t)(hs & 0xFFFFu) << 32;
                            v1 = (lw >> 32) | (uint64_t)((hs >> 16) & 0xFFFFu) << 32;
                        } else {
                            v0 = lw;
                            v1 = hw;
                        }
                    } else if constexpr (EDGES) {
                        // the edges of entry (ti, td): slot td-1 of column ti, I and S in the
                        // first 16 bytes, D (and M) in the second
                        const uint32_t ro = gbyte + __umul24(slot_of((uint32_t)(max(td, 1) - 1)), rowbytes);
                        const uint4* const e = reinterpret_cast<const uint4*>(bdent + (ro + (uint32_t)min(ti, stride - 1) * ESZ));
                        const uint4 is = e[0], dm = e[1];
                        v0 = (uint64_t)is.y << 32 | is.x;   // I edge
                        v1 = (uint64_t)is.w << 32 | is.z;   // S edge
                        tb_de = (uint64_t)dm.y << 32 | dm.x;   // D edge
                    } else {
                        const uint32_t ro = gbyte + __umul24(slot_of((uint32_t)(max(td, 1) - 1)), rowbytes);
                        const char* const e0 = bdent + (ro + (uint32_t)min(ti, stride - 1) * ESZ);
                        const char* const e1 = bdent + (ro + (uint32_t)min(ti + 1, stride - 1) * ESZ);
                        if (NARROW) {
                            w0 = *reinterpret_cast<const uint32_t*>(e0);
                            w1 = *reinterpret_cast<const uint32_t*>(e1);
                        } else if (SPLIT) {
                            // columns ti and ti+1 of both planes, one 8-byte load per plane (the
                            // 16-bit words from the 4-byte boundary at or below column ti)
                            struct __attribute__((packed, aligned(4))) W2 { uint2 v; };
                            const uint32_t rr = slot_of((uint32_t)(max(td, 1) - 1));
                            const uint32_t c0 = (uint32_t)min(ti, stride - 1);
                            const uint2 lw = reinterpret_cast<const W2*>(bdent + (gbyte + __umul24(rr, lobytes) + c0 * 4u))->v;
                            const uint2 hw = reinterpret_cast<const W2*>(bdent + (hiplane + __umul24(rr, hibytes) + (c0 & ~1u) * 2u))->v;
                            w0 = lw.x;
                            w1 = lw.y;
                            // high halves of columns ti (bits 0..15) and ti+1 (bits 16..31)
                            wh = __builtin_amdgcn_alignbit(hw.y, hw.x, (c0 & 1u) * 16u);
                        } else {
                            v0 = *reinterpret_cast<const uint64_t*>(e0);
                            v1 = *reinterpret_cast<const uint64_t*>(e1);
                        }
                    }
                    // the run list always holds the open run at index nruns, so
                    // extending or starting a run is one unconditional store
                    {
                        const bool same = cur_op == 0;
                        nruns += (!same && cur_len > 0 && L > 0) ? 1 : 0;
                        cur_len = L == 0 ? cur_len : (same ? cur_len + L : L);
                        cur_op = L == 0 ? cur_op : 0;
                        rout[(uint32_t)min(nruns, rlast)] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                    }
                    const bool edit = !(tj >= jlim || ti >= cap);
                    const int has_t = ti < nw;
                    int sb, ib, db;
                    if constexpr (EDGES) {
                        // the stored edges, bit tj (their bit 63 is the shifted-in 1)
                        sb = has_t & (int)((v1 >> (tj & 63)) & 1ull);
                        ib = (int)((v0 >> (tj & 63)) & 1ull);
                        db = has_t & (int)((tb_de >> (tj & 63)) & 1ull);
                    } else if constexpr (NARROW || SPLIT) {
                        // W-O <= 47: an edit step has tj <= 46, so bits tj and tj+1 are stored
                        // bits and no implicit bit 64 is read.  Bits tj.. of each entry: a
                        // 32-bit entry shifted, or a 48-bit one funnel-shifted out of its high
                        // half and low word (out of the high half alone from bit 32 on)
                        const uint32_t sh = (uint32_t)tj & 31u;
                        uint32_t a0, a1;
                        if constexpr (NARROW) {
                            a0 = w0 >> sh;
                            a1 = w1 >> sh;
                        } else {
                            const bool up = tj >= 32;
                            const uint32_t h1 = wh >> 16;
                            a0 = __builtin_amdgcn_alignbit(wh, up ? wh : w0, sh);
                            a1 = __builtin_amdgcn_alignbit(h1, up ? h1 : w1, sh);
                        }
                        // columns at or past n_w hold the initial column
                        const uint32_t rcb = (uint32_t)(tb_rc >> (tj & 63));
                        a0 = ti < nw ? a0 : rcb;                          // Z[ti][td-1] >> tj
                        a1 = ti + 1 < nw ? a1 : rcb;                      // Z[ti+1][td-1] >> tj
                        sb = has_t & (int)((a1 >> 1) & 1u);
                        ib = (int)((a0 >> 1) & 1u);
                        db = has_t & (int)(a1 & 1u);
                    } else {
                        const uint64_t za = ti < nw ? v0 : tb_rc;        // Z[ti][td-1]
                        const uint64_t zb = ti + 1 < nw ? v1 : tb_rc;    // Z[ti+1][td-1]
                        // bits tj and tj+1 (tj <= 63 in an edit step; bit 64 is the implicit set bit)
                        const uint64_t sa = za >> (tj & 63), sz = zb >> (tj & 63);
                        const int top = tj >= 63 ? 1 : 0;
                        sb = has_t & (((int)(sz >> 1) & 1) | top);
                        ib = ((int)(sa >> 1) & 1) | top;
                        db = has_t & (int)(sz & 1);
                    }
                    const int op = sb ? 1 : (ib ? 2 : 3);
                    tb_bad |= edit & ((td <= 0) | !(sb | ib | db));
                    tb_i = ti + (edit && op != 2 ? 1 : 0);
                    tb_j = tj + (edit && op != 3 ? 1 : 0);
                    tb_d = td - (edit ? 1 : 0);
                    tb_e += edit ? 1 : 0;
                    tb_rc = edit ? tb_rc << 1 : tb_rc;   // one row down: m_w - d grows by one (it is >= 1 here)
                    {
                        const bool same = cur_op == op;
                        nruns += (edit && !same && cur_len > 0) ? 1 : 0;
                        cur_len = !edit ? cur_len : (same ? cur_len + 1 : 1);
                        cur_op = !edit ? cur_op : op;
                        rout[(uint32_t)min(nruns, rlast)] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                    }
                    fin = (!edit || tb_j >= jlim || tb_i >= cap || tb_bad) ? 1 : 0;
                }
            }
            if (tracing && fin) {
                // advance the pair past the traced characters
                edits += tb_e;
                p0 += tb_j;
                t0 += tb_i;
                gst = G_EMPTY;
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
                    if (a.helper) atomicSub(&a.qctl[kQcHInFlight], 1u);
                } else if (a.mig_k > 0 && deep_run >= a.mig_k) {
                    // off track: hand the pair to the helper launch, which gives a window
                    // more lanes (each pair moves at most once, so hring never overflows).
                    // The in-flight word reserves a helper slot; once a helper has closed
                    // the gate it exceeds the cap and the pair stays here
                    if (atomicAdd(&a.qctl[kQcHInFlight], 1u) < (uint32_t)a.mig_cap) {
                        const uint32_t tq = atomicAdd(&a.qctl[kQcHTail], 1u);
                        int32_t* st = a.pstate + 8 * (int64_t)pair;
                        st[0] = p0; st[1] = t0; st[2] = edits; st[3] = nruns; st[4] = cur_op; st[5] = cur_len;
                        st[6] = 0; st[7] = 0;
                        __hip_atomic_store(&a.hring[tq], pair + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        pair = -1;
                        c_yield += 1;
                    } else {
                        atomicSub(&a.qctl[kQcHInFlight], 1u);
                        deep_run = 0;   // the helpers are full: try again after mig_k more deep windows
                    }
                } else if (a.yield_chars > 0 && p0 - p0_take >= a.yield_chars) {
                    // hand the pair back to the queue between windows
                    const uint32_t tq = atomicAdd(&a.qctl[1], 1u);
                    if ((int64_t)tq < a.qcap) {
                        int32_t* st = a.pstate + 8 * (int64_t)pair;
                        st[0] = p0; st[1] = t0; st[2] = edits; st[3] = nruns; st[4] = cur_op; st[5] = cur_len;
                        st[6] = 0; st[7] = 0;
                        __hip_atomic_store(&a.ring[tq], pair + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        pair = -1;
                        c_yield += 1;
                    }
                }
            }
        }
        // the group's L lanes learn that its traceback ended
        {
            const uint64_t tbm = __ballot(slot && gst == G_TB);
            if ((tbm & gbit) == 0 && gst == G_TB) gst = G_EMPTY;
        }
        // traceback's reads of the stored rows finish before the next pass overwrites them
        __syncthreads();
    }

    // ---- counters ----
    if (slot) {
        c_fallback = over_events;
        if (c_windows) atomicAdd(&a.stats[ST_WINDOWS], c_windows);
        if (c_ops) atomicAdd(&a.stats[ST_OPS_ALG], c_ops);
        if (c_fallback) atomicAdd(&a.stats[ST_FALLBACK], c_fallback);
        if (c_rows) atomicAdd(&a.stats[ST_ROWS], c_rows);
        if (c_err) atomicAdd(&a.stats[ST_ERRORS], c_err);
        if (c_yield) atomicAdd(&a.stats[ST_YIELDS], c_yield);
    }
    if (lane == 0) {
        atomicAdd(&a.stats[ST_LANE_STEPS], c_lane_steps);
        atomicAdd(&a.stats[ST_ROUNDS], c_rounds);
    }
}

}  // namespace

int cols_dent_stride(int cap, int ng) {
    const int cols = cap + 1 < 64 ? cap + 1 : 64;   // stored columns 0..min(cap, 63)
    const int cb = cols_per_lane(ng);
    return (cols + cb - 1) / cb * cb;               // whole lanes of CB columns
}

size_t cols_dent_bytes(int grid, int cap, int ng, bool edges, int ring_rows) {
    const int rows = ring_rows > 0 ? ring_rows : kStoredRows;
    return (size_t)grid * ng * rows * (size_t)cols_dent_stride(cap, ng) * sizeof(uint64_t) * (edges ? 4 : 1);
}

// 32-bit stored entries when traceback reads bits 0..31 at most, 48-bit ones
// (two planes) when it reads bits 0..47 at most; the learned form keeps 64-bit
// entries at every W-O
static int cols_store(bool learned, int cap) { return learned ? 0 : (cap <= 31 ? 1 : (cap <= 47 ? 2 : 0)); }

// bytes of one stored row of one group (both planes of the 48-bit form)
size_t cols_lds_row_bytes(bool learned, int cap, int stride) {
    const int st = cols_store(learned, cap);
    return (size_t)stride * (st == 1 ? 4 : (st == 2 ? 6 : 8));
}

template <bool LEARNED, int ST>
static const void* cols_fn(int ng) {
    switch (ng) {
    case 4: return (const void*)cols_kernel<LEARNED, 4, ST, 0>;
    case 8: return (const void*)cols_kernel<LEARNED, 8, ST, 0>;
    default: return (const void*)cols_kernel<LEARNED, 16, ST, 0>;
    }
}

// plain mode also has 32 windows per wavefront (two lanes per window, 32
// columns each: the lane-per-pair end of the mapping) and 10 (six lanes of 12
// columns; four lanes idle), which puts one wavefront on each SIMD for about
// ten pairs per SIMD; and, with 4, 8 or 16 windows, the form that keeps the
// lowest stored rows in LDS
template <int ST>
static const void* cols_fn_plain(int ng, int sm) {
    if (sm == 1) {
        if (ng == 4) return (const void*)cols_kernel<false, 4, ST, 1>;
        if (ng == 8) return (const void*)cols_kernel<false, 8, ST, 1>;
        return (const void*)cols_kernel<false, 16, ST, 1>;
    }
    if (sm == 2) {
        if (ng == 4) return (const void*)cols_kernel<false, 4, ST, 2>;
        if (ng == 8) return (const void*)cols_kernel<false, 8, ST, 2>;
        return (const void*)cols_kernel<false, 16, ST, 2>;
    }
    if (ng == 32) return (const void*)cols_kernel<false, 32, ST, 0>;
    if (ng == 10) return (const void*)cols_kernel<false, 10, ST, 0>;
    return cols_fn<false, ST>(ng);
}

// the one-wavefront-per-SIMD forms: plain mode, rows in global memory, 4, 8,
// 10 or 16 windows per wavefront
template <int ST>
static const void* cols_fn_one(int ng, int sm) {
    if (sm == 1) return ng == 16 ? (const void*)cols_kernel<false, 16, ST, 1, true> : (const void*)cols_kernel<false, 4, ST, 1, true>;
    if (ng == 4) return (const void*)cols_kernel<false, 4, ST, 0, true>;
    if (ng == 8) return (const void*)cols_kernel<false, 8, ST, 0, true>;
    if (ng == 16) return (const void*)cols_kernel<false, 16, ST, 0, true>;
    return (const void*)cols_kernel<false, 10, ST, 0, true>;
}

bool cols_one_per_simd_ok(bool learned, int ng, int sm, bool edges) {
    return !learned && !edges && ((sm == 0 && (ng == 4 || ng == 8 || ng == 10 || ng == 16)) || (sm == 1 && (ng == 4 || ng == 16)));
}

// the edge-storing ablation form: plain mode, 4, 8 or 16 windows per wavefront
static const void* cols_fn_edges(int ng, int sm) {
    if (sm == 2) {
        if (ng == 4) return (const void*)cols_kernel<false, 4, 3, 2>;
        if (ng == 8) return (const void*)cols_kernel<false, 8, 3, 2>;
        return (const void*)cols_kernel<false, 16, 3, 2>;
    }
    if (ng == 4) return (const void*)cols_kernel<false, 4, 3, 0>;
    if (ng == 8) return (const void*)cols_kernel<false, 8, 3, 0>;
    return (const void*)cols_kernel<false, 16, 3, 0>;
}

int cols_max_blocks_per_cu(bool learned, int ng, size_t lds, int cap, int sm, bool edges, bool one) {
    int nb = 0;
    const int st = cols_store(learned, cap);
    if (one && !cols_one_per_simd_ok(learned, ng, sm, edges)) return 1;
    const void* f = one ? (st == 1 ? cols_fn_one<1>(ng, sm) : (st == 2 ? cols_fn_one<2>(ng, sm) : cols_fn_one<0>(ng, sm)))
                  : learned ? cols_fn<true, 0>(ng)
                  : edges ? cols_fn_edges(ng, sm == 2 ? 2 : 0)
                  : (st == 1 ? cols_fn_plain<1>(ng, sm)
                             : (st == 2 ? cols_fn_plain<2>(ng, sm) : cols_fn_plain<0>(ng, sm)));
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64, lds) != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_align_cols(const AlignArgs& a, int grid, int ng, size_t lds, hipStream_t s) {
    const bool learned = a.mode == 1;
    const int st = cols_store(learned, a.cap);
    const bool small = ng == 4 || ng == 8 || ng == 16;
    const int sm = learned || !small ? 0 : (a.lds_rows > 0 ? 1 : (a.ring_rows > 0 ? 2 : 0));
    // the host sized the stored-row region for the ring (or the LDS rows): every
    // launch below must use that layout, so a combination without one is refused
    if ((a.ring_rows > 0 || a.lds_rows > 0) && (learned || !small)) return hipErrorInvalidValue;
    if (a.edges && a.lds_rows > 0) return hipErrorInvalidValue;
    if (a.one_per_simd && !cols_one_per_simd_ok(learned, ng, sm, a.edges != 0)) return hipErrorInvalidValue;
#define SCG_COLS_LAUNCH(LRN, NGV, STV, LRV) \
    hipLaunchKernelGGL((cols_kernel<LRN, NGV, STV, LRV>), dim3(grid), dim3(64), lds, s, a)
#define SCG_COLS_ONE(STV)                                                                          \
    do {                                                                                           \
        if (sm == 1 && ng == 16) hipLaunchKernelGGL((cols_kernel<false, 16, STV, 1, true>), dim3(grid), dim3(64), lds, s, a); \
        else if (sm == 1) hipLaunchKernelGGL((cols_kernel<false, 4, STV, 1, true>), dim3(grid), dim3(64), lds, s, a);  \
        else if (ng == 4) hipLaunchKernelGGL((cols_kernel<false, 4, STV, 0, true>), dim3(grid), dim3(64), lds, s, a);  \
        else if (ng == 8) hipLaunchKernelGGL((cols_kernel<false, 8, STV, 0, true>), dim3(grid), dim3(64), lds, s, a);  \
        else if (ng == 16) hipLaunchKernelGGL((cols_kernel<false, 16, STV, 0, true>), dim3(grid), dim3(64), lds, s, a); \
        else hipLaunchKernelGGL((cols_kernel<false, 10, STV, 0, true>), dim3(grid), dim3(64), lds, s, a);              \
    } while (0)
#define SCG_COLS_PLAIN(STV)                                  \
    do {                                                     \
        if (sm == 1) {                                       \
            if (ng == 4) SCG_COLS_LAUNCH(false, 4, STV, 1);          \
            else if (ng == 8) SCG_COLS_LAUNCH(false, 8, STV, 1);     \
            else SCG_COLS_LAUNCH(false, 16, STV, 1);                 \
        } else if (sm == 2) {                                \
            if (ng == 4) SCG_COLS_LAUNCH(false, 4, STV, 2);          \
            else if (ng == 8) SCG_COLS_LAUNCH(false, 8, STV, 2);     \
            else SCG_COLS_LAUNCH(false, 16, STV, 2);                 \
        } else if (ng == 4) SCG_COLS_LAUNCH(false, 4, STV, 0);       \
        else if (ng == 8) SCG_COLS_LAUNCH(false, 8, STV, 0);         \
        else if (ng == 16) SCG_COLS_LAUNCH(false, 16, STV, 0);       \
        else if (ng == 10) SCG_COLS_LAUNCH(false, 10, STV, 0);       \
        else SCG_COLS_LAUNCH(false, 32, STV, 0);                     \
    } while (0)
    if (a.one_per_simd) {
        if (st == 1) SCG_COLS_ONE(1);
        else if (st == 2) SCG_COLS_ONE(2);
        else SCG_COLS_ONE(0);
    } else if (a.edges) {
        // the stored-row layout (64 rows or the ring) must be the one the host allocated
        if (sm == 2) {
            if (ng == 4) SCG_COLS_LAUNCH(false, 4, 3, 2);
            else if (ng == 8) SCG_COLS_LAUNCH(false, 8, 3, 2);
            else SCG_COLS_LAUNCH(false, 16, 3, 2);
        } else if (ng == 4) SCG_COLS_LAUNCH(false, 4, 3, 0);
        else if (ng == 8) SCG_COLS_LAUNCH(false, 8, 3, 0);
        else SCG_COLS_LAUNCH(false, 16, 3, 0);
    } else if (learned) {
        if (ng == 4) SCG_COLS_LAUNCH(true, 4, 0, 0);
        else if (ng == 8) SCG_COLS_LAUNCH(true, 8, 0, 0);
        else SCG_COLS_LAUNCH(true, 16, 0, 0);
    } else if (st == 1) {
        SCG_COLS_PLAIN(1);
    } else if (st == 2) {
        SCG_COLS_PLAIN(2);
    } else {
        SCG_COLS_PLAIN(0);
    }
#undef SCG_COLS_PLAIN
#undef SCG_COLS_ONE
#undef SCG_COLS_LAUNCH
    return hipGetLastError();
}
