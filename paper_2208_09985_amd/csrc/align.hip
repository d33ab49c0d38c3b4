// Fused, persistent windowed GenASM-DC + GenASM-TB kernel for gfx950.
//
// Mapping (one wavefront = one workgroup, 64 lanes):
//   * Lanes are error rows.  A window that computes w rows occupies a
//     contiguous segment of w lanes (lane base+d = row d); several windows of
//     different pairs share a wavefront, one idle "gap" lane after each
//     segment, so the first row of every segment receives zeros from below.
//   * Rows advance over the text columns on an anti-diagonal schedule: at
//     step s, row d works on column i = n_w-1-s+d.  Entries on one NW-SE
//     diagonal are independent (Section 2.2.1, intra-task parallelism).
//     Row d needs R[i][d-1] and R[i+1][d-1] from row d-1; both arrive from
//     the neighbouring lane through one DPP wave_shr:1 per 32-bit half.
//   * Each lane holds one 64-bit bitvector (two VGPRs).  The kernel keeps the
//     complement Z = ~R in LSB-first order (bit j = pattern position j), so
//     the update of Algorithm 1 becomes
//         Z[i][d] = ((Z[i][d-1] | Z[i+1][d-1]) >> 1 | top)   -- ~I, ~S
//                 | Z[i+1][d-1]                              -- ~D
//                 | ((Z[i+1][d] >> 1 | top) & EQ[text[i]])   -- ~M
//     with EQ = ~PM and `top` the bit shifted in where R shifts in a 0.
//     A 0 in the msb of R[0][d] is bit 0 of Z[0][d] set.
//   * Only entries that traceback can read are stored (Section 2.4.1: the
//     entries, not the edges; Section 2.4.2: columns 0..W-O only), in LDS as
//     dent[column][lane], 8 bytes each.
//   * Early termination (Section 2.4.3): the first row whose column-0 entry
//     has the msb cleared is d_w.  Every four steps a wavefront ballot over
//     the rows that have passed column 0 ends the pass once every window in
//     it has found its d_w.
//   * Traceback runs in the slot lane of each window (lanes 0..ns-1).  Along
//     a tight path with text[i] == pattern[j] the M term always holds (the
//     suffix distance never increases along a diagonal of matches), so match
//     runs are skipped with one XOR of the 2-bit planes and a trailing-zero
//     count; only edit steps read LDS, and only row d-1.
//   * Pairs are taken from a global atomic queue (the paper's global queue of
//     pairs, Section 2.5).  A pair that has advanced yield_chars pattern
//     characters saves its small state and goes back to the queue, so pairs
//     whose windows need many rows do not pin one wavefront.  A wavefront
//     exits when every pair is finished or none of its slots can receive one.
//   * Row budgets: plain mode computes rows 0..k_w of every window.  The
//     learned and fixed modes first compute fewer rows; a window that finds
//     no d_w within them is retried with a larger budget (w -> 2w+1, at most
//     all rows).  Rows <= d never depend on rows > d, so the result is
//     bit-identical.
#include "predictor.h"

namespace {

constexpr uint32_t kDppWaveShr1 = 0x138;
constexpr int kEqPadBefore = 64;   // EQ-table entries before the first slot's table
constexpr int kEqPadAfter = 72;    // and after the last one: reads reach index steps+6 <= 133 past a table start

__device__ __forceinline__ uint32_t from_lower_lane(uint32_t x) {
    // lane l receives lane l-1's value; lane 0 receives 0
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kDppWaveShr1, 0xF, 0xF, true);
}

// Z of the right column (i = n_w): bit j set iff m_w - j <= d
__device__ __forceinline__ uint64_t z_right_column(int mw, int d) {
    const int s = mw - d;
    return s <= 0 ? ~0ull : (s >= 64 ? 0ull : (~0ull << s));
}

__device__ __forceinline__ int zbit(uint64_t z, int p) { return p >= 64 ? 1 : (int)((z >> p) & 1ull); }

// Append `len` operations `op` to a pair's run list, merging equal neighbours.
__device__ __forceinline__ void emit_run(int op, int len, int& cur_op, int& cur_len, int& nruns,
                                         uint32_t* __restrict__ runs, int64_t roff, int64_t rcap) {
    const bool same = cur_op == op;
    if (!same && cur_len > 0) {
        if (nruns < rcap) runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
        ++nruns;
    }
    cur_len = same ? cur_len + len : len;
    cur_op = op;
}

struct SlotRec {       // LDS record of a window scheduled in the current round
    int32_t base;      // first lane of its segment, -1 if not scheduled
    int32_t width;     // rows (lanes) computed
    int32_t n_w, m_w;
};

// Three consecutive Plane2 words of one sequence, starting at word q.  A
// window starting inside word q needs words q and q+1; the third word is
// loaded one round ahead, so advancing by at most 64 characters never waits
// on global memory.
struct PlaneBuf {
    Plane2 w0, w1, w2;
    int q;
};

__device__ __forceinline__ Plane2 load_word(const Plane2* __restrict__ seq, int q, int qmax) {
    return q <= qmax ? seq[q] : Plane2{0, 0};
}

__device__ __forceinline__ void buf_fill(PlaneBuf& b, const Plane2* __restrict__ seq, int q, int qmax) {
    b.q = q;
    b.w0 = load_word(seq, q, qmax);
    b.w1 = load_word(seq, q + 1, qmax);
    b.w2 = load_word(seq, q + 2, qmax);
}

__device__ __forceinline__ void buf_seek(PlaneBuf& b, const Plane2* __restrict__ seq, int q, int qmax) {
    if (q == b.q) return;
    if (q == b.q + 1) {
        b.w0 = b.w1;
        b.w1 = b.w2;
        b.w2 = load_word(seq, q + 2, qmax);
        b.q = q;
    } else {
        buf_fill(b, seq, q, qmax);
    }
}

__device__ __forceinline__ void buf_window(const PlaneBuf& b, int pos, uint64_t& lo, uint64_t& hi) {
    const int r = pos & 63;
    if (r == 0) {
        lo = b.w0.lo;
        hi = b.w0.hi;
    } else {
        lo = (b.w0.lo >> r) | (b.w1.lo << (64 - r));
        hi = (b.w0.hi >> r) | (b.w1.hi << (64 - r));
    }
}

// One diagonal step of one lane: column c of this lane's row.  Branch-free:
// lanes outside their column range keep their value (a lane that has not
// started holds its right-column entry), and stores outside the traceback
// region go to a per-lane dump slot.
#define DC_STEP(E, C)                                                                        \
    do {                                                                                     \
        const uint32_t nlo = from_lower_lane(zlo);                                           \
        const uint32_t nhi = from_lower_lane(zhi);                                           \
        const int c_ = (C);                                                                  \
        const uint32_t tl = nlo | nelo, th = nhi | nehi;                                     \
        const uint32_t al = __builtin_amdgcn_alignbit(th, tl, 1);                            \
        const uint32_t ah = __builtin_amdgcn_alignbit(cin, th, 1);                           \
        const uint32_t bl = __builtin_amdgcn_alignbit(zhi, zlo, 1);                          \
        const uint32_t bh = __builtin_amdgcn_alignbit(1u, zhi, 1);                           \
        const uint32_t ulo = (bl & (uint32_t)(E)) | al | nelo;                               \
        const uint32_t uhi = (bh & (uint32_t)((E) >> 32)) | ah | nehi;                       \
        const bool valid_ = (unsigned)c_ < (unsigned)rnw;                                    \
        zlo = valid_ ? ulo : zlo;                                                            \
        zhi = valid_ ? uhi : zhi;                                                            \
        uint64_t* const at_ = (unsigned)c_ < (unsigned)nstore ? dp + c_ * 64 : dump;         \
        *at_ = ((uint64_t)zhi << 32) | zlo;                                                  \
        nelo = nlo;                                                                          \
        nehi = nhi;                                                                          \
    } while (0)

template <bool LEARNED>
__global__ __launch_bounds__(64) void align_kernel(const AlignArgs a) {
    extern __shared__ uint64_t smem[];
    const int lane = threadIdx.x;
    const int NS = a.ns;
    uint64_t* dent = smem;                                                     // [ccols + 1][64]; last = dump
    uint64_t* eqt = dent + (size_t)(a.ccols + 1) * 64;                         // pads + [NS][64]
    WinPlanes* wpl = (WinPlanes*)(eqt + kEqPadBefore + (size_t)NS * 64 + kEqPadAfter);  // [NS]
    SlotRec* srec = (SlotRec*)(wpl + NS);                                      // [NS]
    PlaneBuf* pbufs = (PlaneBuf*)(srec + NS);                                  // [NS] pattern words
    PlaneBuf* tbufs = pbufs + NS;                                              // [NS] text words

    const int cap = a.cap;

    // ---- slot-lane state (meaningful in lanes < NS) ----
    int pair = -1, p0 = 0, t0 = 0, m = 0, n = 0, edits = 0, nruns = 0, cur_op = 0, cur_len = 0;
    int next_w = 0, bad_state = 0, pqmax = 0, tqmax = 0, p0_take = 0;
    int64_t roff = 0, rcap = 0, pending = -1;
    int polled = 0;       // ring[pending] as last read (0: not yet written)
    const Plane2* pseq = nullptr;
    const Plane2* tseq = nullptr;
    bool exhausted = lane >= NS;
    unsigned long long c_windows = 0, c_ops = 0, c_fallback = 0, c_rows = 0, c_err = 0, c_yield = 0;
    unsigned long long c_lane_steps = 0, c_rounds = 0;
    int rot = 0;

    for (;;) {
        // ---- 1. refill empty slots from the queue ----
        // A slot reserves one queue index (pop) and keeps it until the entry
        // is written: a yielding pair may reserve a tail index just before it
        // stores there.  Pop and poll are issued during the previous round's
        // DC pass and traceback, so a round waits on global memory only when
        // a new pair starts (its saved state and first plane words).
        auto activate = [&]() {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const bool fresh = pending < a.npairs;
            const int pid = polled - 1;
            pending = -1;
            polled = 0;
            const int pm = a.plen[pid], pn = a.tlen[pid];
            if (fresh && (a.bad[pid] || pm == 0)) {
                const bool bad = a.bad[pid] != 0;
                a.edits[pid] = bad ? -1 : 0;
                a.text_end[pid] = bad ? -1 : 0;
                a.status[pid] = bad ? 2 : 0;
                a.n_runs[pid] = 0;
                atomicAdd(&a.qctl[2], 1u);
                return;
            }
            pair = pid; m = pm; n = pn; bad_state = 0;
            if (fresh) {
                p0 = 0; t0 = 0; edits = 0; nruns = 0; cur_op = 0; cur_len = 0; next_w = 0;
            } else {
                const int32_t* st = a.pstate + 8 * (int64_t)pid;
                p0 = st[0]; t0 = st[1]; edits = st[2]; nruns = st[3]; cur_op = st[4]; cur_len = st[5];
                next_w = st[6];
            }
            p0_take = p0;
            roff = a.runs_off[pid];
            rcap = a.runs_off[pid + 1] - roff;
            pseq = a.pplanes + a.pword[pid];
            tseq = a.tplanes + a.tword[pid];
            pqmax = (pm + 63) >> 6;   // the padding word
            tqmax = (pn + 63) >> 6;
            buf_fill(pbufs[lane], pseq, p0 >> 6, pqmax);
            buf_fill(tbufs[lane], tseq, t0 >> 6, tqmax);
        };
        // with no active slot in the wavefront, pop and poll now
        if (__ballot(pair >= 0 || (!exhausted && polled != 0)) == 0 && !exhausted && pair < 0) {
            if (pending < 0) pending = (int64_t)atomicAdd(&a.qctl[0], 1u);
            if (pending >= a.qcap) exhausted = true;
            else polled = __hip_atomic_load(&a.ring[pending], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!exhausted && pair < 0 && polled != 0) activate();
        if (__ballot(pair >= 0) == 0) {
            // leave once every pair is finished or no slot can ever receive
            // one; otherwise wait for yielded pairs
            const bool waiting = !exhausted && pair < 0;
            if (__ballot(waiting) == 0) break;
            if (__hip_atomic_load(&a.qctl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (uint32_t)a.npairs) break;
            __builtin_amdgcn_s_sleep(16);
            continue;
        }
        const bool active = pair >= 0;

        // ---- 2. window geometry of each active slot ----
        int mw = 0, nw = 0, kw = 0, rows_full = 0, w = 0;
        WinPlanes wp{0, 0, 0, 0, 0, 0};
        if (active) {
            mw = min(a.W, m - p0);
            nw = min(a.W, n - t0);
            kw = min(a.k, mw);
            rows_full = (kw == mw) ? mw : kw + 1;   // row m_w is implicit: D(0,0) <= m_w
            PlaneBuf pb = pbufs[lane];
            buf_seek(pb, pseq, p0 >> 6, pqmax);
            buf_window(pb, p0, wp.plo, wp.phi);
            pbufs[lane] = pb;
            if (nw > 0) {
                PlaneBuf tb = tbufs[lane];
                buf_seek(tb, tseq, t0 >> 6, tqmax);
                buf_window(tb, t0, wp.tlo, wp.thi);
                tbufs[lane] = tb;
            }
            wp.m_w = mw;
            wp.n_w = nw;
            wpl[lane] = wp;
            if (next_w > 0) w = min(next_w, rows_full);
            else if (a.mode == 2) w = min(a.fixed_rows, rows_full);
            else w = rows_full;
        }

        // ---- 3. learned row budget: features -> MLP (MFMA) -> smallest confident budget ----
        if constexpr (LEARNED) {
            // operand registers are reloaded each round (L1-resident weights)
            // so they do not stay live across the DC pass
            MlpRegs mlp;
            mlp_load_packed(mlp, a.model.operands, lane);
            __syncthreads();
            const int s = lane & 15, g = lane >> 4;
            half4_t x4 = {0, 0, 0, 0};
            if (s < NS) {
                const WinPlanes o = wpl[s];
                for (int e = 0; e < 4; ++e) x4[e] = feature_to_input(window_feature(o, 4 * g + e));
            }
            half4_t hid[4];
            const float4_t logit = mlp_tile_forward(mlp, x4, hid);
            if (active && next_w == 0) {
                // lane s < 16 holds classes 0..3 of slot s
                const int C = a.model.C;
                float mx = logit[0];
                for (int c = 1; c < C; ++c) mx = fmaxf(mx, logit[c]);
                float p[4], tot = 0.f;
                for (int c = 0; c < C; ++c) { p[c] = __expf(logit[c] - mx); tot += p[c]; }
                int cls = C - 1;
                float cum = 0.f;
                for (int c = 0; c < C; ++c) {
                    cum += p[c];
                    if (cum >= a.model.tau * tot) { cls = c; break; }
                }
                w = min(a.model.budget_rows[cls], rows_full);
            }
        }
        if (active) w = max(w, 1);

        // ---- 4. pack scheduled windows into lane segments (one gap lane after each) ----
        // Widest first (threshold passes), rotating within a pass: a window
        // that needs many rows is never starved by narrow ones filling the
        // wavefront, and narrow windows fill what is left.
        int mybase = -1, used = 0;
        for (int pass = 0; pass < 4; ++pass) {
            const int lo = pass == 0 ? 33 : (pass == 1 ? 17 : (pass == 2 ? 9 : 1));
            const int hi = pass == 0 ? 65 : (pass == 1 ? 33 : (pass == 2 ? 17 : 9));
            for (int t = 0; t < NS; ++t) {
                const int s = (rot + t) % NS;
                const int ws = __builtin_amdgcn_readlane(w, s);
                if (ws >= lo && ws < hi && used + ws <= 64) {
                    if (lane == s) mybase = used;
                    used += ws + 1;
                }
            }
        }
        rot = (rot + 1) % NS;
        if (lane < NS) srec[lane] = SlotRec{active ? mybase : -1, w, nw, mw};
        __syncthreads();

        // ---- 5. row-lane setup: segment, row index, EQ table in step order ----
        int rs = -1, rd = 0, rw = 0, rnw = 0, rmw = 0, steps = 0;
        for (int s = 0; s < NS; ++s) {
            const SlotRec r = srec[s];
            if (r.base >= 0) {
                steps = max(steps, r.n_w + r.width - 1);
                if (lane >= r.base && lane < r.base + r.width) {
                    rs = s; rd = lane - r.base; rw = r.width; rnw = r.n_w; rmw = r.m_w;
                }
            }
        }
        steps = __builtin_amdgcn_readfirstlane(steps);
        const bool inseg = rs >= 0;
        if (inseg) {
            // table entry u holds EQ of column n_w-1-u: row d reads entry s-d at step s
            const WinPlanes o = wpl[rs];
            const uint64_t beyond = rmw >= 64 ? 0ull : (~0ull << rmw);
            uint64_t* tab = eqt + kEqPadBefore + rs * 64;
            for (int u = rd; u < rnw; u += rw) {
                const int c = rnw - 1 - u;
                const uint64_t ph = ((o.thi >> c) & 1ull) ? o.phi : ~o.phi;
                const uint64_t pl = ((o.tlo >> c) & 1ull) ? o.plo : ~o.plo;
                tab[u] = (ph & pl) | beyond;
            }
        }
        __syncthreads();

        // empty slots reserve their next queue index now; the atomic's
        // latency hides behind the DC pass
        if (!exhausted && pair < 0 && pending < 0) pending = (int64_t)atomicAdd(&a.qctl[0], 1u);

        // ---- 6. DC pass over the anti-diagonals ----
        if (!inseg) rnw = 0;
        const int col0 = inseg ? rnw - 1 + rd : -1;    // column at step 0; column at step s is col0 - s
        const int nstore = min(cap + 1, rnw);           // stored columns 0..nstore-1
        const int last_col0 = inseg ? rnw + rw - 2 : -1;  // col0 of the segment's last row
        const uint32_t cin = (inseg && rd > 0) ? 1u : 0u;
        const uint64_t zr = inseg ? z_right_column(rmw, rd) : 0ull;
        uint32_t zlo = (uint32_t)zr, zhi = (uint32_t)(zr >> 32);
        uint32_t nelo = 0, nehi = 0;
        const uint64_t segmask = inseg ? (low_bits(rw) << (lane - rd)) : 0ull;
        const uint64_t* eqp = eqt + kEqPadBefore + (inseg ? rs * 64 : 0) - rd;
        uint64_t* dp = dent + lane;
        uint64_t* dump = dent + (size_t)a.ccols * 64 + lane;
        int s = 0;
        uint64_t e0 = eqp[0], e1 = eqp[1], e2 = eqp[2], e3 = eqp[3];
        while (s < steps) {
            const uint64_t f0 = eqp[s + 4], f1 = eqp[s + 5], f2 = eqp[s + 6], f3 = eqp[s + 7];
            DC_STEP(e0, col0 - s);
            DC_STEP(e1, col0 - s - 1);
            DC_STEP(e2, col0 - s - 2);
            DC_STEP(e3, col0 - s - 3);
            s += 4;
            e0 = f0; e1 = f1; e2 = f2; e3 = f3;
            if ((s & 7) == 0) {
                // rows with col0 <= s-1 have computed column 0 and hold Z[0][d]
                const uint64_t h = __ballot(inseg && col0 <= s - 1 && (zlo & 1u));
                const bool segdone = !inseg || (h & segmask) != 0 || last_col0 <= s - 1;
                if (__ballot(!segdone) == 0) break;
            }
        }
        const uint64_t hits = __ballot(inseg && col0 <= s - 1 && (zlo & 1u));
        c_lane_steps += (unsigned long long)min(used, 64) * s;
        c_rounds += 1;
        __syncthreads();

        // poll reserved queue entries; read at the next round's start
        if (!exhausted && pair < 0 && pending >= 0 && polled == 0) {
            if (pending >= a.qcap) exhausted = true;
            else polled = __hip_atomic_load(&a.ring[pending], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }

        // ---- 7. decide d_w, trace back, advance (slot lanes) ----
        if (active && mybase >= 0) {
            const uint64_t seg = (hits >> mybase) & low_bits(w);
            int dw = -1;
            bool not_aligned = false;
            c_rows += w;
            if (seg) {
                dw = __builtin_ctzll(seg);
            } else if (w >= rows_full) {
                if (kw == mw) dw = mw; else not_aligned = true;
            } else {
                next_w = min(2 * w + 1, rows_full);
                c_fallback += 1;
            }
            if (dw >= 0) {
                next_w = 0;
                c_windows += 1;
                c_ops += (unsigned long long)(dw + 1) + 2ull * nw + 7ull * nw * dw;
                int ti = 0, tj = 0, td = dw, wed = 0;
                const int jlim = min(mw, cap);
                const uint64_t* drow = dent + mybase - 1;   // row r of this window: drow[c * 64 + r + 1]
                for (;;) {
                    // match run at (ti, tj); characters past n_w never match
                    const uint64_t x = ((wp.thi >> ti) ^ (wp.phi >> tj)) | ((wp.tlo >> ti) ^ (wp.plo >> tj));
                    int L = x ? (int)__builtin_ctzll(x) : 64;
                    L = min(L, min(nw - ti, min(jlim - tj, cap - ti)));
                    if (L > 0) emit_run(0, L, cur_op, cur_len, nruns, a.runs, roff, rcap);
                    ti += L;
                    tj += L;
                    if (tj >= jlim || ti >= cap) break;
                    // edit step: row td-1 at columns ti and ti+1 (one ds_read2; ti+1 <= cap is stored)
                    const uint64_t* p = drow + ti * 64 + max(td, 1);   // td >= 1 on a valid path
                    const uint64_t v0 = p[0], v1 = p[64];
                    const uint64_t rc = z_right_column(mw, td - 1);
                    const uint64_t za = ti < nw ? v0 : rc;        // Z[ti][td-1]
                    const uint64_t zb = ti + 1 < nw ? v1 : rc;    // Z[ti+1][td-1]
                    const int has_t = ti < nw;
                    const int sb = has_t & zbit(zb, tj + 1);
                    const int ib = zbit(za, tj + 1);
                    const int db = has_t & zbit(zb, tj);
                    bad_state |= (td <= 0) | !(sb | ib | db);
                    const int op = sb ? 1 : (ib ? 2 : 3);
                    ti += op != 2;
                    tj += op != 3;
                    td -= 1;
                    wed += 1;
                    emit_run(op, 1, cur_op, cur_len, nruns, a.runs, roff, rcap);
                    if (tj >= jlim || ti >= cap || bad_state) break;
                }
                edits += wed;
                p0 += tj;
                t0 += ti;
                if (bad_state || p0 >= m) {
                    if (cur_len > 0) {
                        if (nruns < rcap) a.runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                        ++nruns;
                    }
                    const bool ok = !bad_state && nruns <= rcap;
                    if (!ok) c_err += 1;
                    a.edits[pair] = ok ? edits : -1;
                    a.text_end[pair] = ok ? t0 : -1;
                    a.status[pair] = ok ? 0 : 3;
                    a.n_runs[pair] = ok ? nruns : 0;
                    pair = -1;
                    atomicAdd(&a.qctl[2], 1u);
                } else if (a.yield_chars > 0 && p0 - p0_take >= a.yield_chars) {
                    // hand the pair back to the queue so that the pairs of a
                    // wavefront rotate and the wavefronts stay balanced
                    const uint32_t t = atomicAdd(&a.qctl[1], 1u);
                    if ((int64_t)t < a.qcap) {
                        int32_t* st = a.pstate + 8 * (int64_t)pair;
                        st[0] = p0; st[1] = t0; st[2] = edits; st[3] = nruns; st[4] = cur_op; st[5] = cur_len;
                        st[6] = next_w; st[7] = 0;
                        __hip_atomic_store(&a.ring[t], pair + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        pair = -1;
                        c_yield += 1;
                    }
                }
            } else if (not_aligned) {
                c_windows += 1;
                c_ops += (unsigned long long)(kw + 1) + 2ull * nw + 7ull * nw * kw;
                a.edits[pair] = -1;
                a.text_end[pair] = -1;
                a.status[pair] = 1;
                a.n_runs[pair] = 0;
                pair = -1;
                atomicAdd(&a.qctl[2], 1u);
            }
        }
        __syncthreads();
    }

    // ---- counters ----
    if (lane < NS) {
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

#undef DC_STEP

}  // namespace

size_t align_lds_bytes(int ccols, int ns) {
    return (size_t)(ccols + 1) * 64 * 8 + (size_t)(kEqPadBefore + ns * 64 + kEqPadAfter) * 8 +
           (size_t)ns * sizeof(WinPlanes) + (size_t)ns * sizeof(SlotRec) + 2 * (size_t)ns * sizeof(PlaneBuf);
}

int align_max_blocks_per_cu(size_t lds_bytes, bool learned) {
    int nb = 0;
    hipError_t e = learned ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, align_kernel<true>, 64, lds_bytes)
                           : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, align_kernel<false>, 64, lds_bytes);
    if (e != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_align(const AlignArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
    if (a.mode == 1)
        hipLaunchKernelGGL(align_kernel<true>, dim3(grid), dim3(64), lds_bytes, s, a);
    else
        hipLaunchKernelGGL(align_kernel<false>, dim3(grid), dim3(64), lds_bytes, s, a);
    return hipGetLastError();
}
