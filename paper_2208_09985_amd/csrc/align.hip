// Fused, persistent windowed GenASM-DC + GenASM-TB kernel for gfx950.
//
// Mapping (one wavefront = one workgroup, 64 lanes):
//   * Lanes are error rows.  A window that computes w rows occupies a
//     contiguous segment of w lanes (lane base+d = row d); several windows of
//     different pairs share a wavefront when their segments fit in 64 lanes.
//   * Rows advance over the text columns on an anti-diagonal schedule: at
//     step s, row d works on column i = n_w-1-s+d.  Entries on one NW-SE
//     diagonal are independent (Section 2.2.1, intra-task parallelism).
//     Row d needs R[i][d-1] and R[i+1][d-1] from row d-1; both come from the
//     neighbouring lane through one DPP wave_shr:1 per 32-bit half.
//   * Each lane holds one 64-bit bitvector (two VGPRs).  The kernel keeps the
//     complement Z = ~R in LSB-first order (bit j = pattern position j), so
//     the update of Algorithm 1 becomes
//         Z[i][d] = ((Z[i][d-1] | Z[i+1][d-1]) >> 1 | top)   -- ~I, ~S
//                 | Z[i+1][d-1]                              -- ~D
//                 | ((Z[i+1][d] >> 1 | top) & EQ[text[i]])   -- ~M
//     with EQ = ~PM and `top` the bit shifted in where R shifts in a 0.
//     A 0 in the msb of R[0][d] is bit 0 of Z[0][d] set.
//   * Only entries that traceback can read are stored (Section 2.4.1: the
//     entries, not the edges; Section 2.4.2: columns 0..W-O only).  They live
//     in LDS as dent[column][lane], 8 bytes each.
//   * Early termination (Section 2.4.3): the first row whose column-0 entry
//     has the msb cleared is d_w; a wavefront ballot on that condition ends
//     the pass once every window in it has found its d_w.
//   * Traceback runs in the slot lane of each window (lanes 0..ns-1).  Along
//     a tight path with text[i] == pattern[j] the M term always holds (the
//     suffix distance never increases along a diagonal of matches), so match
//     runs are skipped with one XOR of the 2-bit planes and a trailing-zero
//     count; only edit steps read LDS, and only row d-1.
//   * Pairs are taken from a global atomic queue (the paper's global queue of
//     pairs, Section 2.5) until it is empty; every wavefront then exits.
//   * Row budgets: plain mode computes rows 0..k_w of every window.  The
//     learned and fixed modes first compute fewer rows; a window that finds
//     no d_w within them is recomputed with all rows in a later round.  Rows
//     <= d never depend on rows > d, so the result is bit-identical.
#include "predictor.h"

namespace {

constexpr uint32_t kDppWaveShr1 = 0x138;

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

struct SlotRec {       // LDS record of a window scheduled in the current round
    int32_t base;      // first lane of its segment, -1 if not scheduled
    int32_t width;     // rows (lanes) computed
    int32_t n_w, m_w;
};

__global__ __launch_bounds__(64) void align_kernel(const AlignArgs a) {
    extern __shared__ uint64_t smem[];
    const int lane = threadIdx.x;
    const int NS = a.ns;
    uint64_t* dent = smem;                                  // [ccols][64]
    uint64_t* eqt = dent + (size_t)a.ccols * 64;            // [NS][64]
    WinPlanes* wpl = (WinPlanes*)(eqt + (size_t)NS * 64);   // [NS]
    SlotRec* srec = (SlotRec*)(wpl + NS);                   // [NS]

    const int cap = a.cap;
    const bool learned = a.mode == 1;
    MlpRegs mlp;
    if (learned) mlp_load_regs(mlp, a.model.w1, a.model.b1, a.model.w2, a.model.b2, a.model.H, a.model.C, lane);

    // ---- slot-lane state (meaningful in lanes < NS) ----
    int pair = -1, p0 = 0, t0 = 0, m = 0, n = 0, edits = 0, nruns = 0, cur_op = 0, cur_len = 0;
    int fallback = 0, bad_state = 0;
    int64_t roff = 0, rcap = 0;
    bool exhausted = lane >= NS;
    unsigned long long c_windows = 0, c_ops = 0, c_fallback = 0, c_rows = 0, c_err = 0;
    unsigned long long c_lane_steps = 0, c_rounds = 0;
    int rot = 0;

    for (;;) {
        // ---- 1. refill empty slots from the queue ----
        if (!exhausted && pair < 0) {
            for (;;) {
                const uint32_t q = atomicAdd(a.queue, 1u);
                if (q >= (uint32_t)a.npairs) { exhausted = true; break; }
                const int pid = a.order[q];
                const int pm = a.plen[pid], pn = a.tlen[pid];
                const int64_t ro = a.runs_off[pid];
                if (a.bad[pid]) {
                    a.edits[pid] = -1; a.text_end[pid] = -1; a.status[pid] = 2; a.n_runs[pid] = 0;
                    continue;
                }
                if (pm == 0) {
                    a.edits[pid] = 0; a.text_end[pid] = 0; a.status[pid] = 0; a.n_runs[pid] = 0;
                    continue;
                }
                pair = pid; m = pm; n = pn; p0 = 0; t0 = 0; edits = 0; nruns = 0; cur_op = 0; cur_len = 0;
                fallback = 0; bad_state = 0; roff = ro; rcap = a.runs_off[pid + 1] - ro;
                break;
            }
        }
        const bool active = pair >= 0;
        if (__ballot(active) == 0) break;

        // ---- 2. window geometry of each active slot ----
        int mw = 0, nw = 0, kw = 0, rows_full = 0, w = 0;
        WinPlanes wp{0, 0, 0, 0, 0, 0};
        if (active) {
            mw = min(a.W, m - p0);
            nw = min(a.W, n - t0);
            kw = min(a.k, mw);
            rows_full = (kw == mw) ? mw : kw + 1;   // row m_w is implicit: D(0,0) <= m_w
            load_window(a.pplanes + a.pword[pair], p0, wp.plo, wp.phi);
            if (nw > 0) load_window(a.tplanes + a.tword[pair], t0, wp.tlo, wp.thi);
            wp.m_w = mw;
            wp.n_w = nw;
            wpl[lane] = wp;
            w = rows_full;
            if (!fallback && a.mode == 2) w = min(a.fixed_rows, rows_full);
        }

        // ---- 3. learned row budget: features -> MLP (MFMA) -> smallest confident budget ----
        if (learned) {
            __syncthreads();
            const int s = lane & 15, g = lane >> 4;
            half4_t x4 = {0, 0, 0, 0};
            if (s < NS) {
                const WinPlanes o = wpl[s];
                for (int e = 0; e < 4; ++e) x4[e] = feature_to_input(window_feature(o, 4 * g + e));
            }
            half4_t hid[4];
            const float4_t logit = mlp_tile_forward(mlp, x4, hid);
            if (active && !fallback) {
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

        // ---- 4. pack scheduled windows into lane segments ----
        int mybase = -1, used = 0;
        for (int t = 0; t < NS; ++t) {
            const int s = (rot + t) % NS;
            const int ws = __builtin_amdgcn_readlane(w, s);
            if (ws > 0 && used + ws <= 64) {
                if (lane == s) mybase = used;
                used += ws;
            }
        }
        rot = (rot + 1) % NS;
        if (lane < NS) srec[lane] = SlotRec{active ? mybase : -1, w, nw, mw};
        __syncthreads();

        // ---- 5. row-lane setup: segment, row index, EQ table ----
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
        if (rs >= 0) {
            const WinPlanes o = wpl[rs];
            const uint64_t beyond = rmw >= 64 ? 0ull : (~0ull << rmw);
            for (int c = rd; c < rnw; c += rw) {
                const uint64_t ph = ((o.thi >> c) & 1ull) ? o.phi : ~o.phi;
                const uint64_t pl = ((o.tlo >> c) & 1ull) ? o.plo : ~o.plo;
                eqt[rs * 64 + c] = (ph & pl) | beyond;
            }
        }
        __syncthreads();

        // ---- 6. DC pass over the anti-diagonals ----
        const bool inseg = rs >= 0;
        const uint32_t notstart = (inseg && rd > 0) ? 0xFFFFFFFFu : 0u;
        const uint32_t cin = (inseg && rd > 0) ? 1u : 0u;
        const uint64_t zr = inseg ? z_right_column(rmw, rd) : 0ull;
        uint32_t zlo = (uint32_t)zr, zhi = (uint32_t)(zr >> 32);
        uint32_t nelo = 0, nehi = 0;
        const uint64_t segmask = inseg ? (low_bits(rw) << (lane - rd)) : 0ull;
        const uint64_t* eqrow = eqt + (inseg ? rs : 0) * 64;
        int col = rnw - 1 + rd;
        uint64_t hits = 0;
        int s = 0;
        for (; s < steps; ++s, --col) {
            const uint32_t nlo = from_lower_lane(zlo) & notstart;
            const uint32_t nhi = from_lower_lane(zhi) & notstart;
            bool hit = false;
            if ((unsigned)col < (unsigned)rnw) {
                const uint64_t e = eqrow[col];
                const uint32_t tl = nlo | nelo, th = nhi | nehi;
                const uint32_t al = __builtin_amdgcn_alignbit(th, tl, 1);
                const uint32_t ah = __builtin_amdgcn_alignbit(cin, th, 1);
                const uint32_t bl = __builtin_amdgcn_alignbit(zhi, zlo, 1);
                const uint32_t bh = __builtin_amdgcn_alignbit(1u, zhi, 1);
                zlo = (bl & (uint32_t)e) | al | nelo;
                zhi = (bh & (uint32_t)(e >> 32)) | ah | nehi;
                if (col <= cap) dent[col * 64 + lane] = ((uint64_t)zhi << 32) | zlo;
                hit = (col == 0) && (zlo & 1u);
            }
            nelo = nlo;
            nehi = nhi;
            hits |= __ballot(hit);
            if ((s & 3) == 3) {
                const bool done = !inseg || (hits & segmask) != 0 || s >= rnw + rw - 2;
                if (__ballot(!done) == 0) { ++s; break; }
            }
        }
        c_lane_steps += (unsigned long long)used * s;
        c_rounds += 1;
        __syncthreads();

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
                fallback = 1;
                c_fallback += 1;
            }
            if (dw >= 0) {
                fallback = 0;
                c_windows += 1;
                c_ops += (unsigned long long)(dw + 1) + 2ull * nw + 7ull * nw * dw;
                int ti = 0, tj = 0, td = dw, wed = 0;
                const int jlim = min(mw, cap);
                while (tj < jlim && ti < cap) {
                    if (ti < nw) {
                        const uint64_t x = ((wp.thi >> ti) ^ (wp.phi >> tj)) | ((wp.tlo >> ti) ^ (wp.plo >> tj));
                        int L = x ? __builtin_ctzll(x) : 64;
                        L = min(L, min(nw - ti, min(jlim - tj, cap - ti)));
                        if (L > 0) {
                            if (cur_len > 0 && cur_op == 0) cur_len += L;
                            else {
                                if (cur_len > 0) {
                                    if (nruns < rcap) a.runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                                    ++nruns;
                                }
                                cur_op = 0; cur_len = L;
                            }
                            ti += L; tj += L;
                            continue;
                        }
                    }
                    if (td <= 0) { bad_state = 1; break; }
                    const int r = mybase + td - 1;
                    const uint64_t rc = z_right_column(mw, td - 1);
                    const uint64_t za = (ti < nw) ? dent[ti * 64 + r] : rc;            // Z[ti][td-1]
                    const uint64_t zb = (ti + 1 < nw) ? dent[(ti + 1) * 64 + r] : rc;  // Z[ti+1][td-1]
                    int op;
                    if (ti < nw && zbit(zb, tj + 1)) { op = 1; ++ti; ++tj; }
                    else if (zbit(za, tj + 1)) { op = 2; ++tj; }
                    else if (ti < nw && zbit(zb, tj)) { op = 3; ++ti; }
                    else { bad_state = 1; break; }
                    --td; ++wed;
                    if (cur_len > 0 && cur_op == op) cur_len += 1;
                    else {
                        if (cur_len > 0) {
                            if (nruns < rcap) a.runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
                            ++nruns;
                        }
                        cur_op = op; cur_len = 1;
                    }
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
                }
            } else if (not_aligned) {
                c_windows += 1;
                c_ops += (unsigned long long)(kw + 1) + 2ull * nw + 7ull * nw * kw;
                a.edits[pair] = -1;
                a.text_end[pair] = -1;
                a.status[pair] = 1;
                a.n_runs[pair] = 0;
                pair = -1;
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
    }
    if (lane == 0) {
        atomicAdd(&a.stats[ST_LANE_STEPS], c_lane_steps);
        atomicAdd(&a.stats[ST_ROUNDS], c_rounds);
    }
}

}  // namespace

size_t align_lds_bytes(int ccols, int ns) {
    return (size_t)ccols * 64 * 8 + (size_t)ns * 64 * 8 + (size_t)ns * sizeof(WinPlanes) +
           (size_t)ns * sizeof(SlotRec);
}

int align_max_blocks_per_cu(size_t lds_bytes) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, align_kernel, 64, lds_bytes) != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_align(const AlignArgs& a, int grid, size_t lds_bytes, hipStream_t s) {
    hipLaunchKernelGGL(align_kernel, dim3(grid), dim3(64), lds_bytes, s, a);
    return hipGetLastError();
}
