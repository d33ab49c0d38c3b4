// Windowed GenASM-DC + GenASM-TB with one lane per pair: the row-wise
// mapping of the paper's CPU implementation (Section 2.5), on a GPU lane.
//
//   * Each lane takes pairs from the global queue and aligns them window by
//     window on its own; the 64 lanes of a wavefront hold 64 pairs.
//   * Row-wise DC (Algorithm 1): row d is computed for all 64 text columns
//     inside the lane, from column 63 down to column 0 (the M term needs the
//     right neighbour's row d), over the lane's row d-1 held in 128 VGPRs and
//     updated in place.  Columns at or beyond n_w have an empty match mask and
//     a right neighbour equal to the initial column, so they carry the
//     initial column and short windows need no special case.
//   * Early termination (Section 2.4.3): the window stops at the first row
//     whose column-0 entry has the msb of R clear; with rows computed in
//     order nothing above d_w is computed.
//   * DENT extended to rows (supplementary Section 1): traceback reads at most
//     W-O rows below d_w, so only the latest W-O+1 rows are kept, as a ring of
//     slots in global memory, [slot][column 0..W-O][lane] (entries, not edges:
//     Section 2.4.1), the 64 lanes' entries of one slot and column contiguous.
//   * Traceback as in the other kernels: match runs skipped with the 2-bit
//     planes, each edit reading row d-1 at columns i and i+1.
//   * A wavefront runs until all its lanes' pairs are done; lanes wait for the
//     slowest window of the wavefront at every row loop (lockstep), which is
//     the cost of this mapping on a SIMD machine.
#include "predictor.h"

namespace {

__device__ __forceinline__ uint64_t z_init64(int mw, int d) {
    // Z of the initial column (i = n_w): bit j set iff m_w - j <= d
    const int s = mw - d;
    return s <= 0 ? ~0ull : (s >= 64 ? 0ull : (~0ull << s));
}

__global__ __launch_bounds__(64) void lane_kernel(const AlignArgs a) {
    const int lane = threadIdx.x;
    const int cap = a.cap;
    const int ncols = cap + 1;                 // stored columns 0..W-O
    const int nring = cap + 1;                 // stored rows: the latest W-O+1
    uint64_t* const ringbase = a.dent + (size_t)blockIdx.x * (size_t)nring * ncols * 64;
    auto slot_at = [&](int row, int col) -> uint64_t* {
        return ringbase + ((size_t)(row % nring) * ncols + col) * 64 + lane;
    };
    // lane state
    int pair = -1, p0 = 0, t0 = 0, m = 0, n = 0, edits = 0, nruns = 0, cur_op = 0, cur_len = 0;
    int64_t roff = 0, rcap = 0;
    bool exhausted = false;
    unsigned long long c_windows = 0, c_ops = 0, c_rows = 0, c_err = 0, c_steps = 0, c_rounds = 0;

    auto emit = [&](int op, int len) {
        const bool same = cur_op == op;
        if (len > 0 && !same && cur_len > 0) {
            if (nruns < rcap) a.runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
            ++nruns;
        }
        if (len > 0) {
            cur_len = same ? cur_len + len : len;
            cur_op = op;
        }
    };
    auto finish = [&](bool bad) {
        if (cur_len > 0) {
            if (nruns < rcap) a.runs[roff + nruns] = ((uint32_t)cur_len << 2) | (uint32_t)cur_op;
            ++nruns;
        }
        const bool ok = !bad && nruns <= rcap;
        if (!ok) c_err += 1;
        a.edits[pair] = ok ? edits : -1;
        a.text_end[pair] = ok ? t0 : -1;
        a.status[pair] = ok ? 0 : 3;
        a.n_runs[pair] = ok ? nruns : 0;
        pair = -1;
        atomicAdd(&a.qctl[2], 1u);
    };

    for (;;) {
        // ---- take a pair (lanes without one) ----
        while (!exhausted && pair < 0) {
            // the queue holds exactly the pairs (this kernel never yields): entries
            // from npairs on are never taken
            const uint32_t q = atomicAdd(&a.qctl[0], 1u);
            if ((int64_t)q >= a.qcap || (int64_t)q >= a.npairs) {
                exhausted = true;
                break;
            }
            const int pid = __hip_atomic_load(&a.ring[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - 1;
            if (pid < 0 || pid >= a.npairs) {   // not a pair id: nothing more to take
                exhausted = true;
                break;
            }
            const int pm = a.plen[pid], pn = a.tlen[pid];
            if (a.bad[pid] || pm == 0) {
                const bool bad = a.bad[pid] != 0;
                a.edits[pid] = bad ? -1 : 0;
                a.text_end[pid] = bad ? -1 : 0;
                a.status[pid] = bad ? 2 : 0;
                a.n_runs[pid] = 0;
                atomicAdd(&a.qctl[2], 1u);
                continue;
            }
            pair = pid;
            m = pm;
            n = pn;
            p0 = t0 = edits = nruns = cur_op = cur_len = 0;
            roff = a.runs_off[pid];
            rcap = a.runs_off[pid + 1] - roff;
        }
        if (__ballot(pair >= 0) == 0) break;
        const bool active = pair >= 0;

        // ---- the window and its match masks by text code ----
        int mw = 0, nw = 0, kw = 0, full = 0;
        uint64_t plo = 0, phi = 0, tlo = 0, thi = 0;
        if (active) {
            mw = min(a.W, m - p0);
            nw = min(a.W, n - t0);
            kw = min(a.k, mw);
            full = (kw == mw) ? mw : kw + 1;   // row m_w is implicit: D(0,0) <= m_w
            load_window(a.pplanes + a.pword[pair], p0, plo, phi);
            if (nw > 0) load_window(a.tplanes + a.tword[pair], t0, tlo, thi);
        }
        const uint64_t beyond = mw >= 64 ? 0ull : (~0ull << mw);
        // Z form: bit j of eq[c] is set when pattern[j] has code c (or j >= m_w)
        const uint64_t eq0 = (~plo & ~phi) | beyond, eq1 = (plo & ~phi) | beyond;
        const uint64_t eq2 = (~plo & phi) | beyond, eq3 = (plo & phi) | beyond;
        const uint64_t tin = nw >= 64 ? ~0ull : ((1ull << nw) - 1ull);   // text columns inside the window

        // ---- row-wise DC with early termination ----
        uint64_t row[64];
        int dw = -1;
        int d = 0;
        bool running = active;
        for (;; ++d) {
            if (__ballot(running) == 0) break;
            if (running) {
                const uint64_t zr = z_init64(mw, d);        // the initial column at row d
                uint64_t right_old = d > 0 ? z_init64(mw, d - 1) : 0ull;   // Z[i+1][d-1]
                uint64_t right_new = zr;                    // Z[i+1][d]
                const uint64_t cin = d > 0 ? (1ull << 63) : 0ull;
#pragma unroll
                for (int i = 63; i >= 0; --i) {
                    const int tl = (int)((tlo >> i) & 1ull), th = (int)((thi >> i) & 1ull);
                    const uint64_t e = ((tin >> i) & 1ull) ? (th ? (tl ? eq3 : eq2) : (tl ? eq1 : eq0)) : beyond;
                    const uint64_t old = d > 0 ? row[i] : 0ull;   // Z[i][d-1]
                    uint64_t z = ((right_new >> 1) | (1ull << 63)) & e;   // M
                    if (d > 0) z |= ((old >> 1) | cin) | ((right_old >> 1) | cin) | right_old;   // I, S, D
                    row[i] = z;
                    right_old = old;
                    right_new = z;
                }
                // keep columns 0..W-O of this row for traceback (its ring slot)
                uint64_t* const srow = ringbase + (size_t)(d % nring) * ncols * 64 + lane;
#pragma unroll
                for (int c = 0; c < 64; ++c)
                    if (c < ncols) srow[(size_t)c * 64] = row[c];
                if (row[0] & 1ull) {
                    dw = d;
                    running = false;
                } else if (d + 1 >= full) {
                    running = false;   // no hit within rows 0..k_w
                }
            }
            c_steps += 1;
        }
        c_rounds += 1;
        // every lane's ring stores are visible to its own loads below
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

        // ---- traceback, advance, output ----
        if (active) {
            int td = dw;
            if (td < 0 && kw == mw) td = mw;   // no hit in rows 0..m_w-1: distance m_w
            c_rows += (unsigned long long)(dw < 0 ? full : dw + 1);
            c_windows += 1;
            if (td < 0) {
                c_ops += (unsigned long long)(kw + 1) + 2ull * nw + 7ull * nw * kw;
                a.edits[pair] = -1;
                a.text_end[pair] = -1;
                a.status[pair] = 1;
                a.n_runs[pair] = 0;
                pair = -1;
                atomicAdd(&a.qctl[2], 1u);
            } else {
                c_ops += (unsigned long long)(td + 1) + 2ull * nw + 7ull * nw * td;
                const int jlim = min(mw, cap), ilim = min(nw, cap);
                int ti = 0, tj = 0, we = 0, bad = 0;
                for (;;) {
                    const uint64_t x = ((thi >> ti) ^ (phi >> tj)) | ((tlo >> ti) ^ (plo >> tj));
                    int L = x ? (int)__builtin_ctzll(x) : 64;
                    L = max(min(L, min(ilim - ti, jlim - tj)), 0);
                    emit(0, L);
                    ti += L;
                    tj += L;
                    if (tj >= jlim || ti >= cap) break;
                    // edit step: row td-1 at columns ti and ti+1 (ti + 1 <= W-O is stored)
                    const int r = max(td, 1) - 1;
                    const uint64_t rc = z_init64(mw, td - 1);
                    const uint64_t za = ti < nw ? *slot_at(r, ti) : rc;
                    const uint64_t zb = ti + 1 < nw ? *slot_at(r, ti + 1) : rc;
                    const int has_t = ti < nw;
                    // bits tj and tj+1 (tj <= 63 in an edit step; bit 64 is the implicit set bit)
                    const uint64_t sa = za >> (tj & 63), sz = zb >> (tj & 63);
                    const int top = tj >= 63 ? 1 : 0;
                    const int sb = has_t & (((int)(sz >> 1) & 1) | top);
                    const int ib = ((int)(sa >> 1) & 1) | top;
                    const int db = has_t & (int)(sz & 1);
                    bad |= (td <= 0) | !(sb | ib | db);
                    const int op = sb ? 1 : (ib ? 2 : 3);
                    emit(op, 1);
                    ti += op != 2;
                    tj += op != 3;
                    td -= 1;
                    we += 1;
                    if (tj >= jlim || ti >= cap || bad) break;
                }
                edits += we;
                p0 += tj;
                t0 += ti;
                if (bad || p0 >= m) finish(bad != 0);
            }
        }
        // the next window overwrites the ring: every lane's traceback reads come first
        __syncthreads();
    }

    if (c_windows) atomicAdd(&a.stats[ST_WINDOWS], c_windows);
    if (c_ops) atomicAdd(&a.stats[ST_OPS_ALG], c_ops);
    if (c_rows) atomicAdd(&a.stats[ST_ROWS], c_rows);
    if (c_err) atomicAdd(&a.stats[ST_ERRORS], c_err);
    if (lane == 0) {
        atomicAdd(&a.stats[ST_LANE_STEPS], 64ull * c_steps);
        atomicAdd(&a.stats[ST_ROUNDS], c_rounds);
    }
}

}  // namespace

size_t lane_dent_bytes(int grid, int cap) {
    return (size_t)grid * (size_t)(cap + 1) * (size_t)(cap + 1) * 64 * sizeof(uint64_t);
}

int lane_max_blocks_per_cu() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_kernel, 64, 0) != hipSuccess) return 1;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_align_lane(const AlignArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(lane_kernel, dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}
