// Host runtime behind include/rcpsp.h: instance validation and packing,
// search plans (device state + captured HIP graph), result read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "rcpsp.h"
#include "rcpsp_internal.h"
#include "rcpsp_launch.h"
#include "rcpsp_runtime.h"

using namespace rcpsp;

namespace rcpsp {

thread_local std::string g_err;

rcpsp_status fail(rcpsp_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

int potential_moves(int n, int delta) {
    const int Lp = n - 2;
    if (Lp < 2 || delta < 1) return 0;
    const int dd = std::min(delta, Lp - 1);
    return dd * Lp - dd * (dd + 1) / 2;
}

}  // namespace rcpsp

namespace {

int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

struct Blob {
    std::vector<uint32_t> w;
    int add16(const std::vector<int> &v) {
        const int off = (int)w.size();
        w.resize(w.size() + (v.size() + 1) / 2, 0u);
        for (size_t i = 0; i < v.size(); ++i)
            w[off + i / 2] |= (uint32_t)(v[i] & 0xffff) << (16 * (i & 1));
        return off;
    }
    int add32(const std::vector<uint32_t> &v) {
        const int off = (int)w.size();
        w.insert(w.end(), v.begin(), v.end());
        return off;
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// instances

extern "C" const char *rcpsp_last_error(void) { return g_err.c_str(); }
extern "C" const char *rcpsp_version(void) { return "rcpsp-mi355x 0.1 (gfx950)"; }
extern "C" int32_t rcpsp_potential_moves(int32_t n, int32_t swap_range) { return potential_moves(n, swap_range); }

static rcpsp_status validate_and_derive(rcpsp_instance *I, int32_t n, int32_t m, const int32_t *duration,
                                        const int32_t *capacity, const int32_t *request,
                                        const int32_t *succ_off, const int32_t *succ) {
    if (!duration || !capacity || !request || !succ_off) return fail(RCPSP_E_ARG, "null input array");
    if (n < 3) return fail(RCPSP_E_ARG, "N must be at least 3 (two dummies and one activity), got %d", n);
    if (n > kMaxN) return fail(RCPSP_E_TOO_LARGE, "N=%d exceeds %d", n, kMaxN);
    if (m < 1 || m > kMaxM) return fail(m < 1 ? RCPSP_E_ARG : RCPSP_E_TOO_LARGE, "M=%d outside 1..%d", m, kMaxM);
    I->n = n;
    I->m = m;
    I->d.assign(duration, duration + n);
    I->R.assign(capacity, capacity + m);
    I->r.assign(request, request + (size_t)n * m);
    long long H = 0;
    for (int i = 0; i < n; ++i) {
        if (I->d[i] < 0) return fail(RCPSP_E_ARG, "negative duration d_%d", i);
        H += I->d[i];
        I->dmax = std::max(I->dmax, I->d[i]);
    }
    if (I->d[0] != 0 || I->d[n - 1] != 0) return fail(RCPSP_E_DUMMY, "dummy activities must have zero duration");
    if (H > kMaxHorizon) return fail(RCPSP_E_TOO_LARGE, "sum of durations %lld exceeds %d", H, kMaxHorizon);
    I->H = (int)H;
    for (int k = 0; k < m; ++k) {
        if (I->R[k] < 0) return fail(RCPSP_E_REQUEST, "negative capacity R_%d", k);
        if (I->R[k] > kMaxHorizon) return fail(RCPSP_E_TOO_LARGE, "capacity R_%d=%d too large", k, I->R[k]);
    }
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < m; ++k) {
            const int rik = I->r[(size_t)i * m + k];
            if (rik < 0 || rik > I->R[k]) return fail(RCPSP_E_REQUEST, "request r_%d,%d=%d outside 0..R_%d=%d", i, k, rik, k, I->R[k]);
            if ((i == 0 || i == n - 1) && rik != 0) return fail(RCPSP_E_DUMMY, "dummy activity %d has a request", i);
        }
    if (succ_off[0] != 0) return fail(RCPSP_E_ARG, "succ_off[0] must be 0");
    for (int i = 0; i < n; ++i)
        if (succ_off[i + 1] < succ_off[i]) return fail(RCPSP_E_ARG, "succ_off not non-decreasing at %d", i);
    const int E = succ_off[n];
    if (E > 0 && !succ) return fail(RCPSP_E_ARG, "null successor array");
    if (E > 65535) return fail(RCPSP_E_TOO_LARGE, "%d arcs exceed 65535", E);
    I->n_arcs = E;
    I->succ_off.assign(succ_off, succ_off + n + 1);
    I->succ.assign(succ, succ + E);
    std::vector<char> seen((size_t)n * n, 0);
    std::vector<int> indeg(n, 0), outdeg(n, 0);
    for (int i = 0; i < n; ++i) {
        for (int e = succ_off[i]; e < succ_off[i + 1]; ++e) {
            const int j = succ[e];
            if (j < 0 || j >= n) return fail(RCPSP_E_ARG, "successor id %d of %d out of range", j, i);
            if (j == i) return fail(RCPSP_E_CYCLE, "self loop on %d", i);
            if (seen[(size_t)i * n + j]) return fail(RCPSP_E_ARG, "duplicate arc %d->%d", i, j);
            seen[(size_t)i * n + j] = 1;
            indeg[j]++;
            outdeg[i]++;
        }
    }
    if (indeg[0] != 0) return fail(RCPSP_E_DUMMY, "activity 0 must have no predecessor");
    if (outdeg[n - 1] != 0) return fail(RCPSP_E_DUMMY, "activity N-1 must have no successor");
    for (int i = 1; i < n; ++i)
        if (indeg[i] == 0) return fail(RCPSP_E_DUMMY, "activity %d has no predecessor (arc 0->%d missing)", i, i);
    for (int i = 0; i < n - 1; ++i)
        if (outdeg[i] == 0) return fail(RCPSP_E_DUMMY, "activity %d has no successor (arc %d->N-1 missing)", i, i);
    // topological order (Kahn) -> acyclicity, critical path, levels
    std::vector<int> topo, deg = indeg;
    topo.reserve(n);
    for (int i = 0; i < n; ++i)
        if (deg[i] == 0) topo.push_back(i);
    for (size_t h = 0; h < topo.size(); ++h) {
        const int i = topo[h];
        for (int e = succ_off[i]; e < succ_off[i + 1]; ++e)
            if (--deg[succ[e]] == 0) topo.push_back(succ[e]);
    }
    if ((int)topo.size() != n) return fail(RCPSP_E_CYCLE, "precedence graph has a cycle");
    // predecessors, ascending id
    I->pred_off.assign(n + 1, 0);
    for (int j = 0; j < n; ++j) I->pred_off[j + 1] = I->pred_off[j] + indeg[j];
    I->pred.assign(E, 0);
    {
        std::vector<int> fill(I->pred_off.begin(), I->pred_off.end() - 1);
        for (int i = 0; i < n; ++i)
            for (int e = succ_off[i]; e < succ_off[i + 1]; ++e) I->pred[fill[succ[e]]++] = i;
    }
    // critical path: longest path with arc (i,j) weighted d_i (Section 2)
    std::vector<int> est(n, 0), level(n, 0);
    for (int i : topo)
        for (int e = succ_off[i]; e < succ_off[i + 1]; ++e) {
            const int j = succ[e];
            est[j] = std::max(est[j], est[i] + I->d[i]);
            level[j] = std::max(level[j], level[i] + 1);
        }
    I->cp = est[n - 1];
    // pack
    InstDesc &D = I->desc;
    D = InstDesc{};
    D.n = n;
    D.m = m;
    D.n_arcs = E;
    D.horizon = I->H;
    D.cp = I->cp;
    int rmax_cap = 0, rq_max = 1, sum_r = 0, min_cap = INT_MAX;
    for (int k = 0; k < m; ++k) {
        rmax_cap = std::max(rmax_cap, I->R[k]);
        min_cap = std::min(min_cap, I->R[k]);
        D.R[k] = I->R[k];
        D.cbase[k] = sum_r;
        sum_r += I->R[k];
    }
    for (int v : I->r) rq_max = std::max(rq_max, v);
    D.sum_r = sum_r;
    D.copy_p = std::max(2, next_pow2(rq_max));
    D.fbits = rmax_cap <= 127 ? 8 : 16;
    const int fpw = 32 / D.fbits;
    int nw = (m + fpw - 1) / fpw;
    if (nw == 3) nw = 4;
    D.nw = nw <= kMaxNW ? nw : 0;   // 0: time-indexed decoding unsupported
    const int nwp = std::max(D.nw, 1);
    for (int w = 0; w < nwp && D.nw; ++w) {
        uint32_t g = 0, f = 0;
        for (int fi = 0; fi < fpw; ++fi) {
            const int sh = fi * D.fbits;
            g |= 1u << (sh + D.fbits - 1);
            const int k = w * fpw + fi;
            if (k < m) f |= (uint32_t)I->R[k] << sh;
        }
        D.guard[w] = g;
        D.full[w] = f | g;   // stored units keep the guard bits set
    }
    Blob bl;
    std::vector<int> v16;
    v16.assign(I->d.begin(), I->d.end());
    D.off_dur = bl.add16(v16);
    v16.assign(I->pred_off.begin(), I->pred_off.end());
    D.off_predoff = bl.add16(v16);
    v16.assign(I->pred.begin(), I->pred.end());
    if (v16.empty()) v16.push_back(0);
    D.off_pred = bl.add16(v16);
    v16.assign(I->succ_off.begin(), I->succ_off.end());
    D.off_succoff = bl.add16(v16);
    v16.assign(I->succ.begin(), I->succ.end());
    if (v16.empty()) v16.push_back(0);
    D.off_succ = bl.add16(v16);
    {
        std::vector<uint32_t> rq((size_t)n * nwp, 0u);
        if (D.nw)
            for (int i = 0; i < n; ++i)
                for (int k = 0; k < m; ++k)
                    rq[(size_t)i * nwp + k / fpw] |= (uint32_t)I->r[(size_t)i * m + k] << ((k % fpw) * D.fbits);
        D.off_rq = bl.add32(rq);
    }
    v16.assign(I->r.begin(), I->r.end());
    D.off_reqk = bl.add16(v16);
    // level order (Section 4.1): levels ascending, ids ascending inside a level
    int lmax = 0;
    for (int i = 0; i < n; ++i) lmax = std::max(lmax, level[i]);
    std::vector<int> base, lvl_off;
    for (int l = 0; l <= lmax; ++l) {
        lvl_off.push_back((int)base.size());
        for (int i = 0; i < n; ++i)
            if (level[i] == l) base.push_back(i);
    }
    lvl_off.push_back((int)base.size());
    D.n_levels = lmax + 1;
    D.off_base = bl.add16(base);
    D.off_lvl = bl.add16(lvl_off);
    {
        // per resource: (R_k, first entry of c_k) as dword pairs
        std::vector<uint32_t> res(2 * (size_t)m);
        for (int k = 0; k < m; ++k) {
            res[2 * k] = (uint32_t)I->R[k];
            res[2 * k + 1] = (uint32_t)D.cbase[k];
        }
        D.off_res = bl.add32(res);
    }
    D.blob_dwords = (int)bl.w.size();
    HIP_TRY(hipGetDevice(&I->device));
    HIP_TRY(hipMalloc(&I->d_blob, bl.w.size() * sizeof(uint32_t)));
    HIP_TRY(hipMemcpy(I->d_blob, bl.w.data(), bl.w.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    D.blob = I->d_blob;
    // attributes (Table tab:attr)
    rcpsp_info &f = I->info;
    f.n = n;
    f.m = m;
    f.n_arcs = E;
    f.horizon = I->H;
    f.critical_path = I->cp;
    f.min_capacity = min_cap;
    f.max_capacity = rmax_cap;
    f.sum_capacity = sum_r;
    f.field_bits = D.fbits;
    f.avg_capacity_x1000 = (int)(1000ll * sum_r / m);
    f.avg_duration_x1000 = (int)(1000ll * I->H / n);
    f.branch_factor_x1000 = (int)(1000ll * E / n);
    return RCPSP_OK;
}

// Default decoder when none is requested: the capacity-indexed arrays cost
// about R_k/2 loop steps per request, the time-indexed profile about one
// packed slot per time unit (Section 5.4: capacity-indexed pays off for long
// schedules with small capacities).
static int auto_eval(const rcpsp_instance *I) {
    if (I->desc.nw == 0) return kEvalCapacity;
    long long ci = 0;
    for (int i = 0; i < I->n; ++i)
        for (int k = 0; k < I->m; ++k)
            if (I->r[(size_t)i * I->m + k] > 0) ci += I->R[k] / 2 + 1;
    const long long ti = (long long)I->desc.nw * I->H;
    return ti <= ci ? kEvalTime : kEvalCapacity;
}

extern "C" rcpsp_status rcpsp_create_instance(int32_t n, int32_t m, const int32_t *duration,
                                              const int32_t *capacity, const int32_t *request,
                                              const int32_t *succ_off, const int32_t *succ, rcpsp_eval eval,
                                              rcpsp_instance **out) {
    if (!out) return fail(RCPSP_E_ARG, "null output pointer");
    *out = nullptr;
    if (eval < RCPSP_EVAL_AUTO || eval > RCPSP_EVAL_CAPACITY) return fail(RCPSP_E_ARG, "unknown decoder %d", (int)eval);
    rcpsp_instance *I = new (std::nothrow) rcpsp_instance();
    if (!I) return fail(RCPSP_E_NOMEM, "out of host memory");
    rcpsp_status st = validate_and_derive(I, n, m, duration, capacity, request, succ_off, succ);
    if (st != RCPSP_OK) {
        if (I->d_blob) (void)hipFree(I->d_blob);
        delete I;
        return st;
    }
    if (eval == RCPSP_EVAL_TIME && I->desc.nw == 0) {
        (void)hipFree(I->d_blob);
        delete I;
        return fail(RCPSP_E_TOO_LARGE, "time-indexed profile needs more than %d dwords per time unit", kMaxNW);
    }
    I->eval = eval == RCPSP_EVAL_AUTO ? auto_eval(I) : (int)eval;
    I->info.eval = I->eval;
    *out = I;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_instance_info(const rcpsp_instance *inst, rcpsp_info *out) {
    if (!inst || !out) return fail(RCPSP_E_ARG, "null pointer");
    *out = inst->info;
    return RCPSP_OK;
}

extern "C" void rcpsp_destroy_instance(rcpsp_instance *inst) {
    if (!inst) return;
    if (inst->d_blob) (void)hipFree(inst->d_blob);
    delete inst;
}

// ---------------------------------------------------------------------------
// LDS layout

// G = 1: one candidate per lane, lane-interleaved state; G = 2 (time-indexed):
// the same with 8-bit finish times (lane profiles of at most 255 units);
// G = 16 (time-indexed) and G = 8 (capacity-indexed, a lane per resource):
// one candidate per G lanes, contiguous state per candidate.
static Layout make_layout(const InstDesc &D, int T, int tcw, int tl, int pmax, int L, int dec, int G = 1) {
    Layout Ly{};
    const int N2h = n2(D.n) / 2;
    const int F0 = (D.n + 1) / 2;
    int o = 0;
    Ly.blob = o; o += D.blob_dwords;
    Ly.W = o; o += N2h;
    Ly.Wimp = o; o += N2h;
    Ly.pos = o; o += N2h;
    Ly.fs = o; o += N2h;
    Ly.lp = o; o += N2h;
    Ly.cnt = o; o += T / 64 + 2;
    Ly.tc = o; o += D.n * tcw;
    Ly.ring = o; o += tl;
    Ly.moves = o; o += std::max(pmax, 1);
    o = (o + 1) & ~1;
    o = (o + 3) & ~3;
    Ly.prec = o; o += 4 * D.n;
    Ly.prq = o; o += D.n * std::max(D.nw, 1);
    Ly.predT = o; o += std::max(D.n_arcs, 1);
    // one candidate per lane, time-indexed: the lane offsets of the first
    // four predecessors' finish times per position (16-byte entries)
    const bool group = layout_is_group(G);
    const bool reg = G == kLayoutRegs;
    const bool wave = G == kLayoutWave;
    o = (o + 3) & ~3;
    Ly.pin = 0;
    if (dec == kEvalTime && !group && !wave) {
        Ly.pin = o;
        o += 4 * D.n;
    }
    // one candidate per wave: the first four predecessors' ids per position
    Ly.pid = 0;
    if (wave) {
        Ly.pid = o;
        o += 2 * D.n;
    }
    o = (o + 1) & ~1;
    Ly.red = o; o += 2 * (T / 64);
    Ly.scal = o; o += std::max(6, 2 + 3 * (T / 64));
    // per candidate: finish times, then the time-indexed profile (L units
    // plus 4 of slack for the 4-wide scan) or the capacity arrays and the
    // copy ring
    // G = 2: one candidate per lane with 8-bit finish times
    const int Fl = (dec == kEvalTime && layout_finish_bits(G) == 8) ? finish_dwords(D.n, 8) : F0;
    if (reg) Ly.per_lane = Fl;   // finish times only: the profile lives in registers
    else if (wave) {
        // a wave's finish times (the profile lives in registers); the region
        // also holds the finish times and a profile of L units for the
        // group decode of candidates past the register profile (L: the horizon)
        const int waves = T / 64;
        Ly.per_lane = std::max((F0 + 3) & ~3, ((F0 + (L + 4) * D.nw + waves - 1) / waves + 3) & ~3);
    }
    else if (group && dec == kEvalTime) Ly.per_lane = (F0 + L * D.nw + 3) & ~3;
    else if (group) Ly.per_lane = (F0 + (D.sum_r + 1) / 2 + (G * D.copy_p + 1) / 2 + 3) & ~3;   // a copy ring per lane
    else if (dec == kEvalTime) Ly.per_lane = Fl + (L + 4) * D.nw;
    else Ly.per_lane = F0 + (D.sum_r + 1) / 2 + D.copy_p / 2;
    Ly.cands = group ? T / G : (wave ? T / 64 : T);
    o = (o + 3) & ~3;
    Ly.bst = o;
    // one base state per workgroup (the register layout's base keeps its
    // profile in LDS: finish times placed so that the L + 4 units after them
    // start 16-byte aligned)
    Ly.base_stride = reg ? ((Fl + 3) & ~3) + (L + 4) * D.nw : ((Ly.per_lane + 3) & ~3);
    o += wave ? 0 : (group ? Ly.per_lane : Ly.base_stride);
    o = (o + 3) & ~3;
    Ly.region = o;
    o += Ly.cands * Ly.per_lane;
    // the long-profile decode (one thread, 16-bit finish times) uses the whole region
    Ly.long_len = dec == kEvalTime ? (Ly.cands * Ly.per_lane - F0) / D.nw - 4 : 0;
    Ly.total = o;
    return Ly;
}

// Workgroups of `bytes` dynamic LDS (and `reserve` static) that fit on one CU.
static int lds_occupancy(size_t bytes, int reserve) { return (int)(kMaxLds / (bytes + (size_t)reserve)); }

// Per-lane time-indexed profile length.  Without a request: at least
// 1.4 x the critical path plus two longest durations (neighbourhood
// makespans rarely pass it; longer schedules take the exact long-profile
// path), then as long as possible without lowering the number of
// workgroups per CU, never beyond the horizon.  The whole region must also
// hold one profile of the full horizon for the long-profile decode.
static rcpsp_status plan_layout(const rcpsp_instance *I, int dec, int T, int tcw, int tl, int pmax, int L_req,
                                int reserve, int *L_out, Layout *Ly_out, int G = 1) {
    const InstDesc &D = I->desc;
    const int budget = kMaxLds - 1024;  // static shared variables
    if (G == kLayoutWave && dec != kEvalTime) return fail(RCPSP_E_ARG, "one candidate per wave is time-indexed");
    if (dec == kEvalCapacity) {
        Layout Ly = make_layout(D, T, tcw, tl, pmax, 0, dec, G);
        if ((size_t)Ly.total * 4 > (size_t)budget)
            return fail(RCPSP_E_TOO_LARGE, "LDS %d bytes exceed %d (threads %d)", Ly.total * 4, budget, T);
        *L_out = 0;
        *Ly_out = Ly;
        return RCPSP_OK;
    }
    if (G == kLayoutWave) {
        // the profile is wave_profile_units(nw) units in the wave's registers
        if (T != kWaveThreads) return fail(RCPSP_E_ARG, "one candidate per wave runs at %d threads", kWaveThreads);
        if (I->n > kWaveMaxN)
            return fail(RCPSP_E_TOO_LARGE, "one candidate per wave holds at most %d activities", kWaveMaxN);
        if (L_req > 0 && L_req != wave_profile_units(D.nw))
            return fail(RCPSP_E_TOO_LARGE, "wave profiles hold %d units", wave_profile_units(D.nw));
        Layout Ly = make_layout(D, T, tcw, tl, pmax, std::max(I->H, 1), dec, G);
        if (Ly.long_len < I->H || (size_t)Ly.total * 4 > (size_t)budget)
            return fail(RCPSP_E_TOO_LARGE, "LDS %d bytes exceed %d (threads %d, wave profile)", Ly.total * 4, budget, T);
        *L_out = wave_profile_units(D.nw);
        *Ly_out = Ly;
        return RCPSP_OK;
    }
    if (G == kLayoutRegs) {
        // the lane profile is kRegUnits units in registers (one dword per unit)
        if (D.nw != 1 || (L_req > 0 && L_req != kRegUnits))
            return fail(RCPSP_E_TOO_LARGE, "register profiles hold %d units of one dword", kRegUnits);
        Layout Ly = make_layout(D, T, tcw, tl, pmax, kRegUnits, dec, G);
        if (Ly.long_len < I->H || (size_t)Ly.total * 4 > (size_t)budget)
            return fail(RCPSP_E_TOO_LARGE, "LDS %d bytes exceed %d (threads %d, register profile)", Ly.total * 4,
                        budget, T);
        *L_out = kRegUnits;
        *Ly_out = Ly;
        return RCPSP_OK;
    }
    // 8-bit finish times (G = 2) hold lane profiles of at most 255 units
    const int H = G == 2 ? std::min(std::max(I->H, 1), 255) : std::max(I->H, 1);
    auto fits = [&](int L, Layout *Ly) {
        *Ly = make_layout(D, T, tcw, tl, pmax, L, dec, G);
        return Ly->long_len >= I->H && (size_t)Ly->total * 4 <= (size_t)budget;
    };
    // smallest L' >= L (at most H) whose region holds the long profile
    // (long_len grows with L, so a binary search finds it)
    auto cover = [&](int L) {
        if (L >= H || make_layout(D, T, tcw, tl, pmax, L, dec, G).long_len >= I->H) return std::min(L, H);
        int lo = L, hi = H;  // long_len(lo) < H; hi satisfies or is H
        while (hi - lo > 1) {
            const int mid = lo + (hi - lo) / 2;
            if (make_layout(D, T, tcw, tl, pmax, mid, dec, G).long_len >= I->H) hi = mid;
            else lo = mid;
        }
        return hi;
    };
    Layout Ly;
    if (L_req > 0) {
        if (G == 2 && L_req > 255) return fail(RCPSP_E_TOO_LARGE, "8-bit finish times need a profile of at most 255");
        int L = cover(std::min(L_req, H));
        if (!fits(L, &Ly))
            return fail(RCPSP_E_TOO_LARGE, "LDS %d bytes exceed %d (threads %d, profile %d)", Ly.total * 4, budget, T, L);
        *L_out = L;
        *Ly_out = Ly;
        return RCPSP_OK;
    }
    int L = std::min(H, ((14 * I->cp + 9) / 10 + 2 * I->dmax + 15) / 16 * 16);
    L = cover(std::max(L, 1));
    // shorter profiles trade LDS for long-profile decodes; below 1.25 x the
    // critical path plus the longest duration most candidates of a search
    // take that path (schedules of tight instances run well past the critical
    // path), so the decoder does not fit
    const int Lfloor = std::max(16, std::min(H, (5 * I->cp + 3) / 4 + I->dmax));
    while (!fits(L, &Ly)) {
        if (L <= Lfloor)
            return fail(RCPSP_E_TOO_LARGE, "LDS %d bytes exceed %d (threads %d, profile %d)", Ly.total * 4, budget,
                        T, L);
        L = std::max(Lfloor, L * 3 / 4);
    }
    // stretch by steps of 4 while it fits and the workgroups per CU stay the
    // same (both monotone in L: binary search over the number of steps)
    const int k0 = lds_occupancy((size_t)Ly.total * 4, reserve);
    Layout Ln;
    auto ok = [&](int k) {
        const int Lk = L + 4 * k;
        return Lk <= H && fits(Lk, &Ln) && lds_occupancy((size_t)Ln.total * 4, reserve) >= k0;
    };
    int klo = 0, khi = (H - L) / 4 + 1;  // ok(klo) holds, ok(khi) does not
    while (khi - klo > 1) {
        const int mid = klo + (khi - klo) / 2;
        if (ok(mid)) klo = mid;
        else khi = mid;
    }
    L += 4 * klo;
    fits(L, &Ly);
    *L_out = L;
    *Ly_out = Ly;
    return RCPSP_OK;
}

// ---------------------------------------------------------------------------
// neighbourhood evaluation

rcpsp_status rcpsp::eval_device(const rcpsp_instance *I, const int32_t *order, int32_t delta, const uint8_t *tabu,
                                int32_t asp, int32_t *makespan, rcpsp_move *best, hipStream_t st) {
    if (delta < 1 || delta > kMaxDelta) return fail(RCPSP_E_ARG, "swap_range %d outside 1..%d", delta, kMaxDelta);
    const int P = potential_moves(I->n, delta);
    int T = 256, G = 1;
    int L = 0;
    Layout Ly;
    rcpsp_status s = RCPSP_E_TOO_LARGE;
    // one candidate per lane first (the profile in registers where a time
    // unit packs into one dword, else in LDS); groups when no lane state fits
    for (int g : {kLayoutRegs, 2, 1, 16, 8}) {
        if ((g == kLayoutRegs || g == 2 || g == 16) && I->eval != kEvalTime) continue;
        if (g == kLayoutRegs && I->desc.nw != 1) continue;
        if (g == 8 && I->eval != kEvalCapacity) continue;
        for (T = 256; T >= (g == kLayoutRegs ? 256 : 64); T /= 2) {
            s = plan_layout(I, I->eval, T, 0, 0, P, 0, 256, &L, &Ly, g);
            if (s != RCPSP_E_TOO_LARGE) break;
        }
        G = g;
        if (s != RCPSP_E_TOO_LARGE) break;
    }
    if (s != RCPSP_OK) return s;
    EvalArgs A{};
    A.D = I->desc;
    A.Ly = Ly;
    A.delta = delta;
    A.L = L;
    A.aspiration = asp;
    A.P = P;
    A.order = order;
    A.tabu = tabu;
    A.makespan = makespan;
    A.best = reinterpret_cast<int32_t *>(best);
    HIP_TRY(launch_eval(A, T, I->desc.nw, I->eval, G, (size_t)Ly.total * 4, st));
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_evaluate_neighbourhood_device(const rcpsp_instance *inst, const int32_t *order,
                                                            int32_t swap_range, const uint8_t *tabu,
                                                            int32_t aspiration, int32_t *makespan, rcpsp_move *best,
                                                            void *hip_stream) {
    if (!inst || !order || !best) return fail(RCPSP_E_ARG, "null pointer");
    return eval_device(inst, order, swap_range, tabu, aspiration, makespan, best, (hipStream_t)hip_stream);
}

bool rcpsp::feasible_order(const rcpsp_instance *I, const int32_t *order) {
    const int n = I->n;
    if (order[0] != 0 || order[n - 1] != n - 1) return false;
    std::vector<int> pos(n, -1);
    for (int p = 0; p < n; ++p) {
        if (order[p] < 0 || order[p] >= n || pos[order[p]] >= 0) return false;
        pos[order[p]] = p;
    }
    for (int i = 0; i < n; ++i)
        for (int e = I->succ_off[i]; e < I->succ_off[i + 1]; ++e)
            if (pos[i] >= pos[I->succ[e]]) return false;
    return true;
}

extern "C" rcpsp_status rcpsp_evaluate_neighbourhood(const rcpsp_instance *inst, const int32_t *order,
                                                     int32_t swap_range, const uint8_t *tabu, int32_t aspiration,
                                                     int32_t *makespan, int32_t cap, int32_t *n_potential,
                                                     rcpsp_move *best, void *hip_stream) {
    if (!inst || !order) return fail(RCPSP_E_ARG, "null pointer");
    if (swap_range < 1 || swap_range > kMaxDelta)
        return fail(RCPSP_E_ARG, "swap_range %d outside 1..%d", swap_range, kMaxDelta);
    const int P = potential_moves(inst->n, swap_range);
    if (n_potential) *n_potential = P;
    if (makespan && cap < P) return fail(RCPSP_E_BUFFER, "makespan buffer holds %d entries, %d needed", cap, P);
    if (!feasible_order(inst, order)) return fail(RCPSP_E_ORDER, "order is not a precedence-feasible permutation");
    hipStream_t st = (hipStream_t)hip_stream;
    const int n = inst->n;
    int32_t *d_order = nullptr, *d_mk = nullptr;
    rcpsp_move *d_best = nullptr;
    uint8_t *d_tabu = nullptr;
    rcpsp_status rs = RCPSP_OK;
    auto cleanup = [&]() {
        if (d_order) (void)hipFree(d_order);
        if (d_mk) (void)hipFree(d_mk);
        if (d_best) (void)hipFree(d_best);
        if (d_tabu) (void)hipFree(d_tabu);
    };
    do {
        hipError_t e;
        if ((e = hipMalloc(&d_order, sizeof(int32_t) * n)) != hipSuccess) break;
        if ((e = hipMalloc(&d_mk, sizeof(int32_t) * std::max(P, 1))) != hipSuccess) break;
        if ((e = hipMalloc(&d_best, sizeof(rcpsp_move))) != hipSuccess) break;
        if (tabu && (e = hipMalloc(&d_tabu, (size_t)n * n)) != hipSuccess) break;
        if ((e = hipMemcpyAsync(d_order, order, sizeof(int32_t) * n, hipMemcpyHostToDevice, st)) != hipSuccess) break;
        if (tabu && (e = hipMemcpyAsync(d_tabu, tabu, (size_t)n * n, hipMemcpyHostToDevice, st)) != hipSuccess) break;
        rs = eval_device(inst, d_order, swap_range, d_tabu, aspiration, d_mk, d_best, st);
        if (rs != RCPSP_OK) {
            cleanup();
            return rs;
        }
        rcpsp_move hb{};
        if ((e = hipMemcpyAsync(&hb, d_best, sizeof(rcpsp_move), hipMemcpyDeviceToHost, st)) != hipSuccess) break;
        if (makespan && (e = hipMemcpyAsync(makespan, d_mk, sizeof(int32_t) * P, hipMemcpyDeviceToHost, st)) != hipSuccess)
            break;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
        if (best) *best = hb;
        cleanup();
        return RCPSP_OK;
    } while (0);
    hipError_t e = hipGetLastError();
    cleanup();
    return fail(RCPSP_E_DEVICE, "device error in neighbourhood evaluation: %s", hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// search plans

// eq. 8 decay table: E[0] = 2^24, E[j] = floor(E[j-1] K / 2^32) with
// K = round(2^32 exp(-1/256)), until it reaches 0.
std::vector<uint32_t> rcpsp::decay_table() {
    const uint64_t K = 4278222805ull;
    std::vector<uint32_t> t;
    uint64_t e = 1ull << 24;
    while (e > 0) {
        t.push_back((uint32_t)e);
        e = (e * K) >> 32;
    }
    return t;
}

template <typename P>
static hipError_t dalloc(rcpsp_search *s, P **ptr, size_t bytes) {
    void *v = nullptr;
    const size_t nb = std::max<size_t>(bytes, 4);
    hipError_t e = s->allocator ? s->allocator->alloc(&v, nb) : hipMalloc(&v, nb);
    if (e == hipSuccess) {
        s->allocs.push_back(v);
        *ptr = static_cast<P *>(v);
    }
    return e;
}

extern "C" void rcpsp_search_destroy(rcpsp_search *s) {
    if (!s) return;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    for (void *v : s->allocs) {
        if (s->allocator) s->allocator->release(v);
        else (void)hipFree(v);
    }
    delete s;
}

// Timing of one eager run: HIP events recorded on the launch stream around
// every iteration-kernel and exchange-round launch.
struct RunTimer {
    std::vector<hipEvent_t> it_ev, rd_ev;
    size_t it_n = 0, rd_n = 0;
    hipError_t mark(std::vector<hipEvent_t> &v, size_t &n, hipStream_t st) {
        if (n == v.size()) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            v.push_back(ev);
        }
        return hipEventRecord(v[n++], st);
    }
    ~RunTimer() {
        for (hipEvent_t e : it_ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : rd_ev) (void)hipEventDestroy(e);
    }
};

// The launch sequence of one run: reset, then for a working set the record
// decodes, the initial exchange round and iteration/round pairs; without a
// working set one launch runs every iteration.
static hipError_t enqueue_run(rcpsp_search *s, hipStream_t st, RunTimer *tm) {
    const rcpsp_search_params &p = s->p;
    const SearchArgs &a = s->a;
    const int T = s->T, NF = p.elite;
    hipError_t e;
    auto search = [&](int it0, int n_it) -> hipError_t {
        SearchArgs ai = a;
        ai.it0 = it0;
        ai.n_it = n_it;
        hipError_t r;
        if (tm && (r = tm->mark(tm->it_ev, tm->it_n, st)) != hipSuccess) return r;
        if ((r = launch_search(ai, T, s->nw, s->dec, s->G, s->lds, st)) != hipSuccess) return r;
        if (tm && (r = tm->mark(tm->it_ev, tm->it_n, st)) != hipSuccess) return r;
        return hipSuccess;
    };
    auto round = [&](int parity, int init) -> hipError_t {
        hipError_t r;
        if (tm && (r = tm->mark(tm->rd_ev, tm->rd_n, st)) != hipSuccess) return r;
        if ((r = launch_round(a, parity, init, st)) != hipSuccess) return r;
        if (tm && (r = tm->mark(tm->rd_ev, tm->rd_n, st)) != hipSuccess) return r;
        return hipSuccess;
    };
    int nit = 0, nrd = 0;
    if ((e = launch_reset(a, st)) != hipSuccess) return e;
    if (p.fbi && (e = launch_fbi(a, T, s->nw, s->dec, s->lds, st)) != hipSuccess) return e;
    if (NF > 0) {
        if ((e = launch_decode_records(a, T, s->nw, s->dec, s->lds, st)) != hipSuccess) return e;
        if ((e = round(0, 1)) != hipSuccess) return e;
        ++nrd;
        // blocks of `every` iterations, each followed by an exchange round
        // (none after the last); exports and rounds alternate their buffers
        // by the parity of the block
        const int every = a.every;
        for (int it = 0; it < p.iterations; it += every) {
            const int n = std::min(every, p.iterations - it);
            if ((e = search(it, n)) != hipSuccess) return e;
            ++nit;
            if (it + n < p.iterations) {
                if ((e = round((it / every) & 1, 0)) != hipSuccess) return e;
                ++nrd;
            }
        }
        if (p.iterations == 0) {
            if ((e = search(0, 0)) != hipSuccess) return e;
            ++nit;
        }
    } else {
        if ((e = search(0, p.iterations)) != hipSuccess) return e;
        ++nit;
    }
    s->iteration_launches = nit;
    s->round_launches = nrd;
    return hipSuccess;
}

// Decoder, threads, lane layout and LDS of a plan (no allocation).
static rcpsp_status shape_plan(rcpsp_search *s) {
    const rcpsp_instance *I = s->inst;
    const rcpsp_search_params &p = s->p;
    const int N = I->n, B = p.searches, NF = p.elite;
    s->dec = p.eval ? p.eval : I->eval;
    s->nw = I->desc.nw;
    if (s->dec == kEvalTime && s->nw == 0)
        return fail(RCPSP_E_TOO_LARGE, "time-indexed profile needs more than %d dwords per time unit", kMaxNW);
    s->tcw = (p.swap_range + 31) / 32;
    s->P = potential_moves(N, p.swap_range);
    int T0 = p.threads ? p.threads : (B >= 256 ? 64 : (B >= 64 ? 128 : 256));
    if (T0 != 64 && T0 != 128 && T0 != 192 && T0 != 256 && T0 != 512)
        return fail(RCPSP_E_ARG, "threads must be 0, 64, 128, 192, 256 or 512");
    if (T0 == 192 && (s->dec != kEvalTime || p.lanes > 1))
        return fail(RCPSP_E_ARG, "192 threads per search needs the time-indexed decoder with one candidate per lane");
    if (p.lanes != 0 && p.lanes != 1 && p.lanes != 8 && p.lanes != 16 && p.lanes != kLayoutWave)
        return fail(RCPSP_E_ARG, "lanes must be 0, 1, 8, 16 or 64");
    if (p.lanes == 16 && s->dec != kEvalTime) return fail(RCPSP_E_ARG, "16 lanes per candidate needs the time-indexed decoder");
    if (p.lanes == 8 && s->dec != kEvalCapacity)
        return fail(RCPSP_E_ARG, "8 lanes per candidate needs the capacity-indexed decoder");
    if (p.lanes == kLayoutWave && (s->dec != kEvalTime || (p.threads != 0 && p.threads != kWaveThreads)))
        return fail(RCPSP_E_ARG, "one candidate per wave needs the time-indexed decoder and %d threads", kWaveThreads);
    if (T0 == 512 && p.lanes != kLayoutWave && !(p.lanes == 8 && s->dec == kEvalCapacity))
        return fail(RCPSP_E_ARG, "512 threads per search are for one candidate per wave (lanes 64) or "
                                 "8 lanes per capacity-indexed candidate");
    int T = T0;
    rcpsp_status st = RCPSP_E_TOO_LARGE;
    auto try_shape = [&](int G, int Lreq) {
        // 192 threads exist for the one-candidate-per-lane time-indexed layouts
        // only, kWaveThreads for one candidate per wave (and nothing else)
        T = (T0 == 192 && (s->dec != kEvalTime || layout_is_group(G) || G == kLayoutRegs)) ? 128 : T0;
        if (G == kLayoutWave) {
            T = kWaveThreads;
            st = plan_layout(I, s->dec, T, s->tcw, p.tabu_len, s->P, Lreq, s->reserve, &s->L, &s->Ly, G);
            s->G = G;
            return;
        }
        st = plan_layout(I, s->dec, T, s->tcw, p.tabu_len, s->P, Lreq, s->reserve, &s->L, &s->Ly, G);
        while (st == RCPSP_E_TOO_LARGE && p.threads == 0 && T > 64) {
            T /= 2;
            st = plan_layout(I, s->dec, T, s->tcw, p.tabu_len, s->P, Lreq, s->reserve, &s->L, &s->Ly, G);
        }
        s->G = G;
    };
    // one candidate per lane unless requested otherwise (time-indexed: 8-bit
    // finish times when the lane profile stays within 255 units, else
    // 16-bit); when no per-lane state fits, one candidate per 16 lanes
    // (time-indexed) or per 8 lanes (capacity-indexed)
    if (p.lane_profile == 2) {
        // time-indexed profile in registers: one candidate per lane, 256 threads
        if (s->dec != kEvalTime || p.lanes > 1 || (p.threads != 0 && p.threads != 256))
            return fail(RCPSP_E_ARG, "a register profile needs the time-indexed decoder, one candidate per lane "
                                     "and 256 threads");
        T0 = 256;
        try_shape(kLayoutRegs, p.profile_len);
        if (st != RCPSP_OK) return st;
    } else if (p.lanes > 1) {
        try_shape(p.lanes, p.profile_len);
    } else if (s->dec == kEvalTime) {
        // automatic: the register profile where it applies (a time unit in
        // one dword, 256 threads, no profile length asked for), else LDS
        if (p.lane_profile == 0 && s->nw == 1 && (p.threads == 0 || p.threads == 256) && p.profile_len == 0) {
            const int T0s = T0;
            T0 = 256;
            try_shape(kLayoutRegs, 0);
            if (st != RCPSP_OK) T0 = T0s;
        }
        if (st == RCPSP_E_TOO_LARGE) try_shape(2, p.profile_len);
        if (st == RCPSP_E_TOO_LARGE) try_shape(1, p.profile_len);
    } else {
        try_shape(1, p.profile_len);
    }
    // no lane state fits: one time-indexed candidate per wave, else per 16
    // lanes; one capacity-indexed candidate per 8 lanes
    if (st == RCPSP_E_TOO_LARGE && p.lanes == 0 && s->dec == kEvalTime && p.threads == 0 && p.profile_len == 0)
        try_shape(kLayoutWave, 0);
    if (st == RCPSP_E_TOO_LARGE && p.lanes == 0) try_shape(s->dec == kEvalTime ? 16 : 8, p.profile_len);
    if (st == RCPSP_E_TOO_LARGE && p.eval == RCPSP_EVAL_AUTO && s->dec == kEvalTime) {
        // automatic choice: no time-indexed profile fits, take the capacity-indexed decoder
        s->dec = kEvalCapacity;
        try_shape(1, 0);
        if (st == RCPSP_E_TOO_LARGE && p.lanes == 0) try_shape(8, 0);
    }
    if (st != RCPSP_OK) return st;
    s->T = T;
    s->lds = (size_t)s->Ly.total * 4;
    if (NF > 0 && round_lds_bytes(B, NF) > (size_t)kMaxLds)
        return fail(RCPSP_E_TOO_LARGE, "%d searches with a working set exceed the exchange kernel's LDS", B);
    return RCPSP_OK;
}

// Iteration-kernel workgroups of a shaped plan: those that fit the GPU at
// once, at most one per search.
static rcpsp_status plan_grid(const rcpsp_search *s, int *grid) {
    int per_cu = 0, cus = 0, dev = 0;
    HIP_TRY(prepare_search(s->T, s->nw, s->dec, s->G, s->lds, s->p.searches, s->p.elite));
    HIP_TRY(search_occupancy(s->T, s->nw, s->dec, s->G, s->lds, &per_cu));
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *grid = per_cu > 0 ? std::min(s->p.searches, per_cu * cus) : s->p.searches;
    return RCPSP_OK;
}

// Device wall-clock ticks per microsecond, measured once per device: two
// readings of the clock kernel 20 ms apart on the host's steady clock (the
// rate the driver reports has disagreed with the counter).
static rcpsp_status wall_ticks_per_us(double *out) {
    static std::mutex mu;
    static std::map<int, double> rate;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto found = rate.find(dev);
    if (found != rate.end()) {
        *out = found->second;
        return RCPSP_OK;
    }
    long long *d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(long long)));
    long long ticks[2] = {0, 0};
    std::chrono::steady_clock::time_point host[2];
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        if (i) std::this_thread::sleep_for(std::chrono::milliseconds(20));
        e = launch_clock(d, nullptr);
        if (e == hipSuccess) e = hipMemcpy(&ticks[i], d, sizeof(long long), hipMemcpyDeviceToHost);
        host[i] = std::chrono::steady_clock::now();
    }
    (void)hipFree(d);
    if (e != hipSuccess) return fail(RCPSP_E_DEVICE, "device clock: %s", hipGetErrorString(e));
    const double us = std::chrono::duration<double, std::micro>(host[1] - host[0]).count();
    if (!(us > 0.0) || ticks[1] <= ticks[0]) return fail(RCPSP_E_DEVICE, "device wall clock does not advance");
    rate[dev] = *out = (double)(ticks[1] - ticks[0]) / us;
    return RCPSP_OK;
}

// Layout and device state of a plan (no launches).
rcpsp_status rcpsp::alloc_plan(rcpsp_search *s) {
    const rcpsp_instance *I = s->inst;
    const rcpsp_search_params &p = s->p;
    const int N = I->n, N2 = n2(N), B = p.searches, NF = p.elite;
    rcpsp_status st = shape_plan(s);
    if (st != RCPSP_OK) return st;

    SearchArgs &a = s->a;
    a = SearchArgs{};
    a.D = I->desc;
    a.Ly = s->Ly;
    a.delta = p.swap_range;
    a.tl = p.tabu_len;
    a.iters = p.iterations;
    a.B = B;
    a.NF = NF;
    a.phi_max = p.phi_max;
    a.phi_steps = p.phi_steps;
    a.tcw = s->tcw;
    a.L = s->L;
    a.record = p.record_trajectory ? 1 : 0;
    a.count_work = p.count_work ? 1 : 0;
    a.full_decode = p.full_decode ? 1 : 0;
    a.seed = p.seed;
    a.every = std::max(1, p.exchange_every);
    a.budget_ticks = 0;
    if (p.time_budget_us > 0) {
        double per_us = 0.0;
        rcpsp_status cst = wall_ticks_per_us(&per_us);
        if (cst != RCPSP_OK) return cst;
        a.budget_ticks = std::max(1ll, (long long)std::llround(per_us * (double)p.time_budget_us));
    }
    const int tcn = N * s->tcw;
    HIP_TRY(dalloc(s, &a.sc, sizeof(SearchScalars) * B));
    HIP_TRY(dalloc(s, &a.Wcur, sizeof(uint16_t) * (size_t)B * N2));
    HIP_TRY(dalloc(s, &a.Wimp, sizeof(uint16_t) * (size_t)B * N2));
    HIP_TRY(dalloc(s, &a.Wbest, sizeof(uint16_t) * (size_t)B * N2));
    HIP_TRY(dalloc(s, &a.ring, sizeof(uint32_t) * (size_t)B * p.tabu_len));
    HIP_TRY(dalloc(s, &a.tc, sizeof(uint32_t) * (size_t)B * tcn));
    if (NF > 0) {
        HIP_TRY(dalloc(s, &a.Xw, sizeof(uint16_t) * 2 * (size_t)B * N2));
        HIP_TRY(dalloc(s, &a.Xring, sizeof(uint32_t) * 2 * (size_t)B * p.tabu_len));
        HIP_TRY(dalloc(s, &a.Xtc, sizeof(uint32_t) * 2 * (size_t)B * tcn));
        HIP_TRY(dalloc(s, &a.Xwidx, sizeof(int) * 2 * (size_t)B));
        HIP_TRY(dalloc(s, &a.Fw, sizeof(uint16_t) * 2 * (size_t)NF * N2));
        HIP_TRY(dalloc(s, &a.Fring, sizeof(uint32_t) * 2 * (size_t)NF * p.tabu_len));
        HIP_TRY(dalloc(s, &a.Ftc, sizeof(uint32_t) * 2 * (size_t)NF * tcn));
        HIP_TRY(dalloc(s, &a.Fwidx, sizeof(int) * 2 * (size_t)NF));
        HIP_TRY(dalloc(s, &a.Fmeta, sizeof(SlotMeta) * NF));
    }
    HIP_TRY(dalloc(s, &a.g, sizeof(Global)));
    if (a.record) HIP_TRY(dalloc(s, &a.traj, sizeof(int) * 4 * (size_t)B * std::max(p.iterations, 1)));
    if (s->shared_decay) {
        a.decay = s->shared_decay;
        a.decay_len = s->shared_decay_len;
    } else {
        std::vector<uint32_t> E = decay_table();
        uint32_t *dE = nullptr;
        HIP_TRY(dalloc(s, &dE, sizeof(uint32_t) * E.size()));
        HIP_TRY(hipMemcpy(dE, E.data(), sizeof(uint32_t) * E.size(), hipMemcpyHostToDevice));
        a.decay = dE;
        a.decay_len = (int)E.size();
    }
    // the set-up kernels initialise every state a run reads; the clears
    // below only keep never-written buffers from being copied uninitialised
    if (s->allocator) return RCPSP_OK;
    HIP_TRY(hipMemset(a.g, 0, sizeof(Global)));
    if (NF > 0) {
        // export and record buffers are always written before they are read;
        // clear them once so that no uninitialised memory is ever copied
        HIP_TRY(hipMemset(a.Xwidx, 0, sizeof(int) * 2 * (size_t)B));
        HIP_TRY(hipMemset(a.Fwidx, 0, sizeof(int) * 2 * (size_t)NF));
    }

    return RCPSP_OK;
}

static rcpsp_status build_plan(rcpsp_search *s, hipStream_t user_stream) {
    rcpsp_status st0 = alloc_plan(s);
    if (st0 == RCPSP_OK) st0 = plan_grid(s, &s->a.grid);
    if (st0 != RCPSP_OK) return st0;
    // capture the whole run as one graph
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(RCPSP_E_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    e = enqueue_run(s, cs, nullptr);
    if (e != hipSuccess) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cs, &g);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        return fail(RCPSP_E_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    e = hipStreamEndCapture(cs, &s->graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return fail(RCPSP_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    HIP_TRY(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0));
    (void)user_stream;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_search_create(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                            void *hip_stream, rcpsp_search **out) {
    if (!inst || !params || !out) return fail(RCPSP_E_ARG, "null pointer");
    *out = nullptr;
    const rcpsp_search_params &p = *params;
    rcpsp_status st0 = validate_params(p);
    if (st0 != RCPSP_OK) return st0;
    if ((long long)p.searches * std::max(p.iterations, 1) * 4 > (1ll << 40))
        return fail(RCPSP_E_TOO_LARGE, "trajectory too large");
    rcpsp_search *s = new (std::nothrow) rcpsp_search();
    if (!s) return fail(RCPSP_E_NOMEM, "out of host memory");
    s->inst = inst;
    s->p = p;
    rcpsp_status st = build_plan(s, (hipStream_t)hip_stream);
    if (st != RCPSP_OK) {
        rcpsp_search_destroy(s);
        return st;
    }
    *out = s;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_search_run(rcpsp_search *s, void *hip_stream) {
    if (!s) return fail(RCPSP_E_ARG, "null search");
    HIP_TRY(hipGraphLaunch(s->exec, (hipStream_t)hip_stream));
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_search_run_timed(rcpsp_search *s, void *hip_stream, double *iteration_ms,
                                               double *round_ms, double *total_ms) {
    if (!s) return fail(RCPSP_E_ARG, "null search");
    hipStream_t st = (hipStream_t)hip_stream;
    RunTimer tm;
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    HIP_TRY(hipEventRecord(t0, st));
    hipError_t e = enqueue_run(s, st, &tm);
    if (e == hipSuccess) e = hipEventRecord(t1, st);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    double it = 0.0, rd = 0.0;
    float ms = 0.f;
    for (size_t i = 0; e == hipSuccess && i + 1 < tm.it_n; i += 2)
        if ((e = hipEventElapsedTime(&ms, tm.it_ev[i], tm.it_ev[i + 1])) == hipSuccess) it += ms;
    for (size_t i = 0; e == hipSuccess && i + 1 < tm.rd_n; i += 2)
        if ((e = hipEventElapsedTime(&ms, tm.rd_ev[i], tm.rd_ev[i + 1])) == hipSuccess) rd += ms;
    if (e == hipSuccess && (e = hipEventElapsedTime(&ms, t0, t1)) == hipSuccess && total_ms) *total_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return fail(RCPSP_E_DEVICE, "timed run: %s", hipGetErrorString(e));
    if (iteration_ms) *iteration_ms = it;
    if (round_ms) *round_ms = rd;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_search_get_config(const rcpsp_search *s, rcpsp_search_config *out) {
    if (!s || !out) return fail(RCPSP_E_ARG, "null pointer");
    out->threads = s->T;
    out->profile_len = s->L;
    out->lds_bytes = (int)s->lds;
    out->eval = s->dec;
    out->iteration_launches = s->iteration_launches;
    out->round_launches = s->round_launches;
    out->lanes = (layout_is_group(s->G) || s->G == kLayoutWave) ? s->G : 1;
    out->finish_bits = layout_finish_bits(s->G);
    out->register_profile = s->G == kLayoutRegs ? 1 : 0;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_search_results(rcpsp_search *s, rcpsp_search_result *res, void *hip_stream) {
    if (!s || !res) return fail(RCPSP_E_ARG, "null pointer");
    const SearchArgs &a = s->a;
    const int N = s->inst->n, N2 = n2(N), B = a.B, NF = a.NF;
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    std::vector<SearchScalars> sc(B);
    HIP_TRY(hipMemcpy(sc.data(), a.sc, sizeof(SearchScalars) * B, hipMemcpyDeviceToHost));
    int gbest = INT_MAX;
    long long tot = 0, ovf = 0, work = 0, cells = 0;
    for (int b = 0; b < B; ++b) {
        gbest = std::min(gbest, sc[b].C_best);
        tot += sc[b].evals;
        ovf += sc[b].overflow;
        work += sc[b].work;
        cells += sc[b].cells;
        if (res->best_makespan) res->best_makespan[b] = sc[b].C_best;
        if (res->iterations_done) res->iterations_done[b] = sc[b].it_done;
        if (res->evaluations) res->evaluations[b] = sc[b].evals;
    }
    if (res->best_order) {
        std::vector<uint16_t> w((size_t)B * N2);
        HIP_TRY(hipMemcpy(w.data(), a.Wbest, sizeof(uint16_t) * w.size(), hipMemcpyDeviceToHost));
        for (int b = 0; b < B; ++b)
            for (int i = 0; i < N; ++i) res->best_order[(size_t)b * N + i] = w[(size_t)b * N2 + i];
    }
    if (res->trajectory) {
        if (!a.record) return fail(RCPSP_E_ARG, "trajectory requested but the plan does not record it");
        HIP_TRY(hipMemcpy(res->trajectory, a.traj, sizeof(int) * 4 * (size_t)B * a.iters, hipMemcpyDeviceToHost));
    }
    if (NF > 0) {
        std::vector<SlotMeta> meta(NF);
        HIP_TRY(hipMemcpy(meta.data(), a.Fmeta, sizeof(SlotMeta) * NF, hipMemcpyDeviceToHost));
        std::vector<uint16_t> fw(2 * (size_t)NF * N2);
        if (res->elite_order)
            HIP_TRY(hipMemcpy(fw.data(), a.Fw, sizeof(uint16_t) * fw.size(), hipMemcpyDeviceToHost));
        for (int k = 0; k < NF; ++k) {
            gbest = std::min(gbest, meta[k].C);
            if (res->elite_makespan) res->elite_makespan[k] = meta[k].C;
            if (res->elite_order)
                for (int i = 0; i < N; ++i)
                    res->elite_order[(size_t)k * N + i] = fw[((size_t)meta[k].buf * NF + k) * N2 + i];
        }
    }
    res->global_best = gbest;
    res->total_evaluations = tot;
    res->overflow_decodes = (int32_t)std::min<long long>(ovf, INT_MAX);
    res->total_work = work;
    res->total_cells = cells;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_tabu_search(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                          rcpsp_search_result *res, void *hip_stream) {
    rcpsp_search *s = nullptr;
    rcpsp_status st = rcpsp_search_create(inst, params, hip_stream, &s);
    if (st != RCPSP_OK) return st;
    st = rcpsp_search_run(s, hip_stream);
    if (st == RCPSP_OK) st = rcpsp_search_results(s, res, hip_stream);
    rcpsp_search_destroy(s);
    return st;
}

// Heterogeneous model (the CPU-driven alternative the paper sets against its
// homogeneous one, Section 1): the host runs every search's loop and the GPU
// only evaluates each iteration's neighbourhood (the device entry point of
// rcpsp_evaluate_neighbourhood, one launch and one read-back per
// iteration).  Initial orders and their makespans come from the reset and
// decode kernels of a plan of the same searches run for no iteration, so a
// host-driven search follows exactly the trajectory of the homogeneous one.
extern "C" rcpsp_status rcpsp_tabu_search_hosted(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                                 rcpsp_search_result *res, void *hip_stream) {
    if (!inst || !params || !res) return fail(RCPSP_E_ARG, "null pointer");
    const rcpsp_search_params &p = *params;
    rcpsp_status st = validate_params(p);
    if (st != RCPSP_OK) return st;
    if (p.elite != 0) return fail(RCPSP_E_ARG, "host-driven searches are independent (elite must be 0)");
    if (p.count_work) return fail(RCPSP_E_ARG, "count_work is not available for host-driven searches");
    if (p.eval != 0 && p.eval != inst->eval)
        return fail(RCPSP_E_ARG, "host-driven searches decode with the instance's decoder");
    if (p.time_budget_us != 0) return fail(RCPSP_E_ARG, "host-driven searches take no time budget");
    hipStream_t hs = (hipStream_t)hip_stream;
    const int N = inst->n, B = p.searches, iters = p.iterations, tl = p.tabu_len;
    // initial orders and makespans
    rcpsp_search_params p0 = p;
    p0.iterations = 0;
    p0.record_trajectory = 0;
    p0.eval = inst->eval;
    rcpsp_search *s0 = nullptr;
    st = rcpsp_search_create(inst, &p0, hip_stream, &s0);
    if (st != RCPSP_OK) return st;
    std::vector<int32_t> W0((size_t)B * N), C0(B);
    st = rcpsp_search_run(s0, hip_stream);
    if (st == RCPSP_OK) {
        rcpsp_search_result r0{};
        r0.best_order = W0.data();
        r0.best_makespan = C0.data();
        st = rcpsp_search_results(s0, &r0, hip_stream);
    }
    rcpsp_search_destroy(s0);
    if (st != RCPSP_OK) return st;
    struct Bufs {
        int32_t *order = nullptr;
        uint8_t *tabu = nullptr;
        rcpsp_move *best = nullptr;
        ~Bufs() {
            if (order) (void)hipFree(order);
            if (tabu) (void)hipFree(tabu);
            if (best) (void)hipFree(best);
        }
    } d;
    HIP_TRY(hipMalloc(&d.order, sizeof(int32_t) * N));
    HIP_TRY(hipMalloc(&d.tabu, (size_t)N * N));
    HIP_TRY(hipMalloc(&d.best, sizeof(rcpsp_move)));
    std::vector<uint8_t> tabu((size_t)N * N);
    std::vector<uint32_t> ring(tl);
    int gbest = INT_MAX;
    long long tot = 0;
    for (int b = 0; b < B; ++b) {
        std::vector<int32_t> W(W0.begin() + (size_t)b * N, W0.begin() + (size_t)(b + 1) * N), Wb = W;
        int Cbest = C0[b], it = 0, widx = 0;
        long long ev = 0;
        std::fill(tabu.begin(), tabu.end(), 0);
        std::fill(ring.begin(), ring.end(), 0u);
        HIP_TRY(hipMemcpyAsync(d.tabu, tabu.data(), tabu.size(), hipMemcpyHostToDevice, hs));
        int32_t *traj = (res->trajectory && p.record_trajectory) ? res->trajectory + (size_t)b * iters * 4 : nullptr;
        if (traj) std::fill(traj, traj + (size_t)iters * 4, -1);
        for (; it < iters; ++it) {
            if (Cbest == inst->cp) break;   // independent searches stop at the critical path
            HIP_TRY(hipMemcpyAsync(d.order, W.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, hs));
            st = eval_device(inst, d.order, p.swap_range, d.tabu, Cbest, nullptr, d.best, hs);
            if (st != RCPSP_OK) return st;
            rcpsp_move mv{};
            HIP_TRY(hipMemcpyAsync(&mv, d.best, sizeof(rcpsp_move), hipMemcpyDeviceToHost, hs));
            HIP_TRY(hipStreamSynchronize(hs));
            if (mv.n_feasible < 0) return fail(RCPSP_E_DEVICE, "neighbourhood evaluation rejected the order");
            if (mv.n_feasible == 0) break;   // no feasible move: the search stops
            const int u = mv.u, v = mv.v, c = mv.makespan;
            std::swap(W[u], W[v]);
            // Alg. 3: evict the oldest entry, insert (u, v), advance the write index
            const uint32_t old = ring[widx];
            if (old != 0u) {
                const size_t e = (size_t)(old & 0xffff) * N + (old >> 16);
                tabu[e] = 0;
                HIP_TRY(hipMemcpyAsync(d.tabu + e, &tabu[e], 1, hipMemcpyHostToDevice, hs));
            }
            ring[widx] = (uint32_t)u | ((uint32_t)v << 16);
            const size_t e = (size_t)u * N + v;
            tabu[e] = 1;
            HIP_TRY(hipMemcpyAsync(d.tabu + e, &tabu[e], 1, hipMemcpyHostToDevice, hs));
            widx = (widx + 1) % tl;
            ev += mv.n_feasible;
            if (c < Cbest) {
                Cbest = c;
                Wb = W;
            }
            if (traj) {
                traj[(size_t)it * 4] = u;
                traj[(size_t)it * 4 + 1] = v;
                traj[(size_t)it * 4 + 2] = c;
                traj[(size_t)it * 4 + 3] = Cbest;
            }
        }
        HIP_TRY(hipStreamSynchronize(hs));
        gbest = std::min(gbest, Cbest);
        tot += ev;
        if (res->best_makespan) res->best_makespan[b] = Cbest;
        if (res->iterations_done) res->iterations_done[b] = it;
        if (res->evaluations) res->evaluations[b] = ev;
        if (res->best_order) std::copy(Wb.begin(), Wb.end(), res->best_order + (size_t)b * N);
    }
    res->global_best = gbest;
    res->total_evaluations = tot;
    res->overflow_decodes = 0;
    res->total_work = 0;
    res->total_cells = 0;
    return RCPSP_OK;
}

// Periodic decoder re-selection (what the paper's sequential CPU version
// does instead of the Section 5.4 rules, Section 7): the searches of one plan
// run on the device as usual, and at the start of every period each decoder
// that fits runs a few iterations, timed with HIP events around its
// iteration launches; the faster one runs the rest of the period.  The two
// decoders are different functions (the time-indexed serial schedule
// back-fills, the capacity-indexed one does not), so the choice changes the
// search: every decode of iteration it (its neighbourhood, a diversified
// read that the preceding exchange round gave it) uses the decoder of the
// segment holding it, and the log of segments is what a replay needs.  The
// plan's device state is shared: each decoder has its own lane layout,
// threads and grid over the same buffers in HBM.
namespace {
struct ReselectShape {
    int dec, T, nw, G;
    size_t lds;
    SearchArgs a;
};
struct PlanGuard {
    rcpsp_search *s = nullptr;
    ~PlanGuard() { rcpsp_search_destroy(s); }
};
struct EventPool {
    std::vector<hipEvent_t> ev;
    ~EventPool() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};
}  // namespace

extern "C" rcpsp_status rcpsp_tabu_search_reselect(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                                   int32_t period, int32_t probe, rcpsp_search_result *res,
                                                   rcpsp_decoder_segment *log, int32_t log_cap, int32_t *n_log,
                                                   void *hip_stream) {
    if (!inst || !params || !res || !n_log || (log_cap > 0 && !log)) return fail(RCPSP_E_ARG, "null pointer");
    if (log_cap < 0) return fail(RCPSP_E_ARG, "log_cap must be >= 0");
    if (probe < 1 || period < 2 * probe) return fail(RCPSP_E_ARG, "need probe >= 1 and period >= 2 * probe");
    *n_log = 0;
    const rcpsp_search_params &p = *params;
    rcpsp_status st = validate_params(p);
    if (st != RCPSP_OK) return st;
    if (p.eval != 0) return fail(RCPSP_E_ARG, "the decoder is chosen by timing (eval must be 0)");
    if (p.exchange_every > 1 || p.time_budget_us != 0)
        return fail(RCPSP_E_ARG, "re-selecting searches exchange after every iteration and take no time budget");
    if ((long long)p.searches * std::max(p.iterations, 1) * 4 > (1ll << 40))
        return fail(RCPSP_E_TOO_LARGE, "trajectory too large");
    hipStream_t hs = (hipStream_t)hip_stream;
    // the plan (state in HBM, set-up with the instance's decoder) ...
    PlanGuard g;
    g.s = new (std::nothrow) rcpsp_search();
    if (!g.s) return fail(RCPSP_E_NOMEM, "out of host memory");
    rcpsp_search *s = g.s;
    s->inst = inst;
    s->p = p;
    if ((st = alloc_plan(s)) != RCPSP_OK || (st = plan_grid(s, &s->a.grid)) != RCPSP_OK) return st;
    // ... and one shape per decoder over it; a decoder whose layout does not
    // fit, or that the instance cannot use, takes no part
    std::vector<ReselectShape> shapes;
    for (int dec : {kEvalTime, kEvalCapacity}) {
        ReselectShape sh{};
        if (dec == s->dec) {
            sh = ReselectShape{s->dec, s->T, s->nw, s->G, s->lds, s->a};
        } else {
            rcpsp_search alt;
            alt.inst = inst;
            alt.p = p;
            alt.p.eval = dec;
            // threads and lanes the other decoder does not support fall back to its automatic shape
            if (dec == kEvalCapacity && (alt.p.threads == 192 || alt.p.lanes == 16)) {
                alt.p.threads = 0;
                alt.p.lanes = 0;
            }
            if (dec == kEvalTime && alt.p.lanes == 8) alt.p.lanes = 0;
            rcpsp_status sst = shape_plan(&alt);
            if (sst == RCPSP_E_TOO_LARGE) continue;
            if (sst != RCPSP_OK) return sst;
            sh = ReselectShape{alt.dec, alt.T, alt.nw, alt.G, alt.lds, s->a};
            sh.a.Ly = alt.Ly;
            sh.a.L = alt.L;
            if ((sst = plan_grid(&alt, &sh.a.grid)) != RCPSP_OK) return sst;
        }
        shapes.push_back(sh);
    }
    const ReselectShape *cur = nullptr;
    for (const ReselectShape &sh : shapes)
        if (sh.dec == s->dec) cur = &sh;
    const int iters = p.iterations, NF = p.elite;
    const SearchArgs &a0 = s->a;
    EventPool pool;
    size_t n_ev = 0;
    auto mark = [&](hipStream_t stq) -> hipError_t {
        if (n_ev == pool.ev.size()) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            pool.ev.push_back(ev);
        }
        return hipEventRecord(pool.ev[n_ev++], stq);
    };
    // iterations [it0, it0 + n) with one shape; returns the summed
    // iteration-launch milliseconds
    auto run = [&](const ReselectShape &sh, int it0, int n, double *ms) -> rcpsp_status {
        n_ev = 0;
        auto search = [&](int i0, int k) -> hipError_t {
            SearchArgs ai = sh.a;
            ai.it0 = i0;
            ai.n_it = k;
            // the queue of searches starts from zero (an exchange round
            // clears it too, but not every launch follows one)
            hipError_t e = launch_fill_zero(&a0.g->queue, 1, hs);
            if (e != hipSuccess) return e;
            if ((e = mark(hs)) != hipSuccess) return e;
            if ((e = launch_search(ai, sh.T, sh.nw, sh.dec, sh.G, sh.lds, hs)) != hipSuccess) return e;
            return mark(hs);
        };
        if (n == 0) {
            // no iteration: the launch only decodes the initial orders
            HIP_TRY(search(it0, 0));
        } else if (NF > 0) {
            for (int it = it0; it < it0 + n; ++it) {
                HIP_TRY(search(it, 1));
                if (it < iters - 1) HIP_TRY(launch_round(a0, it & 1, 0, hs));
            }
        } else {
            HIP_TRY(search(it0, n));
        }
        HIP_TRY(hipStreamSynchronize(hs));
        double t = 0.0;
        for (size_t i = 0; i + 1 < n_ev; i += 2) {
            float f = 0.f;
            HIP_TRY(hipEventElapsedTime(&f, pool.ev[i], pool.ev[i + 1]));
            t += f;
        }
        *ms = t;
        return RCPSP_OK;
    };
    int32_t nl = 0;
    auto note = [&](int first, int n, int dec, int is_probe, double ms) {
        if (nl < log_cap) log[nl] = rcpsp_decoder_segment{first, n, dec, is_probe, (float)(ms / n)};
        ++nl;
    };
    HIP_TRY(launch_reset(a0, hs));
    if (p.fbi) HIP_TRY(launch_fbi(a0, cur->T, cur->nw, cur->dec, cur->lds, hs));
    if (NF > 0) {
        HIP_TRY(launch_decode_records(a0, cur->T, cur->nw, cur->dec, cur->lds, hs));
        HIP_TRY(launch_round(a0, 0, 1, hs));
    }
    // a launch of no iteration decodes the initial orders (and completes the
    // first reads) with the instance's decoder
    double ms = 0.0;
    if ((st = run(*cur, 0, 0, &ms)) != RCPSP_OK) return st;
    for (int it = 0; it < iters;) {
        const int end = std::min(iters, it + period);
        if (shapes.size() > 1) {
            double best = 0.0;
            for (const ReselectShape &sh : shapes) {
                const int n = std::min(probe, end - it);
                if (n <= 0) break;
                if ((st = run(sh, it, n, &ms)) != RCPSP_OK) return st;
                note(it, n, sh.dec, 1, ms);
                if (&sh == &shapes[0] || ms / n < best) {
                    best = ms / n;
                    cur = &sh;
                }
                it += n;
            }
        }
        if (end > it) {
            if ((st = run(*cur, it, end - it, &ms)) != RCPSP_OK) return st;
            note(it, end - it, cur->dec, 0, ms);
            it = end;
        }
    }
    *n_log = nl;
    s->iteration_launches = 0;
    st = rcpsp_search_results(s, res, hip_stream);
    if (st == RCPSP_OK && nl > log_cap)
        return fail(RCPSP_E_BUFFER, "%d segments, log holds %d (results are complete)", nl, log_cap);
    return st;
}

extern "C" rcpsp_status rcpsp_autotune(const rcpsp_instance *inst, const rcpsp_search_params *params,
                                      int32_t trial_iterations, void *hip_stream, rcpsp_search_params *out,
                                      rcpsp_tuning *info) {
    if (!inst || !params || !out) return fail(RCPSP_E_ARG, "null pointer");
    if (trial_iterations < 1) return fail(RCPSP_E_ARG, "trial_iterations must be >= 1");
    std::vector<int> evals;
    if (params->eval) evals.push_back(params->eval);
    else {
        if (inst->desc.nw) evals.push_back(kEvalTime);
        evals.push_back(kEvalCapacity);
    }
    std::vector<int> threads;
    if (params->threads) threads.push_back(params->threads);
    else {
        threads.push_back(64);
        threads.push_back(128);
        threads.push_back(192);
        if (params->searches < 128) threads.push_back(256);
    }
    // profile lengths: the automatic choice, and a shorter one that may fit
    // more workgroups per CU at the price of more long-profile decodes
    const int Lshort = std::min(inst->H, ((6 * inst->cp + 4) / 5 + 2 * inst->dmax + 15) / 16 * 16);
    bool found = false;
    double best_ns = 0.0;
    rcpsp_search_params best{};
    int trials = 0;
    std::vector<int> lanes_c;
    if (params->lanes) lanes_c.push_back(params->lanes);
    else lanes_c = {1, 8, 16};
    // lane profiles: in LDS (every lane layout), and in registers for the
    // time-indexed one-candidate-per-lane layout at 256 threads
    std::vector<int> lps;
    if (params->lane_profile) lps.push_back(params->lane_profile);
    else lps = {1, 2};
    for (int ev : evals) {
      for (int G : lanes_c) {
        if ((G == 16 && ev != kEvalTime) || (G == 8 && ev != kEvalCapacity) || G == kLayoutWave) continue;
        // register profiles run at 256 threads whatever the search count,
        // capacity-indexed 8-lane groups also at 512
        std::vector<int> Ts = threads;
        if (!params->threads && std::find(Ts.begin(), Ts.end(), 256) == Ts.end()) Ts.push_back(256);
        if (!params->threads && G == 8) Ts.push_back(512);
        for (int T : Ts)
        for (int lp : lps) {
            if (T == 256 && lp == 1 && std::find(threads.begin(), threads.end(), 256) == threads.end()) continue;
            if (T == 192 && (ev != kEvalTime || G != 1)) continue;
            if (lp == 2 && (ev != kEvalTime || G != 1 || T != (params->threads ? params->threads : 256) ||
                            inst->desc.nw != 1))
                continue;
            std::vector<int> Ls;
            if (ev == kEvalTime && !params->profile_len && lp == 1) {
                Ls.push_back(0);
                Ls.push_back(std::max(Lshort, 16));
            } else {
                Ls.push_back(lp == 2 ? 0 : params->profile_len);
            }
            for (int L : Ls) {
                rcpsp_search_params q = *params;
                q.eval = ev;
                q.threads = T;
                q.profile_len = L;
                q.lanes = G;
                q.lane_profile = lp;
                q.iterations = trial_iterations;
                q.record_trajectory = 0;
                q.count_work = 0;
                rcpsp_search *s = nullptr;
                rcpsp_status st = rcpsp_search_create(inst, &q, hip_stream, &s);
                if (st == RCPSP_E_TOO_LARGE) continue;
                if (st != RCPSP_OK) return st;
                double ms = 0.0;
                rcpsp_search_result r{};
                st = rcpsp_search_run(s, hip_stream);
                if (st == RCPSP_OK) st = rcpsp_search_run_timed(s, hip_stream, nullptr, nullptr, &ms);
                if (st == RCPSP_OK) st = rcpsp_search_results(s, &r, hip_stream);
                const int Lused = s->L;
                rcpsp_search_destroy(s);
                if (st != RCPSP_OK) return st;
                ++trials;
                const double ns = r.total_evaluations > 0 ? ms * 1e6 / (double)r.total_evaluations : ms * 1e6;
                if (!found || ns < best_ns) {
                    found = true;
                    best_ns = ns;
                    best = *params;
                    best.eval = ev;
                    best.threads = T;
                    best.lanes = G;
                    best.lane_profile = lp;
                    best.profile_len = (ev == kEvalTime && lp == 1) ? Lused : 0;
                }
            }
        }
      }
    }
    // one time-indexed candidate per wave
    const bool wave_ok = std::find(evals.begin(), evals.end(), kEvalTime) != evals.end() &&
                         (params->lanes == 0 || params->lanes == kLayoutWave) &&
                         (params->threads == 0 || params->threads == kWaveThreads) && !params->profile_len &&
                         params->lane_profile != 2;
    if (wave_ok) {
        rcpsp_search_params q = *params;
        q.eval = kEvalTime;
        q.threads = kWaveThreads;
        q.lanes = kLayoutWave;
        q.lane_profile = 0;
        q.profile_len = 0;
        q.iterations = trial_iterations;
        q.record_trajectory = 0;
        q.count_work = 0;
        rcpsp_search *s = nullptr;
        rcpsp_status st = rcpsp_search_create(inst, &q, hip_stream, &s);
        if (st != RCPSP_OK && st != RCPSP_E_TOO_LARGE) return st;
        if (st == RCPSP_OK) {
            double ms = 0.0;
            rcpsp_search_result r{};
            st = rcpsp_search_run(s, hip_stream);
            if (st == RCPSP_OK) st = rcpsp_search_run_timed(s, hip_stream, nullptr, nullptr, &ms);
            if (st == RCPSP_OK) st = rcpsp_search_results(s, &r, hip_stream);
            rcpsp_search_destroy(s);
            if (st != RCPSP_OK) return st;
            ++trials;
            const double ns = r.total_evaluations > 0 ? ms * 1e6 / (double)r.total_evaluations : ms * 1e6;
            if (!found || ns < best_ns) {
                found = true;
                best_ns = ns;
                best = *params;
                best.eval = kEvalTime;
                best.threads = kWaveThreads;
                best.lanes = kLayoutWave;
                best.lane_profile = 0;
                best.profile_len = 0;
            }
        }
    }
    if (!found) return fail(RCPSP_E_TOO_LARGE, "no decoder/launch shape fits this instance");
    *out = best;
    if (info) {
        info->eval = best.eval;
        info->threads = best.threads;
        info->profile_len = best.profile_len;
        info->lanes = best.lanes;
        info->register_profile = best.lane_profile == 2 ? 1 : 0;
        info->trials = trials;
        info->ns_per_evaluation = best_ns;
    }
    return RCPSP_OK;
}

// ---------------------------------------------------------------------------
// batches

struct rcpsp_batch {
    struct Class {
        int dec = 0, nw = 0, T = 0, G = 1, per_cu = 0, grid = 0, count = 0;
        long long first_tasks = 0;   // search tasks of the first iteration
        size_t lds = 0;
        BatchClassArgs args{};
    };
    std::vector<rcpsp_search *> items;
    std::vector<Class> classes;
    SearchArgs *d_items = nullptr;
    int *d_state = nullptr;        // queues, then per-class epoch and done counters
    long long state_ints = 0;
    std::vector<void *> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" void rcpsp_batch_destroy(rcpsp_batch *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (rcpsp_search *s : b->items) rcpsp_search_destroy(s);
    for (void *v : b->allocs) (void)hipFree(v);
    delete b;
}

rcpsp_status rcpsp::validate_params(const rcpsp_search_params &p) {
    if (p.swap_range < 1 || p.swap_range > kMaxDelta)
        return fail(RCPSP_E_ARG, "swap_range %d outside 1..%d", p.swap_range, kMaxDelta);
    if (p.tabu_len < 1) return fail(RCPSP_E_ARG, "tabu_len must be >= 1");
    if (p.iterations < 0) return fail(RCPSP_E_ARG, "iterations must be >= 0");
    if (p.searches < 1) return fail(RCPSP_E_ARG, "searches must be >= 1");
    if (p.elite < 0) return fail(RCPSP_E_ARG, "elite must be >= 0");
    if (p.phi_max < 0 || p.phi_steps < 0) return fail(RCPSP_E_ARG, "phi_max and phi_steps must be >= 0");
    if (p.eval < 0 || p.eval > 2) return fail(RCPSP_E_ARG, "unknown decoder %d", p.eval);
    if (p.fbi != 0 && p.fbi != 1) return fail(RCPSP_E_ARG, "fbi must be 0 or 1");
    if (p.exchange_every < 0) return fail(RCPSP_E_ARG, "exchange_every must be >= 0");
    if (p.lane_profile < 0 || p.lane_profile > 2) return fail(RCPSP_E_ARG, "lane_profile must be 0, 1 or 2");
    if (p.time_budget_us < 0) return fail(RCPSP_E_ARG, "time_budget_us must be >= 0");
    return RCPSP_OK;
}

// Limit of one dependency wait inside the batch kernel (wall clock, 100 MHz).
constexpr long long kBatchWaitTicks = 20ll * 100 * 1000 * 1000;

static rcpsp_status build_batch(rcpsp_batch *bt, const rcpsp_instance *const *inst, int32_t count,
                                const rcpsp_search_params *params) {
    // per-instance plans (device state only)
    for (int i = 0; i < count; ++i) {
        if (!inst[i]) return fail(RCPSP_E_ARG, "null instance %d", i);
        rcpsp_search_params p = params[i];
        rcpsp_status st = validate_params(p);
        if (st != RCPSP_OK) return st;
        if (p.fbi) return fail(RCPSP_E_ARG, "batch member %d: forward-backward improvement is for search plans only", i);
        if (p.exchange_every > 1 || p.time_budget_us != 0)
            return fail(RCPSP_E_ARG, "batch member %d: batches exchange after every iteration and take no time budget", i);
        if (p.threads == 0) p.threads = p.lanes == kLayoutWave ? kWaveThreads : 64;
        p.count_work = 0;
        // the threads per search (chosen per group by the autotuner) are a
        // preference: a member whose workgroup does not fit takes fewer
        rcpsp_search *s = nullptr;
        for (;;) {
            s = new (std::nothrow) rcpsp_search();
            if (!s) return fail(RCPSP_E_NOMEM, "out of host memory");
            s->inst = inst[i];
            s->p = p;
            s->reserve = kBatchStaticLds;
            st = alloc_plan(s);
            if (st == RCPSP_E_TOO_LARGE && p.lanes == kLayoutWave) {
                // no wave layout for this member: the automatic one
                rcpsp_search_destroy(s);
                p.lanes = 0;
                p.threads = 256;
                continue;
            }
            if (st == RCPSP_E_TOO_LARGE && p.lane_profile == 2) {
                // no register profile for this member: its profile in LDS
                rcpsp_search_destroy(s);
                p.lane_profile = 1;
                continue;
            }
            if (st == RCPSP_E_TOO_LARGE && p.threads > 64) {
                rcpsp_search_destroy(s);
                p.threads = p.threads == 192 ? 128 : p.threads / 2;
                continue;
            }
            break;
        }
        bt->items.push_back(s);
        if (st != RCPSP_OK) return st;
        const int need = 6 * p.searches + 5 * p.elite;
        if (p.elite > 0 && need > s->Ly.cands * s->Ly.per_lane)
            return fail(RCPSP_E_TOO_LARGE, "instance %d: exchange bookkeeping does not fit the workgroup's LDS", i);
    }
    // classes: same decoder, profile width, threads per search and workgroups per CU
    std::vector<std::vector<int>> members;
    for (int i = 0; i < count; ++i) {
        const rcpsp_search *s = bt->items[i];
        const int nw = s->dec == kEvalTime ? s->nw : 1;
        int per_cu = 0;
        HIP_TRY(batch_occupancy(s->T, nw, s->dec, s->G, s->lds, &per_cu));
        if (per_cu < 1) return fail(RCPSP_E_TOO_LARGE, "instance %d: batch workgroup does not fit a CU", i);
        int c = -1;
        for (size_t k = 0; k < bt->classes.size(); ++k) {
            const rcpsp_batch::Class &cl = bt->classes[k];
            if (cl.dec == s->dec && cl.nw == nw && cl.T == s->T && cl.G == s->G && cl.per_cu == per_cu) c = (int)k;
        }
        if (c < 0) {
            rcpsp_batch::Class cl;
            cl.dec = s->dec;
            cl.nw = nw;
            cl.T = s->T;
            cl.G = s->G;
            cl.per_cu = per_cu;
            bt->classes.push_back(cl);
            members.emplace_back();
            c = (int)bt->classes.size() - 1;
        }
        members[c].push_back(i);
        bt->classes[c].lds = std::max(bt->classes[c].lds, s->lds);
    }
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    std::vector<SearchArgs> host_items(count);
    for (int i = 0; i < count; ++i) host_items[i] = bt->items[i]->a;
    void *v = nullptr;
    HIP_TRY(hipMalloc(&v, sizeof(SearchArgs) * std::max(count, 1)));
    bt->allocs.push_back(v);
    bt->d_items = static_cast<SearchArgs *>(v);
    HIP_TRY(hipMemcpy(bt->d_items, host_items.data(), sizeof(SearchArgs) * count, hipMemcpyHostToDevice));
    // counters: the queues first (aligned), then epoch and done per class
    const int nc = (int)bt->classes.size();
    const long long qints = (long long)(batch_queue_bytes() / sizeof(int)) * nc;
    bt->state_ints = qints + 2ll * count;
    HIP_TRY(hipMalloc(&v, sizeof(int) * bt->state_ints));
    bt->allocs.push_back(v);
    bt->d_state = static_cast<int *>(v);
    long long cursor = qints;
    auto steps_of = [&](int i) {
        const rcpsp_search_params &p = bt->items[i]->p;
        return p.elite > 0 ? std::max(p.iterations, 1) : 1;
    };
    for (int c = 0; c < nc; ++c) {
        rcpsp_batch::Class &cl = bt->classes[c];
        std::vector<int> &m = members[c];
        // members with more iterations first (those of an iteration are a
        // prefix), larger searches first within equal iteration counts
        std::stable_sort(m.begin(), m.end(), [&](int x, int y) {
            const int sx = steps_of(x), sy = steps_of(y);
            if (sx != sy) return sx > sy;
            const rcpsp_search *a = bt->items[x], *b = bt->items[y];
            return (long long)a->inst->n * a->p.searches > (long long)b->inst->n * b->p.searches;
        });
        cl.count = (int)m.size();
        const int max_steps = steps_of(m[0]);
        std::vector<int> cumB(cl.count + 1, 0), act(max_steps, 0);
        for (int j = 0; j < cl.count; ++j) cumB[j + 1] = cumB[j] + bt->items[m[j]]->p.searches;
        for (int j = 0; j < cl.count; ++j)
            for (int it = 0; it < steps_of(m[j]); ++it) act[it] = j + 1;
        cl.first_tasks = max_steps > 0 ? cumB[act[0]] : 0;
        std::vector<long long> off(max_steps + 1);
        off[0] = cl.count;
        for (int it = 0; it < max_steps; ++it) off[it + 1] = off[it] + cumB[act[it]];
        BatchClassArgs &A = cl.args;
        A.items = bt->d_items;
        A.count = cl.count;
        A.max_steps = max_steps;
        A.total = off[max_steps];
        A.wait_ticks = kBatchWaitTicks;
        int *d_order = nullptr, *d_cumB = nullptr, *d_act = nullptr;
        long long *d_off = nullptr;
        HIP_TRY(hipMalloc(&v, sizeof(int) * m.size()));
        bt->allocs.push_back(v);
        d_order = static_cast<int *>(v);
        HIP_TRY(hipMemcpy(d_order, m.data(), sizeof(int) * m.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&v, sizeof(int) * cumB.size()));
        bt->allocs.push_back(v);
        d_cumB = static_cast<int *>(v);
        HIP_TRY(hipMemcpy(d_cumB, cumB.data(), sizeof(int) * cumB.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&v, sizeof(int) * act.size()));
        bt->allocs.push_back(v);
        d_act = static_cast<int *>(v);
        HIP_TRY(hipMemcpy(d_act, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMalloc(&v, sizeof(long long) * off.size()));
        bt->allocs.push_back(v);
        d_off = static_cast<long long *>(v);
        HIP_TRY(hipMemcpy(d_off, off.data(), sizeof(long long) * off.size(), hipMemcpyHostToDevice));
        A.order = d_order;
        A.cumB = d_cumB;
        A.act = d_act;
        A.off = d_off;
        A.q = reinterpret_cast<BatchQueue *>(reinterpret_cast<char *>(bt->d_state) + c * batch_queue_bytes());
        A.epoch = bt->d_state + cursor;
        A.done = bt->d_state + cursor + cl.count;
        cursor += 2ll * cl.count;
        HIP_TRY(prepare_batch(cl.T, cl.nw, cl.dec, cl.G, cl.lds));
    }
    for (int c = 0; c < nc; ++c) {
        rcpsp_batch::Class &cl = bt->classes[c];
        cl.grid = (int)std::min<long long>(cl.args.total, (long long)cl.per_cu * cus);
    }
    // one graph: clear the counters, then every class's persistent launch on
    // its own branch so that the classes run side by side
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    std::vector<hipStream_t> side(bt->classes.size());
    std::vector<hipEvent_t> evs;
    for (auto &x : side) HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    auto cleanup = [&]() {
        for (auto x : side) (void)hipStreamDestroy(x);
        for (auto e : evs) (void)hipEventDestroy(e);
        (void)hipStreamDestroy(cs);
    };
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_fill_zero(bt->d_state, bt->state_ints, cs);
    hipEvent_t fork = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) {
        evs.push_back(fork);
        e = hipEventRecord(fork, cs);
    }
    for (size_t c = 0; e == hipSuccess && c < bt->classes.size(); ++c) {
        const rcpsp_batch::Class &cl = bt->classes[c];
        hipEvent_t done = nullptr;
        e = hipStreamWaitEvent(side[c], fork, 0);
        if (e == hipSuccess) e = launch_batch(cl.args, cl.grid, cl.T, cl.nw, cl.dec, cl.G, cl.lds, side[c]);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
        if (e == hipSuccess) {
            evs.push_back(done);
            e = hipEventRecord(done, side[c]);
        }
        if (e == hipSuccess) e = hipStreamWaitEvent(cs, done, 0);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    cleanup();
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(RCPSP_E_DEVICE, "batch graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    bt->graph = g;
    HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
    return RCPSP_OK;
}

// Whether a run of the batch ended early (a dependency wait hit its limit).
static rcpsp_status batch_check(rcpsp_batch *b, hipStream_t st) {
    const size_t qb = batch_queue_bytes() * b->classes.size();
    std::vector<char> q(qb);
    HIP_TRY(hipMemcpyAsync(q.data(), b->d_state, qb, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (size_t c = 0; c < b->classes.size(); ++c) {
        int abort = 0;
        std::memcpy(&abort, q.data() + c * batch_queue_bytes() + sizeof(unsigned long long), sizeof(int));
        if (abort) return fail(RCPSP_E_DEVICE, "batch class %d: a dependency wait exceeded its limit", (int)c);
    }
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_batch_create(const rcpsp_instance *const *inst, int32_t count,
                                           const rcpsp_search_params *params, void *hip_stream,
                                           rcpsp_batch **out) {
    if (!inst || !params || !out || count < 1) return fail(RCPSP_E_ARG, "null pointer or empty batch");
    *out = nullptr;
    rcpsp_batch *bt = new (std::nothrow) rcpsp_batch();
    if (!bt) return fail(RCPSP_E_NOMEM, "out of host memory");
    rcpsp_status st = build_batch(bt, inst, count, params);
    if (st != RCPSP_OK) {
        rcpsp_batch_destroy(bt);
        return st;
    }
    (void)hip_stream;
    *out = bt;
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_batch_run(rcpsp_batch *b, void *hip_stream) {
    if (!b) return fail(RCPSP_E_ARG, "null batch");
    HIP_TRY(hipGraphLaunch(b->exec, (hipStream_t)hip_stream));
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_batch_run_timed(rcpsp_batch *b, void *hip_stream, double *total_ms) {
    if (!b) return fail(RCPSP_E_ARG, "null batch");
    hipStream_t st = (hipStream_t)hip_stream;
    hipEvent_t t0, t1;
    HIP_TRY(hipEventCreate(&t0));
    HIP_TRY(hipEventCreate(&t1));
    hipError_t e = hipEventRecord(t0, st);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
    if (e == hipSuccess) e = hipEventRecord(t1, st);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return fail(RCPSP_E_DEVICE, "timed batch run: %s", hipGetErrorString(e));
    if (total_ms) *total_ms = ms;
    return batch_check(b, st);
}

extern "C" rcpsp_status rcpsp_batch_results(rcpsp_batch *b, int32_t index, rcpsp_search_result *res,
                                            void *hip_stream) {
    if (!b || !res) return fail(RCPSP_E_ARG, "null pointer");
    if (index < 0 || index >= (int32_t)b->items.size()) return fail(RCPSP_E_ARG, "index %d out of range", index);
    rcpsp_status st = batch_check(b, (hipStream_t)hip_stream);
    if (st != RCPSP_OK) return st;
    return rcpsp_search_results(b->items[index], res, hip_stream);
}

extern "C" rcpsp_status rcpsp_batch_get_info(const rcpsp_batch *b, rcpsp_batch_info *out) {
    if (!b || !out) return fail(RCPSP_E_ARG, "null pointer");
    *out = rcpsp_batch_info{};
    out->instances = (int32_t)b->items.size();
    out->classes = (int32_t)b->classes.size();
    for (size_t c = 0; c < b->classes.size() && c < 8; ++c) {
        out->class_eval[c] = b->classes[c].dec;
        out->class_threads[c] = b->classes[c].T;
        out->class_instances[c] = b->classes[c].count;
        out->class_workgroups[c] = b->classes[c].grid;
        out->class_lds_bytes[c] = (int32_t)b->classes[c].lds;
    }
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_batch_autotune(const rcpsp_instance *const *inst, int32_t count,
                                            const rcpsp_search_params *params, int32_t trial_iterations,
                                            int32_t sample, void *hip_stream, rcpsp_search_params *out,
                                            rcpsp_batch_tuning *info) {
    if (!inst || !params || !out || count < 1) return fail(RCPSP_E_ARG, "null pointer or empty batch");
    if (trial_iterations < 1 || sample < 1) return fail(RCPSP_E_ARG, "trial_iterations and sample must be >= 1");
    for (int i = 0; i < count; ++i)
        if (!inst[i]) return fail(RCPSP_E_ARG, "null instance %d", i);
    // groups by (N, M, dwords per time-indexed unit), in order of first
    // appearance: members whose units take more words cannot share the
    // register profiles of the others and are timed on their own
    static_assert(kMaxNW < 8, "M and the words per unit share one key");
    std::vector<std::pair<int, int>> keys;
    std::vector<std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
        const std::pair<int, int> k(inst[i]->n, inst[i]->m * 8 + inst[i]->desc.nw);
        size_t g = 0;
        while (g < keys.size() && keys[g] != k) ++g;
        if (g == keys.size()) {
            keys.push_back(k);
            groups.emplace_back();
        }
        groups[g].push_back(i);
        out[i] = params[i];
    }
    if (info) *info = rcpsp_batch_tuning{};
    int trials = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        const std::vector<int> &mem = groups[g];
        const int ns = std::min<int>(sample, (int)mem.size());
        std::vector<const rcpsp_instance *> si(ns);
        std::vector<rcpsp_search_params> sp(ns);
        for (int k = 0; k < ns; ++k) {
            const int i = mem[(size_t)k * mem.size() / ns];
            si[k] = inst[i];
            sp[k] = params[i];
            sp[k].iterations = trial_iterations;
            sp[k].record_trajectory = 0;
            sp[k].count_work = 0;
        }
        const rcpsp_search_params &p0 = params[mem[0]];
        bool time_ok = true;
        for (int k = 0; k < ns; ++k) time_ok = time_ok && si[k]->desc.nw > 0;
        std::vector<int> evals, threads;
        if (p0.eval) evals.push_back(p0.eval);
        else {
            if (time_ok) evals.push_back(kEvalTime);
            evals.push_back(kEvalCapacity);
        }
        if (p0.threads) threads.push_back(p0.threads);
        else threads = {64, 128, 192, 256};
        std::vector<int> lanes_c;
        if (p0.lanes) lanes_c.push_back(p0.lanes);
        else lanes_c = {1, 8, 16, kLayoutWave};
        std::vector<int> lps;
        if (p0.lane_profile) lps.push_back(p0.lane_profile);
        else lps = {1, 2};
        // register profiles where a member's time unit packs into one dword
        // (the batch keeps the others in LDS): a candidate when any does
        bool nw1 = false;
        for (int k = 0; k < ns; ++k) nw1 = nw1 || si[k]->desc.nw == 1;
        bool found = false;
        double best_rate = 0.0;
        int best_eval = 0, best_T = 0, best_G = 1, best_lp = 1;
        for (int ev : evals) {
          for (int G : lanes_c) {
            if ((G == 16 && ev != kEvalTime) || (G == 8 && ev != kEvalCapacity)) continue;
            if (G == kLayoutWave && (ev != kEvalTime || (p0.threads && p0.threads != kWaveThreads))) continue;
            // one candidate per wave: its own thread count, no lane profile choice
            std::vector<int> Ts = G == kLayoutWave ? std::vector<int>{kWaveThreads} : threads;
            if (G == 8 && !p0.threads) Ts.push_back(512);
            const std::vector<int> lps_g = G == kLayoutWave ? std::vector<int>{0} : lps;
            for (int T : Ts)
            for (int lp : lps_g) {
                if (T == 512 && G != kLayoutWave && G != 8) continue;
                if (T == 192 && (ev != kEvalTime || G != 1)) continue;
                if (lp == 2 && (ev != kEvalTime || G != 1 || T != 256 || !nw1)) continue;
                for (auto &q : sp) {
                    q.eval = ev;
                    q.threads = T;
                    q.lanes = G;
                    q.lane_profile = lp;
                }
                rcpsp_batch *bt = nullptr;
                rcpsp_status st = rcpsp_batch_create(si.data(), ns, sp.data(), hip_stream, &bt);
                if (st == RCPSP_E_TOO_LARGE) continue;
                if (st != RCPSP_OK) return st;
                double ms = 0.0;
                long long ev_total = 0;
                st = rcpsp_batch_run(bt, hip_stream);
                if (st == RCPSP_OK) st = rcpsp_batch_run_timed(bt, hip_stream, &ms);
                for (int k = 0; st == RCPSP_OK && k < ns; ++k) {
                    rcpsp_search_result r{};
                    st = rcpsp_batch_results(bt, k, &r, hip_stream);
                    ev_total += r.total_evaluations;
                }
                rcpsp_batch_destroy(bt);
                if (st != RCPSP_OK) return st;
                ++trials;
                const double rate = ms > 0.0 ? (double)ev_total / (ms * 1e-3) : 0.0;
                if (!found || rate > best_rate) {
                    found = true;
                    best_rate = rate;
                    best_eval = ev;
                    best_T = T;
                    best_G = G;
                    best_lp = lp;
                }
            }
          }
        }
        if (!found) return fail(RCPSP_E_TOO_LARGE, "no decoder/threads candidate fits instances of N=%d, M=%d",
                                keys[g].first, keys[g].second / 8);
        for (int i : mem) {
            out[i].eval = best_eval;
            out[i].threads = best_T;
            out[i].lanes = best_G;
            out[i].lane_profile = best_lp;
        }
        if (info && g < 8) {
            info->group_n[g] = keys[g].first;
            info->group_m[g] = keys[g].second / 8;
            info->group_members[g] = (int32_t)mem.size();
            info->group_eval[g] = best_eval;
            info->group_threads[g] = best_T;
            info->group_lanes[g] = best_G;
            info->group_register[g] = best_lp == 2 ? 1 : 0;
            info->group_evals_per_s[g] = best_rate;
        }
    }
    if (info) {
        info->groups = (int32_t)groups.size();
        info->trials = trials;
    }
    return RCPSP_OK;
}

extern "C" rcpsp_status rcpsp_tabu_search_batch(const rcpsp_instance *const *inst, int32_t count,
                                                const rcpsp_search_params *per_inst, rcpsp_search_result *out,
                                                void *hip_stream) {
    if (!inst || !per_inst || !out) return fail(RCPSP_E_ARG, "null pointer");
    if (count < 1) return fail(RCPSP_E_ARG, "count must be >= 1");
    rcpsp_batch *b = nullptr;
    rcpsp_status st = rcpsp_batch_create(inst, count, per_inst, hip_stream, &b);
    if (st != RCPSP_OK) return st;
    st = rcpsp_batch_run(b, hip_stream);
    for (int i = 0; st == RCPSP_OK && i < count; ++i) st = rcpsp_batch_results(b, i, &out[i], hip_stream);
    rcpsp_batch_destroy(b);
    return st;
}
