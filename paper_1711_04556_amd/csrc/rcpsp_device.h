// Device code of the HIP kernels for gfx950 (included by the kernel
// translation units, each of which instantiates and launches a part of them):
// swap-neighbourhood evaluation with the serial schedule generation scheme,
// and the tabu search built on it.
//
// Design (one workgroup per search, wave64):
//  - the instance (durations, packed requests, precedence lists) is staged
//    from one device blob into LDS once per launch;
//  - feasible moves are found in O(1) each: with a feasible order, eq. 5
//    holds for swap(u,v) iff v is before the first successor of w_u, and
//    eq. 6 iff u is after the last predecessor of w_v (Section 4.3-4.4);
//  - every lane decodes one candidate order with Alg. 7.  Its private state
//    (finish times, resource profile or capacity arrays) sits in LDS with a
//    lane-interleaved layout (dword i of lane l at i*T+l), so lanes never
//    conflict on a bank;
//  - the time-indexed profile packs all resources of one time unit into one
//    or more dwords (8- or 16-bit fields whose top bit, the guard, is kept
//    set in every stored unit), so the capacity test of Alg. 5 for all
//    resources is one subtract and mask (a field short of capacity borrows
//    its guard), and Alg. 6 is one subtract;
//  - the best admissible move is a 64-bit key (non-admissible, C_max, u, v)
//    reduced with cross-lane shuffles inside a wave and LDS across waves.
#pragma once

#include <hip/hip_runtime.h>

#include "rcpsp_internal.h"
#include "rcpsp_launch.h"

namespace rcpsp {

// ---------------------------------------------------------------------------
// LDS views

struct Sh {
    const uint16_t *dur, *predoff, *pred, *succoff, *succ, *reqk, *base, *lvl;
    const uint32_t *rq, *res;
    uint16_t *W, *Wimp, *pos, *fs, *lp;
    int *cnt;
    uint32_t *tc, *ring, *moves, *prec, *prq, *predT, *pin, *pid, *bst;
    unsigned long long *red;
    int *scal;
    uint32_t *region;
};

__device__ inline Sh make_sh(uint32_t *lds, const InstDesc &D, const Layout &Ly) {
    Sh s;
    uint32_t *b = lds + Ly.blob;
    s.dur = reinterpret_cast<const uint16_t *>(b + D.off_dur);
    s.predoff = reinterpret_cast<const uint16_t *>(b + D.off_predoff);
    s.pred = reinterpret_cast<const uint16_t *>(b + D.off_pred);
    s.succoff = reinterpret_cast<const uint16_t *>(b + D.off_succoff);
    s.succ = reinterpret_cast<const uint16_t *>(b + D.off_succ);
    s.reqk = reinterpret_cast<const uint16_t *>(b + D.off_reqk);
    s.base = reinterpret_cast<const uint16_t *>(b + D.off_base);
    s.lvl = reinterpret_cast<const uint16_t *>(b + D.off_lvl);
    s.rq = b + D.off_rq;
    s.res = b + D.off_res;
    s.W = reinterpret_cast<uint16_t *>(lds + Ly.W);
    s.Wimp = reinterpret_cast<uint16_t *>(lds + Ly.Wimp);
    s.pos = reinterpret_cast<uint16_t *>(lds + Ly.pos);
    s.fs = reinterpret_cast<uint16_t *>(lds + Ly.fs);
    s.lp = reinterpret_cast<uint16_t *>(lds + Ly.lp);
    s.cnt = reinterpret_cast<int *>(lds + Ly.cnt);
    s.tc = lds + Ly.tc;
    s.ring = lds + Ly.ring;
    s.moves = lds + Ly.moves;
    s.prec = lds + Ly.prec;
    s.prq = lds + Ly.prq;
    s.predT = lds + Ly.predT;
    s.pin = Ly.pin ? lds + Ly.pin : nullptr;
    s.pid = Ly.pid ? lds + Ly.pid : nullptr;
    s.bst = lds + Ly.bst;
    s.red = reinterpret_cast<unsigned long long *>(lds + Ly.red);
    s.scal = reinterpret_cast<int *>(lds + Ly.scal);
    s.region = lds + Ly.region;
    return s;
}

template <int T>
__device__ inline void stage_blob(uint32_t *lds, const InstDesc &D, const Layout &Ly) {
    for (int i = threadIdx.x; i < D.blob_dwords; i += T) lds[Ly.blob + i] = D.blob[i];
}

// Lane-private storage: dword i at base[i*STRIDE]; 16-bit element e in dword e>>1.
template <int STRIDE>
struct LaneMem {
    uint32_t *base;
    __device__ inline uint32_t ld(int i) const { return base[i * STRIDE]; }
    __device__ inline void st(int i, uint32_t v) const { base[i * STRIDE] = v; }
    __device__ inline int ld16(int e) const {
        return reinterpret_cast<const uint16_t *>(base + (e >> 1) * STRIDE)[e & 1];
    }
    __device__ inline void st16(int e, int v) const {
        reinterpret_cast<uint16_t *>(base + (e >> 1) * STRIDE)[e & 1] = (uint16_t)v;
    }
    // 16-bit element at a precomputed byte offset from this lane's dword 0
    __device__ inline int ld16b(uint32_t off) const {
        return *reinterpret_cast<const uint16_t *>(reinterpret_cast<const char *>(base) + off);
    }
    __device__ inline void st16b(uint32_t off, int v) const {
        *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(base) + off) = (uint16_t)v;
    }
    // finish time of FB bits (8 or 16) at a byte offset
    template <int FB>
    __device__ inline int ldf(uint32_t off) const {
        if (FB == 8) return *(reinterpret_cast<const uint8_t *>(base) + off);
        return ld16b(off);
    }
    template <int FB>
    __device__ inline void stf(uint32_t off, int v) const {
        if (FB == 8) *(reinterpret_cast<uint8_t *>(base) + off) = (uint8_t)v;
        else st16b(off, v);
    }
};

// Dwords of finish times (FB bits each) at the start of a candidate's state.
template <int FB>
__host__ __device__ inline int f_dwords(int n) {
    return finish_dwords(n, FB);
}

// Byte offset of 16-bit element e of a lane's storage when lanes are
// interleaved with the given dword stride (stride 1: a single thread).
template <int STRIDE>
__device__ inline uint32_t off16(int e) {
    return (uint32_t)(((e >> 1) * STRIDE) << 2) + (uint32_t)((e & 1) << 1);
}

// Byte offset of finish time e (FB bits) in a lane's storage.
template <int STRIDE, int FB>
__device__ inline uint32_t offF(int e) {
    if (FB == 8) return (uint32_t)(((e >> 2) * STRIDE) << 2) + (uint32_t)(e & 3);
    return off16<STRIDE>(e);
}

// ---------------------------------------------------------------------------
// Random numbers: counter-based SplitMix64 (Steele, Lea & Flood 2014).

__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline uint32_t rng_below(uint64_t seed, uint64_t stream, uint64_t i, uint32_t n) {
    const uint64_t G = 0x9E3779B97F4A7C15ull;
    uint64_t key = mix64(seed + (stream + 1) * G);
    uint64_t x = mix64(key + (i + 1) * G);
    return (uint32_t)(((x >> 32) * (uint64_t)n) >> 32);
}

// ---------------------------------------------------------------------------
// Workgroup primitives

template <int T>
__device__ inline int block_excl_scan(int x, int *total, int *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < T / 64; ++i) {
            int t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[T / 64] = acc;
    }
    __syncthreads();
    int r = incl - x + sh[w];
    *total = sh[T / 64];
    __syncthreads();
    return r;
}

template <int T>
__device__ inline unsigned long long block_min_u64(unsigned long long x, unsigned long long *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < T / 64; ++i) x = red[i] < x ? red[i] : x;
        red[0] = x;
    }
    __syncthreads();
    x = red[0];
    __syncthreads();
    return x;
}

// ---------------------------------------------------------------------------
// Neighbourhood (Sections 4.2-4.4)

// Per-position records of the current order W, one 16-byte load each:
//   prec[4p..4p+3] = (byte offset of f[w_p] in a lane's storage, d | npred << 16,
//                     first predecessor index, w_p),
//   prq[p*NW + w]  = packed requests of w_p (time-indexed profile words),
//   predT[e]       = byte offset of f[pred[e]] in a lane's storage,
//   pin[4p..4p+3]  = the same offsets for the first four predecessors of w_p
//                    (one 16-byte load; present for one-candidate-per-lane
//                    time-indexed layouts only); absent predecessors get
//                    offset 0, the finish time of the source activity (0);
//   pid[2p..2p+1]  = the ids of the first four predecessors of w_p, 16 bits
//                    each (one 8-byte load; one-candidate-per-wave layout
//                    only), absent ones the source activity 0.
template <int T, int FB = 16>
__device__ inline void build_records(const Sh &S, const InstDesc &D) {
    const int N = D.n, NW = D.nw;
    for (int p = threadIdx.x; p < N; p += T) {
        const int a = S.W[p];
        const int po = S.predoff[a];
        uint4 r;
        r.x = offF<T, FB>(a);
        r.y = (uint32_t)S.dur[a] | ((uint32_t)(S.predoff[a + 1] - po) << 16);
        r.z = (uint32_t)po;
        r.w = (uint32_t)a;
        reinterpret_cast<uint4 *>(S.prec)[p] = r;
        for (int w = 0; w < NW; ++w) S.prq[p * NW + w] = S.rq[a * NW + w];
    }
    for (int e = threadIdx.x; e < D.n_arcs; e += T) S.predT[e] = offF<T, FB>(S.pred[e]);
    if (S.pin) {
        for (int p = threadIdx.x; p < N; p += T) {
            const int a = S.W[p];
            const int po = S.predoff[a], np = S.predoff[a + 1] - po;
            uint32_t o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = k < np ? offF<T, FB>(S.pred[po + k]) : 0u;
            reinterpret_cast<uint4 *>(S.pin)[p] = make_uint4(o[0], o[1], o[2], o[3]);
        }
    }
    if (S.pid) {
        for (int p = threadIdx.x; p < N; p += T) {
            const int a = S.W[p];
            const int po = S.predoff[a], np = S.predoff[a + 1] - po;
            uint32_t o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) o[k] = k < np ? (uint32_t)S.pred[po + k] : 0u;
            reinterpret_cast<uint2 *>(S.pid)[p] = make_uint2(o[0] | (o[1] << 16), o[2] | (o[3] << 16));
        }
    }
}

// Position of the first successor / last predecessor of each w_p, then the
// feasible swaps in canonical order (u ascending, v ascending).  Returns the
// number of feasible moves (uniform across the workgroup).
// Positions of W, then for each position the first successor and the last
// predecessor position (stored +1; 0 = none).
template <int T>
__device__ inline void order_bounds(const Sh &S, const InstDesc &D) {
    const int N = D.n, tid = threadIdx.x;
    for (int p = tid; p < N; p += T) S.pos[S.W[p]] = (uint16_t)p;
    __syncthreads();
    for (int p = tid; p < N; p += T) {
        const int a = S.W[p];
        int fsv = N, lpv = 0;
        for (int e = S.succoff[a]; e < S.succoff[a + 1]; ++e) fsv = min(fsv, (int)S.pos[S.succ[e]]);
        for (int e = S.predoff[a]; e < S.predoff[a + 1]; ++e) lpv = max(lpv, (int)S.pos[S.pred[e]] + 1);
        S.fs[p] = (uint16_t)fsv;
        S.lp[p] = (uint16_t)lpv;
    }
    __syncthreads();
}

// One random feasible swap of W (the diversification of Section 6.1): the
// move of index j in canonical order, j drawn uniformly below the number of
// feasible moves, exactly as build_moves lists them; only the thread whose
// range of u holds j enumerates its moves again.  Returns the number of
// feasible moves (0: W is left as it is).
template <int T>
__device__ int random_swap(const Sh &S, const InstDesc &D, int delta, uint64_t seed, uint64_t stream,
                           unsigned long long *ctr) {
    const int N = D.n, tid = threadIdx.x;
    order_bounds<T>(S, D);
    const int nu = N - 2;
    const int ch = (nu + T - 1) / T;
    const int u0 = 1 + tid * ch, u1 = min(u0 + ch, N - 1);
    int c = 0;
    for (int u = u0; u < u1; ++u) {
        const int vmax = min(min(u + delta, N - 2), (int)S.fs[u] - 1);
        for (int v = u + 1; v <= vmax; ++v) c += (S.lp[v] <= u);
    }
    int total;
    const int off = block_excl_scan<T>(c, &total, S.cnt);
    if (total == 0) return 0;
    int *shj = S.cnt + T / 64 + 1;
    if (tid == 0) *shj = (int)rng_below(seed, stream, (*ctr)++, (uint32_t)total);
    __syncthreads();
    const int j = *shj;
    if (j >= off && j < off + c) {
        int k = off;
        for (int u = u0; u < u1; ++u) {
            const int vmax = min(min(u + delta, N - 2), (int)S.fs[u] - 1);
            for (int v = u + 1; v <= vmax; ++v) {
                if (S.lp[v] <= u) {
                    if (k == j) {
                        const uint16_t t = S.W[u];
                        S.W[u] = S.W[v];
                        S.W[v] = t;
                    }
                    ++k;
                }
            }
        }
    }
    __syncthreads();
    return total;
}

template <int T, int FB = 16>
__device__ int build_moves(const Sh &S, const InstDesc &D, int delta) {
    const int N = D.n, tid = threadIdx.x;
    build_records<T, FB>(S, D);
    order_bounds<T>(S, D);
    const int nu = N - 2;
    const int ch = (nu + T - 1) / T;
    const int u0 = 1 + tid * ch, u1 = min(u0 + ch, N - 1);
    int c = 0;
    for (int u = u0; u < u1; ++u) {
        const int vmax = min(min(u + delta, N - 2), (int)S.fs[u] - 1);
        for (int v = u + 1; v <= vmax; ++v) c += (S.lp[v] <= u);
    }
    int total;
    int off = block_excl_scan<T>(c, &total, S.cnt);
    for (int u = u0; u < u1; ++u) {
        const int vmax = min(min(u + delta, N - 2), (int)S.fs[u] - 1);
        for (int v = u + 1; v <= vmax; ++v)
            if (S.lp[v] <= u) S.moves[off++] = (uint32_t)u | ((uint32_t)v << 16);
    }
    __syncthreads();
    return total;
}

// Canonical index of swap(u,v) among all potential moves.
__device__ inline int canon_index(int N, int delta, int u, int v) {
    const int Lp = N - 2;
    const int dd = min(delta, Lp - 1);
    int cum;
    if (u - 1 <= Lp - dd) {
        cum = (u - 1) * dd;
    } else {
        cum = (Lp - dd) * dd + ((dd - 1) * dd) / 2 - ((Lp - u) * (Lp - u + 1)) / 2;
    }
    return cum + (v - u - 1);
}

// Key of a decoded move: non-admissible moves sort after admissible ones,
// then (C_max, u, v) lexicographically.
__device__ inline unsigned long long move_key(int c, int u, int v, bool tabu, int asp) {
    const bool adm = !tabu || c < asp;
    return ((unsigned long long)(adm ? 0u : 1u) << 63) | ((unsigned long long)(uint32_t)c << 32) |
           ((unsigned long long)(uint32_t)u << 16) | (unsigned long long)(uint32_t)v;
}

__device__ inline bool tc_get(const uint32_t *tc, int tcw, int u, int v) {
    const int o = v - u - 1;
    return (tc[u * tcw + (o >> 5)] >> (o & 31)) & 1u;
}

struct TabuSrc {
    const uint32_t *tc;     // LDS tabu cache bits or null
    const uint8_t *bytes;   // global N*N bytes or null
    int tcw, n;
    __device__ inline bool get(int u, int v) const {
        if (tc) return tc_get(tc, tcw, u, v);
        if (bytes) return bytes[u * n + v] != 0;
        return false;
    }
};


template <int T>
__device__ inline long long block_sum_i64(long long x, unsigned long long *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (unsigned long long)x;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < T / 64; ++i) x += (long long)red[i];
        red[0] = (unsigned long long)x;
    }
    __syncthreads();
    x = (long long)red[0];
    __syncthreads();
    return x;
}


// ---------------------------------------------------------------------------
// Schedule decoders (Section 5).  The candidate order is W with positions u
// and v exchanged (u = v = 0 decodes W itself).  Finish times s_a + d_a are
// kept per activity; C_max is the finish time of the end dummy N-1.
//
// A decode covers positions [p0, p1) and continues from the state the caller
// holds for positions [0, p0) (finish times, resource state, `front`).  All
// candidates of one round share the prefix of W before their smallest u, so
// that prefix is decoded once (Alg. 7 places activities in list order, and
// the state after a list prefix depends on that prefix only).

// es_prec: the latest finish time among the predecessors (two reads in
// flight).  Lane decodes read the precomputed offsets predT, single-thread
// decodes (stride 1) the predecessor ids.
template <int STRIDE, int FB = 16>
__device__ inline int prec_earliest(const Sh &S, const LaneMem<STRIDE> &M, int po, int np) {
    int es = 0;
    for (int e = 0; e < np; e += 2) {
        const int e1 = (e + 1 < np) ? e + 1 : e;
        uint32_t o0, o1;
        if (STRIDE == 1) {
            o0 = (FB / 8) * (uint32_t)S.pred[po + e];
            o1 = (FB / 8) * (uint32_t)S.pred[po + e1];
        } else {
            o0 = S.predT[po + e];
            o1 = S.predT[po + e1];
        }
        es = max(es, max(M.template ldf<FB>(o0), M.template ldf<FB>(o1)));
    }
    return es;
}

// Time-indexed: Alg. 5 scans for the first d consecutive time units at or
// after es_prec with enough capacity on every resource; Alg. 6 subtracts the
// requests over [s, s+d).  Only the first L time units are held (the lane's
// storage has L+4 so the scan may read four units at a time); a candidate
// whose schedule would pass L reports overflow and is decoded again with a
// longer profile.  Time units at or beyond `front` have never been used and
// stand for the full capacity, so a scan that reaches `front` ends there; the
// four units from `front` on are kept at the full capacity (set at entry,
// then by every Alg. 6 that moves the frontier), so a step reading past the
// frontier needs no test of its own.  Each
// scan step tests four units with selects only, so their loads are in
// flight together.  Alg. 6 is a fill of never-written units up to s + d with
// the full capacity, then LDS atomic subtractions: neither waits for a
// returned value.  The record of the next position is loaded while the
// current one is placed, and one-candidate-per-lane layouts read the first
// four predecessor offsets in one load; the work done stays that of Alg. 5
// and 6.
// With COUNT, *wk receives the decode's algorithmic operations: one per
// activity, one per predecessor read, one per time unit examined by Alg. 5
// and one per time unit updated by Alg. 6 (d of each for an activity that
// requests nothing).
// Algorithmic work of decodes (counting kernels only): operations (see
// each decoder) and the resource-state cells among them (time-indexed:
// profile time units examined by Alg. 5 or updated by Alg. 6;
// capacity-indexed: eq. 7 lookups and Alg. 4 loop steps).
struct Work {
    long long ops, cells;
    __device__ inline void add(const Work &o) {
        ops += o.ops;
        cells += o.cells;
    }
};

__device__ inline void lds_sub(uint32_t *p, uint32_t x) {
    __hip_atomic_fetch_sub(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int NW, int STRIDE, bool COUNT = false, int FB = 16>
__device__ int decode_ti(const Sh &S, const InstDesc &D, uint32_t *lane_base, int L, int u, int v, int p0, int p1,
                         int &front, bool &ovf, Work *wk = nullptr) {
    LaneMem<STRIDE> M{lane_base};
    const int F0 = f_dwords<FB>(D.n);
    uint32_t G[NW], FULL[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        G[w] = D.guard[w];
        FULL[w] = D.full[w];
    }
    constexpr bool kPin = STRIDE > 1;
    const uint4 *rec = reinterpret_cast<const uint4 *>(S.prec);
    const uint4 *pin = reinterpret_cast<const uint4 *>(S.pin);
    uint32_t *prof = lane_base + F0 * STRIDE;   // time unit t, word w at prof[(t*NW + w)*STRIDE]
    long long w_ops = 0, w_cells = 0;
    int fr = front;
    // the positions are the same for every lane of the wave (a shared prefix
    // or none), so the loop over them is scalar; a lane whose schedule passes
    // its profile stays in it (over) instead of leaving it alone
    p0 = __builtin_amdgcn_readfirstlane(p0);
    p1 = __builtin_amdgcn_readfirstlane(p1);
    bool over = false;
    // the source (position 0, duration 0) finishes at 0; the predecessor
    // table reads that slot for absent predecessors, so it is set before
    // anything reads it
    if constexpr (kPin) {
        if (p0 == 0) M.template stf<FB>(0u, 0);
    }
    // units from the frontier on are unused: four of them at the full capacity
    for (int x = fr; x < fr + 4; ++x) {
#pragma unroll
        for (int w = 0; w < NW; ++w) prof[(x * NW + w) * STRIDE] = FULL[w];
    }
    // the record and predecessor offsets of a position (clamped to the last
    // one, so the load one position ahead stays in range)
    auto qof = [&](int p) {
        p = min(p, D.n - 1);
        return (p == u) ? v : ((p == v) ? u : p);
    };
    int q = qof(p0);
    uint4 r = rec[q];
    uint4 pi = kPin ? pin[q] : make_uint4(0u, 0u, 0u, 0u);
    for (int p = p0; p < p1; ++p) {
        // requests: loaded with the predecessors' finish times (no wait of their own)
        uint32_t rq[NW];
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            rq[w] = S.prq[q * NW + w];
            any |= rq[w];
        }
        const int d = r.y & 0xffff, np = r.y >> 16;
        const uint32_t fo = (STRIDE == 1) ? (FB / 8) * r.w : r.x;
        int es;
        if constexpr (kPin) {
            const int f0 = M.template ldf<FB>(pi.x), f1 = M.template ldf<FB>(pi.y);
            const int f2 = M.template ldf<FB>(pi.z), f3 = M.template ldf<FB>(pi.w);
            // entries past the predecessors point to the source's finish time (0)
            es = max(max(f0, f1), max(f2, f3));
            for (int e = 4; e < np; ++e) es = max(es, M.template ldf<FB>(S.predT[r.z + e]));
        } else {
            es = prec_earliest<STRIDE, FB>(S, M, (int)r.z, np);
        }
        // next position's record, loaded while this activity is placed
        const int qn = qof(p + 1);
        const uint4 rn = rec[qn];
        const uint4 pn = kPin ? pin[qn] : make_uint4(0u, 0u, 0u, 0u);
        if (COUNT) w_ops += 1 + np;
        int s = es;
        if (!over && any != 0 && d > 0) {
            int t = es, run = 0;   // run: free units just before t
            int r0 = 0, r1 = 0, r2 = 0, r3 = 0;
            while (t < fr) {
                const uint32_t *P = prof + t * NW * STRIDE;
                bool ok[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    bool o = true;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const uint32_t A = P[(k * NW + w) * STRIDE];
                        o = o && (((A - rq[w]) & G[w]) == G[w]);
                    }
                    ok[k] = o;   // units past the frontier hold the full capacity
                }
                r0 = ok[0] ? run + 1 : 0;
                r1 = ok[1] ? r0 + 1 : 0;
                r2 = ok[2] ? r1 + 1 : 0;
                r3 = ok[3] ? r2 + 1 : 0;
                run = r3;
                t += 4;
                // runs grow by one from below d, so one of them equals d
                // exactly when their maximum reaches it
                if (max(max(r0, r1), max(r2, r3)) >= d) break;
            }
            if (max(max(r0, r1), max(r2, r3)) >= d) {
                // earliest unit of the last step where the run reaches d
                const int tb = t - 4;
                s = (r3 == d) ? tb + 4 - d : -1;
                s = (r2 == d) ? tb + 3 - d : s;
                s = (r1 == d) ? tb + 2 - d : s;
                s = (r0 == d) ? tb + 1 - d : s;
            } else {
                s = t - run;  // reached the frontier: all later units are free
            }
            const int e = s + d;
            if (e > L) {
                // past the lane's profile: the lane only runs along with the
                // wave from here (no more profile access) and reports overflow
                over = true;
            } else {
                if (COUNT) {
                    w_ops += (e - es) + d;
                    w_cells += (e - es) + d;
                }
                // [fr, fr + 4) already hold the full capacity; keep four such
                // units past the new frontier
                // two units per step (half the loop control), then the odd one
                int x = fr + 4;
                for (; x + 1 < e + 4; x += 2) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        prof[(x * NW + w) * STRIDE] = FULL[w];
                        prof[((x + 1) * NW + w) * STRIDE] = FULL[w];
                    }
                }
                if (x < e + 4) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) prof[(x * NW + w) * STRIDE] = FULL[w];
                }
                x = s;
                for (; x + 1 < e; x += 2) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        lds_sub(prof + (x * NW + w) * STRIDE, rq[w]);
                        lds_sub(prof + ((x + 1) * NW + w) * STRIDE, rq[w]);
                    }
                }
                if (x < e) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) lds_sub(prof + (x * NW + w) * STRIDE, rq[w]);
                }
                fr = max(fr, e);
            }
        } else if (COUNT) {
            w_ops += 2 * d;
            w_cells += 2 * d;
        }
        // 8-bit finish times hold at most 255: a later finish (possible for
        // an activity that requests nothing, which never touches the
        // profile) takes the candidate to the long-profile path like a
        // profile overflow
        if constexpr (FB == 8) over = over || (s + d > 255);
        M.template stf<FB>(fo, s + d);
        q = qn;
        r = rn;
        pi = pn;
    }
    if (over) {
        ovf = true;
        return -1;
    }
    front = fr;
    if (COUNT) wk->add(Work{w_ops, w_cells});
    return p1 == D.n ? M.template ldf<FB>(STRIDE == 1 ? (FB / 8) * (uint32_t)(D.n - 1) : offF<STRIDE, FB>(D.n - 1)) : 0;
}

// Capacity-indexed: eq. 7 gives the resource earliest start, the update of
// Section 5.1 (Alg. 4) raises the c_k entries.  c_k holds R_k 16-bit times
// (the time from which each unit is free, non-increasing); the times the
// raised units had before are only read r_ik raises later, so a ring of
// copy_p (a power of two >= every request) entries holds them.  Units free
// only at or after s + d are passed over; before the first raise they form
// a prefix (c_k stays non-increasing because s is never below the eq. 7
// start), which a binary search skips.
// With COUNT, *wk receives one operation per activity, per predecessor read,
// per eq. 7 lookup and per Alg. 4 loop step (skipped steps included).
template <int STRIDE, bool COUNT = false>
__device__ int decode_ci(const Sh &S, const InstDesc &D, uint32_t *lane_base, int u, int v, int p0, int p1,
                         Work *wk = nullptr) {
    LaneMem<STRIDE> M{lane_base};
    const int Mr = D.m;
    const int F0 = (D.n + 1) >> 1;
    const int Cd = (D.sum_r + 1) >> 1;
    const int ce0 = 2 * F0;               // first c_k entry (16-bit element index)
    const int pe0 = 2 * (F0 + Cd);        // first copy ring entry
    const int pmask = D.copy_p - 1;
    const uint4 *rec = reinterpret_cast<const uint4 *>(S.prec);
    long long w_ops = 0, w_cells = 0;
    for (int p = p0; p < p1; ++p) {
        const int q = (p == u) ? v : ((p == v) ? u : p);
        const uint4 r = rec[q];
        const int d = r.y & 0xffff, np = r.y >> 16, a = (int)r.w;
        const uint32_t fo = (STRIDE == 1) ? 2u * r.w : r.x;
        const int es = prec_earliest<STRIDE>(S, M, (int)r.z, np);
        if (COUNT) w_ops += 1 + np;
        int esr = 0;
        for (int k = 0; k < Mr; ++k) {
            const int rk = S.reqk[a * Mr + k];
            if (rk > 0) {
                esr = max(esr, M.ld16(ce0 + (int)S.res[2 * k + 1] + (int)S.res[2 * k] - rk));
                if (COUNT) {
                    ++w_ops;
                    ++w_cells;
                }
            }
        }
        const int s = max(es, esr);
        if (d > 0) {
            for (int k = 0; k < Mr; ++k) {
                const int rk = S.reqk[a * Mr + k];
                if (rk == 0) continue;
                const int cb = ce0 + (int)S.res[2 * k + 1], Rk = (int)S.res[2 * k];
                // effort r*d charged to the units below the bound (the finish,
                // then the time the last raised unit got); the first r raised
                // to the finish, later ones to the time of the unit raised r
                // raises before (the ring), the last one by what is left
                int left = rk * d, raised = 0, bound = s + d;
                // the passed-over prefix ends by unit Rk - rk (free from the
                // eq. 7 start); the first unit is tested on its own (about
                // half of the updates pass over nothing)
                int lo = 0, hi = Rk - rk;
                if (M.ld16(cb) < bound) hi = 0;
                else lo = 1;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (M.ld16(cb + mid) < bound) hi = mid;
                    else lo = mid + 1;
                }
                if (COUNT) {
                    w_ops += lo;
                    w_cells += lo;
                }
                for (int j = lo; j < Rk && left > 0; ++j) {
                    if (COUNT) {
                        ++w_ops;
                        ++w_cells;
                    }
                    const int cv = M.ld16(cb + j);
                    if (cv >= bound) continue;
                    if (raised >= rk) bound = M.ld16(pe0 + ((raised - rk) & pmask));
                    const int from = max(cv, s);
                    if (bound - from >= left) {
                        M.st16(cb + j, from + left);
                        left = 0;
                    } else {
                        left -= bound - from;
                        M.st16(pe0 + (raised & pmask), cv);
                        ++raised;
                        M.st16(cb + j, bound);
                    }
                }
            }
        }
        M.st16b(fo, s + d);
    }
    if (COUNT) wk->add(Work{w_ops, w_cells});
    return p1 == D.n ? M.ld16(D.n - 1) : 0;
}

// Fresh decoder state: capacity-indexed arrays start at zero; the
// time-indexed profile needs nothing (front = 0).
template <int DEC, int STRIDE>
__device__ inline void init_state(const InstDesc &D, uint32_t *lane_base) {
    if (DEC == kEvalCapacity) {
        LaneMem<STRIDE> M{lane_base};
        const int F0 = (D.n + 1) >> 1, Cd = (D.sum_r + 1) >> 1;
        for (int i = 0; i < Cd; ++i) M.st(F0 + i, 0u);
    }
}

// Copy a state (finish times + resource state up to `front`) from a
// stride-1 area into a lane's storage.
template <int NW, int DEC, int STRIDE, int FB = 16>
__device__ inline void copy_state(const InstDesc &D, const uint32_t *src, uint32_t *lane_base, int front) {
    LaneMem<STRIDE> M{lane_base};
    const int F0 = f_dwords<FB>(D.n);
    const int n = F0 + (DEC == kEvalCapacity ? (D.sum_r + 1) >> 1 : front * NW);
    int i = 0;
    for (; i + 4 <= n; i += 4) {
        const uint4 x = *reinterpret_cast<const uint4 *>(src + i);
        M.st(i, x.x);
        M.st(i + 1, x.y);
        M.st(i + 2, x.z);
        M.st(i + 3, x.w);
    }
    for (; i < n; ++i) M.st(i, src[i]);
}

// One thread decodes W with positions u, v exchanged from scratch, using the
// whole decode region as its private storage (stride 1): the time-indexed
// profile then spans long_len >= horizon time units.
template <int NW, int DEC, bool COUNT = false>
__device__ int decode_long(const Sh &S, const InstDesc &D, const Layout &Ly, int u, int v,
                           Work *wk = nullptr) {
    init_state<DEC, 1>(D, S.region);
    if (DEC == kEvalTime) {
        bool ovf = false;
        int front = 0;
        return decode_ti<NW, 1, COUNT>(S, D, S.region, Ly.long_len, u, v, 0, D.n, front, ovf, wk);
    }
    return decode_ci<1, COUNT>(S, D, S.region, u, v, 0, D.n, wk);
}

template <int NW, int G, bool COUNT, int FB = 16>
__device__ int decode_tg(const Sh &S, const InstDesc &D, uint32_t *cb, int L, int u, int v, int p0, int p1,
                         int &front, bool &ovf, Work *wk);

// Minimum and maximum over the 64 lanes of a wave as wave-uniform values
// (every lane must be active): DPP moves inside each row of 16 lanes, then
// the four row results in scalar registers.  Every lane of a row has a
// source under these four patterns, so the "old" operand is never taken;
// giving it the identity of min lets the compiler fold each move into the
// min as a DPP operand.
__device__ inline int wave_min_uniform(int x) {
    constexpr int kId = 0x7fffffff;
    x = min(x, __builtin_amdgcn_update_dpp(kId, x, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    x = min(x, __builtin_amdgcn_update_dpp(kId, x, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    x = min(x, __builtin_amdgcn_update_dpp(kId, x, 0x141, 0xF, 0xF, false));   // row_half_mirror
    x = min(x, __builtin_amdgcn_update_dpp(kId, x, 0x140, 0xF, 0xF, false));   // row_mirror
    const int a = __builtin_amdgcn_readlane(x, 0), b = __builtin_amdgcn_readlane(x, 16);
    const int c = __builtin_amdgcn_readlane(x, 32), e = __builtin_amdgcn_readlane(x, 48);
    // the four row minima are scalars: combine them on the scalar unit
    int ab, ce, m;
    asm("s_min_i32 %0, %1, %2" : "=s"(ab) : "s"(a), "s"(b));
    asm("s_min_i32 %0, %1, %2" : "=s"(ce) : "s"(c), "s"(e));
    asm("s_min_i32 %0, %1, %2" : "=s"(m) : "s"(ab), "s"(ce));
    return m;
}
__device__ inline int wave_max_uniform(int x) { return -wave_min_uniform(-x); }

// Time-indexed lane decode with the lane's resource profile in registers
// (layout kLayoutRegs): kRegUnits time units, one dword each (every resource
// of the unit in a guarded field, as in decode_ti), held in an array that is
// only ever indexed with compile-time constants, so it stays in VGPRs.  The
// finish times stay in LDS (8-bit, lane-interleaved, as in decode_ti).
//
// Per activity (the positions are the same for the whole wave), Alg. 5 is a
// sweep over the time units common to the wave: unit t is examined by every
// lane, each keeping the last unit short of capacity inside the free run it
// is growing (a shortfall counts only while the run is open: after the
// lane's earliest start, before d free units followed the last shortfall);
// once the sweep has passed d free units after it, the lane's start is
// fixed.  The sweep starts at the block holding the wave's smallest
// earliest start and ends after the first block (of kRegBlock units) by
// which every lane has its start.  Alg. 6 is a second sweep over the same
// blocks, each lane subtracting its request inside its own [s, s + d) (a
// bit mask of the interval per block).  Blocks outside a sweep's range are
// skipped by scalar branches (eight-unit blocks measured best: fewer block
// tests than four, fewer units past the last start than sixteen).  A lane
// whose start is not found within
// the kRegUnits units (or whose finish passes 255) reports overflow and runs
// along without touching its profile, like decode_ti.  Lanes without a
// candidate (idle) take part in the sweeps' collective steps only.
//
// The profile is initialised from the wave's base decode: units below its
// frontier from the base profile (16-byte aligned, stride 1), the others at
// the full capacity.  COUNT counts what decode_ti counts.
constexpr int kRegBlock = 8;

template <int T, bool COUNT>
__device__ int decode_tv(const Sh &S, const InstDesc &D, uint32_t *lane_base, const uint32_t *bprof, int front,
                         int u, int v, int p0, int p1, bool idle, bool &ovf, Work *wk, int *rel = nullptr,
                         int relk = 0) {
    LaneMem<T> M{lane_base};
    const uint32_t Gd = D.guard[0], FULL = D.full[0];
    const uint4 *rec = reinterpret_cast<const uint4 *>(S.prec);
    const uint4 *pin = reinterpret_cast<const uint4 *>(S.pin);
    long long w_ops = 0, w_cells = 0;
    front = __builtin_amdgcn_readfirstlane(front);
    p0 = __builtin_amdgcn_readfirstlane(p0);
    p1 = __builtin_amdgcn_readfirstlane(p1);
    uint32_t P[kRegUnits];
#pragma unroll
    for (int b = 0; b < kRegUnits; b += 4) {
        if (b + 4 <= front) {
            const uint4 x = *reinterpret_cast<const uint4 *>(bprof + b);
            P[b] = x.x;
            P[b + 1] = x.y;
            P[b + 2] = x.z;
            P[b + 3] = x.w;
        } else if (b >= front) {
            P[b] = P[b + 1] = P[b + 2] = P[b + 3] = FULL;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) P[b + k] = (b + k < front) ? bprof[b + k] : FULL;
        }
    }
    // the shared base decode has been read: hand it on (rel: the ticket of
    // the workgroup's base decode, relk this chunk's index)
    if (rel) {
        __builtin_amdgcn_wave_barrier();
        __hip_atomic_store(rel, relk, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    bool over = idle;
    // the source finishes at 0; absent predecessors read its slot
    if (p0 == 0) M.template stf<8>(0u, 0);
    auto qof = [&](int p) {
        p = min(p, D.n - 1);
        return (p == u) ? v : ((p == v) ? u : p);
    };
    int q = qof(p0);
    uint4 r = rec[q];
    uint4 pi = pin[q];
    for (int p = p0; p < p1; ++p) {
        const uint32_t rq = S.prq[q];
        const int d = r.y & 0xffff, np = r.y >> 16;
        const uint32_t fo = r.x;
        const int f0 = M.template ldf<8>(pi.x), f1 = M.template ldf<8>(pi.y);
        const int f2 = M.template ldf<8>(pi.z), f3 = M.template ldf<8>(pi.w);
        int es = max(max(f0, f1), max(f2, f3));
        for (int e = 4; e < np; ++e) es = max(es, M.template ldf<8>(S.predT[r.z + e]));
        const int qn = qof(p + 1);
        const uint4 rn = rec[qn];
        const uint4 pn = pin[qn];
        if (COUNT) w_ops += 1 + np;
        const bool need = !over && rq != 0u && d > 0;
        int s = es;
        if (__builtin_amdgcn_ballot_w64(need) != 0ull) {
            // Alg. 5: lanes still scanning are `todo`
            const int tmin = wave_min_uniform(need ? es : 0x7fffffff);
            // per lane: g counts the units since the last one short of
            // capacity inside the free run being grown, up to the unit just
            // examined (es - 1 stands for that unit at first, so units before
            // es give negative counts); a shortfall restarts the run only
            // while it is open (0 <= g < d), so once g reaches d the run is
            // closed and g only grows; the start is the last unit examined
            // minus g, plus one.  (Counting from the run's start keeps the
            // step's dependent chain short and its constants out of it.)
            int g = (tmin & ~(kRegBlock - 1)) - es, tl = 0;
            // lanes that place nothing scan with a run length no count can
            // reach, which keeps them out of the block-end test
            int dd = need ? d : -(1 << 20);
            asm volatile("" : "+v"(dd));
            // blocks below tmin are skipped four at a time, then one at a time
            constexpr int kSuper = 4 * kRegBlock;
            static_assert(kRegUnits % kSuper == 0, "profile in whole groups of four blocks");
#pragma unroll
            for (int B = 0; B < kRegUnits; B += kSuper) {
                if (B + kSuper <= tmin) continue;
#pragma unroll
                for (int b = B; b < B + kSuper; b += kRegBlock) {
                    if (b + kRegBlock <= tmin) continue;
#pragma unroll
                    for (int k = 0; k < kRegBlock; ++k) {
                        const bool mis = ((P[b + k] - rq) & Gd) != Gd;
                        const bool open = (unsigned)g < (unsigned)dd;
                        g = (mis && open) ? 0 : g + 1;
                    }
                    tl = b + kRegBlock - 1;
                    if (__builtin_amdgcn_ballot_w64(g < dd) == 0ull) goto scan_done;
                }
            }
        scan_done:
            const bool todo = need && g < d;
            if (need && !todo) s = tl - g + 1;
            // no start within the register profile: the long-profile path
            over = over || todo;
            // Alg. 6 over the units some lane covers
            const bool upd = need && !todo;
            // lanes without an interval subtract over an empty one
            const int se = upd ? s + d : s;
            if (__builtin_amdgcn_ballot_w64(upd) != 0ull) {
                // every interval lies in the swept units [tmin, tl]
#pragma unroll
                for (int B = 0; B < kRegUnits; B += kSuper) {
                    if (B + kSuper <= tmin) continue;
                    if (B > tl) break;
#pragma unroll
                    for (int b = B; b < B + kSuper; b += kRegBlock) {
                        if (b + kRegBlock <= tmin) continue;
                        if (b > tl) break;
                        // the lane's interval as a mask over the block's
                        // units; unit k takes bit k, sign-extended
                        const int a0 = min(max(s - b, 0), kRegBlock);
                        const int a1 = min(max(se - b, 0), kRegBlock);
                        const uint32_t m = ((1u << a1) - 1u) ^ ((1u << a0) - 1u);
#pragma unroll
                        for (int k = 0; k < kRegBlock; ++k)
                            P[b + k] -= (uint32_t)__builtin_amdgcn_sbfe((int)m, k, 1) & rq;
                    }
                }
            }
            if (COUNT && upd) {
                w_ops += (s + d - es) + d;
                w_cells += (s + d - es) + d;
            }
        }
        if (COUNT && !(rq != 0u && d > 0)) {
            w_ops += 2 * d;
            w_cells += 2 * d;
        }
        // 8-bit finish times hold at most 255 (see decode_ti)
        over = over || (s + d > 255);
        M.template stf<8>(fo, s + d);
        q = qn;
        r = rn;
        pi = pn;
    }
    if (over) {
        ovf = true;
        return -1;
    }
    if (COUNT) wk->add(Work{w_ops, w_cells});
    return p1 == D.n ? M.template ldf<8>(offF<T, 8>(D.n - 1)) : 0;
}

// Decode every feasible move; return the workgroup's minimum key.
// out_mk (global, canonical index) receives every makespan when non-null.
//
// Each wave takes chunks of 64 moves in canonical order, one candidate per
// lane: wave w starts with chunk w, then takes the next chunk not yet taken
// from a counter, so the chunks of early u (the longest decodes) go first
// and the waves finish close together.  The workgroup keeps one base decode
// of W itself (no swap), handed from chunk to chunk in canonical order: the
// wave of chunk k waits until chunk k - 1's wave has read it, extends it up
// to the chunk's smallest u (time-indexed: lanes 0-15 with the group decode;
// capacity-indexed: lane 0), every lane copies that state, and chunk k + 1
// may go on while the lanes decode their candidates from there.  If W's own
// schedule passes the lane profile length, lanes decode from scratch
// instead.  Candidates that overflow the
// lane profile are decoded afterwards with a profile of the full horizon.
// With COUNT the algorithmic work of every decode the launch runs is added
// to *work_total: the base extensions and each candidate's suffix (or whole
// decodes when share is off), and the long-profile re-decodes (a lane's
// aborted short-profile decode is not counted).  FB: bits per finish time
// in the lane and base states (8 when the lane profile is at most 255).
template <int NW, int T, int DEC, bool COUNT = false, int FB = 16, bool REG = false>
__device__ unsigned long long evaluate_moves(const Sh &S, const InstDesc &D, const Layout &Ly, int nfeas,
                                             int L, int delta, TabuSrc tabu, int asp, int *out_mk,
                                             long long *ovf_total, Work *work_total = nullptr,
                                             bool share = true) {
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    unsigned long long best = ~0ull;
    Work lw{0, 0};
    int *ovf_n = S.scal;                  // overflowed candidates
    int *bstate = S.scal + 1;             // the base decode: positions done, front, overflowed
    int *next_chunk = S.scal + 4, *copied = S.scal + 5;
    // the base decode, 16-byte aligned (register layout: its profile, after
    // the finish times, is the aligned part)
    uint32_t *bst = S.bst + (REG ? ((-f_dwords<FB>(D.n)) & 3) : 0);
    const bool use_base = share;
    if (tid == 0) {
        *ovf_n = 0;
        *next_chunk = T / 64;
        *copied = -1;
        bstate[0] = 0;
        bstate[1] = 0;
        bstate[2] = 0;
        if (use_base) init_state<DEC, 1>(D, bst);
    }
    __syncthreads();
    uint32_t *lane_base = S.region + tid;
    for (int k = wv; k * 64 < nfeas;) {
        const int j0 = k * 64;
        int p0 = 0, front = 0;
        bool from_base = false;
        if (use_base) {
            // chunk k's turn with the base decode once chunk k - 1's lanes
            // have read it (every lane reads the flag: one load, one value)
            while (__hip_atomic_load(copied, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < k - 1)
                __builtin_amdgcn_s_sleep(1);
            const int ulo = S.moves[j0] & 0xffff;
            if constexpr (DEC == kEvalTime) {
                // lanes 0-15 of the wave extend it together (group decode)
                if (lane < 16 && !bstate[2] && bstate[0] < ulo) {
                    bool bovf = false;
                    int bf = bstate[1];
                    Work bw{0, 0};
                    decode_tg<NW, 16, COUNT, FB>(S, D, bst, L, 0, 0, bstate[0], ulo, bf, bovf, &bw);
                    if (COUNT && !bovf) lw.add(bw);   // lane 0 holds the group's count
                    __builtin_amdgcn_wave_barrier();
                    if (lane == 0) {
                        bstate[0] = ulo;
                        bstate[1] = bf;
                        bstate[2] = bovf ? 1 : 0;
                    }
                }
            } else {
                if (lane == 0 && !bstate[2] && bstate[0] < ulo) {
                    decode_ci<1, COUNT>(S, D, bst, 0, 0, bstate[0], ulo, &lw);
                    bstate[0] = ulo;
                }
            }
            __builtin_amdgcn_wave_barrier();
            from_base = !bstate[2];
            p0 = from_base ? bstate[0] : 0;
            front = from_base ? bstate[1] : 0;
        }
        const int j = j0 + lane;
        const bool has = j < nfeas;
        if constexpr (REG) {
            // register profiles: every lane takes part in the decode's
            // collective steps, lanes past the last move as idle
            const uint32_t mv = has ? S.moves[j] : 0u;
            const int u = mv & 0xffff, v = (mv >> 16) & 0x7fff;
            if (from_base) {
                // the finish times (dword copies: the base's start need not be aligned)
                LaneMem<T> M{lane_base};
                for (int i = 0; i < f_dwords<FB>(D.n); ++i) M.st(i, bst[i]);
            }
            bool ovf = false;
            Work cw{0, 0};
            // the decode hands the base on once its profile is in registers
            const int c = decode_tv<T, COUNT>(S, D, lane_base, bst + f_dwords<FB>(D.n), front, u, v, p0, D.n, !has,
                                              ovf, &cw, use_base ? copied : nullptr, k);
            if (has) {
                if (COUNT && !ovf) lw.add(cw);
                if (ovf) {
                    S.moves[j] = mv | 0x80000000u;
                    atomicAdd(ovf_n, 1);
                } else {
                    const unsigned long long key = move_key(c, u, v, tabu.get(u, v), asp);
                    best = key < best ? key : best;
                    if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                }
            }
        } else {
            const uint32_t mv = has ? S.moves[j] : 0u;
            const int u = mv & 0xffff, v = (mv >> 16) & 0x7fff;
            if (has) {
                if (from_base) copy_state<NW, DEC, T, FB>(D, bst, lane_base, front);
                else init_state<DEC, T>(D, lane_base);
            }
            if (use_base) {
                // the lanes' copies are done: chunk k + 1 may take the base on
                __builtin_amdgcn_wave_barrier();
                __hip_atomic_store(copied, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            if (has) {
                bool ovf = false;
                int c;
                Work cw{0, 0};
                if (DEC == kEvalTime)
                    c = decode_ti<NW, T, COUNT, FB>(S, D, lane_base, L, u, v, p0, D.n, front, ovf, &cw);
                else
                    c = decode_ci<T, COUNT>(S, D, lane_base, u, v, p0, D.n, &cw);
                if (COUNT && !ovf) lw.add(cw);
                if (ovf) {
                    S.moves[j] = mv | 0x80000000u;
                    atomicAdd(ovf_n, 1);
                } else {
                    const unsigned long long key = move_key(c, u, v, tabu.get(u, v), asp);
                    best = key < best ? key : best;
                    if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        int nk = 0;
        if (lane == 0) nk = atomicAdd(next_chunk, 1);
        k = __builtin_amdgcn_readlane(nk, 0);
    }
    __syncthreads();
    if constexpr (DEC == kEvalTime) {
        const int novf = *ovf_n;
        if (novf > 0) {
            // Candidates whose schedule passed the lane profile: groups of
            // 16 lanes decode them side by side (the group decode below),
            // each group in its own slice of the candidate region when a
            // slice holds a profile of the whole horizon (no schedule is
            // longer than the sum of durations); else one thread in the
            // whole region.
            constexpr int GG = 16, NGR = T / GG;
            const int grp = tid / GG, g = tid & (GG - 1), gbase = tid & 63 & ~(GG - 1);
            const int F016 = (D.n + 1) >> 1;
            const int chunk = ((Ly.cands * Ly.per_lane) / NGR) & ~3;
            const int glen = (chunk - F016) / NW;
            if (glen >= D.horizon) {
                uint32_t *cb = S.region + grp * chunk;
                int rank = 0;
                for (int j0 = 0; j0 < nfeas; j0 += GG) {
                    const int jj = j0 + g;
                    const bool flagged = jj < nfeas && (S.moves[jj] & 0x80000000u) != 0u;
                    unsigned long long m = (__ballot(flagged) >> gbase) & 0xffffull;
                    while (m != 0ull) {
                        const int bit = __ffsll(m) - 1;
                        m &= m - 1ull;
                        if (rank++ % NGR != grp) continue;
                        const int j = j0 + bit;
                        const uint32_t mv = S.moves[j];
                        const int u = mv & 0xffff, v = (mv >> 16) & 0x7fff;
                        bool ovf = false;
                        int front = 0;
                        Work cw{0, 0};
                        const int c = decode_tg<NW, GG, COUNT>(S, D, cb, glen, u, v, 0, D.n, front, ovf, &cw);
                        if (g == 0) {
                            if (COUNT) lw.add(cw);
                            const unsigned long long k = move_key(c, u, v, tabu.get(u, v), asp);
                            best = k < best ? k : best;
                            if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                }
                __syncthreads();
                for (int j = tid; j < nfeas; j += T) S.moves[j] &= 0x7fffffffu;
                if (tid == 0 && ovf_total) *ovf_total += novf;
            } else if (tid == 0) {
                for (int j = 0; j < nfeas; ++j) {
                    const uint32_t mv = S.moves[j];
                    if (mv & 0x80000000u) {
                        const int u = mv & 0xffff, v = (mv >> 16) & 0x7fff;
                        const int c = decode_long<NW, DEC, COUNT>(S, D, Ly, u, v, &lw);
                        const unsigned long long k = move_key(c, u, v, tabu.get(u, v), asp);
                        best = k < best ? k : best;
                        if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                        S.moves[j] = mv & 0x7fffffffu;
                    }
                }
                if (ovf_total) *ovf_total += novf;
            }
            __syncthreads();
        }
    }
    if (COUNT) {
        const long long ops = block_sum_i64<T>(lw.ops, S.red);
        const long long cells = block_sum_i64<T>(lw.cells, S.red);
        if (tid == 0) work_total->add(Work{ops, cells});
    }
    return block_min_u64<T>(best, S.red);
}

// ---------------------------------------------------------------------------
// Group decode (time-indexed): G consecutive lanes of a wave share one
// candidate.  Its state is contiguous: finish times (16-bit, by activity),
// then the profile (unit t, word w at prof[t*NW + w]).  Per activity the
// lanes read up to G predecessor finish times and combine them with DPP
// row operations; the Alg. 5 scan tests G consecutive units at once (one per
// lane) and two ballots give the earliest unit from which d units are free;
// the Alg. 6 update writes the d units with d lanes.  Every branch depends
// only on values the whole group shares, so the group stays converged.  The
// lanes of other groups in the wave may have left a loop: ballots are masked
// to the group's own bits.

// Maximum over the G lanes of a group (G in {4, 8, 16}) with DPP moves that
// stay inside a row of 16 lanes: quad swaps, then half-row and row mirrors.
template <int G>
__device__ inline int group_max(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
    x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
    if (G >= 8) x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x141, 0xF, 0xF, false));  // row_half_mirror
    if (G >= 16) x = max(x, __builtin_amdgcn_update_dpp(x, x, 0x140, 0xF, 0xF, false)); // row_mirror
    return x;
}

template <int NW, int G, bool COUNT, int FB>
__device__ int decode_tg(const Sh &S, const InstDesc &D, uint32_t *cb, int L, int u, int v, int p0, int p1,
                         int &front, bool &ovf, Work *wk) {
    static_assert(G == 4 || G == 8 || G == 16, "lanes per candidate");
    const int g = threadIdx.x & (G - 1);
    const int gbase = threadIdx.x & 63 & ~(G - 1);
    constexpr unsigned long long gm = (1ull << G) - 1ull;
    // finish times of FB bits (8: states shared with one-candidate-per-lane
    // layouts of at most 255 units)
    auto fget = [&](int a) -> int {
        if (FB == 8) return reinterpret_cast<const uint8_t *>(cb)[a];
        return reinterpret_cast<const uint16_t *>(cb)[a];
    };
    auto fset = [&](int a, int x) {
        if (FB == 8) reinterpret_cast<uint8_t *>(cb)[a] = (uint8_t)x;
        else reinterpret_cast<uint16_t *>(cb)[a] = (uint16_t)x;
    };
    uint32_t *prof = cb + f_dwords<FB>(D.n);
    uint32_t Gd[NW], FULL[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        Gd[w] = D.guard[w];
        FULL[w] = D.full[w];
    }
    const uint4 *rec = reinterpret_cast<const uint4 *>(S.prec);
    long long w_ops = 0, w_cells = 0;
    int fr = front;
    for (int p = p0; p < p1; ++p) {
        const int q = (p == u) ? v : ((p == v) ? u : p);
        const uint4 r = rec[q];
        const int d = r.y & 0xffff, np = r.y >> 16, a = (int)r.w;
        int es = 0;
        for (int e0 = 0; e0 < np; e0 += G) {
            const int e = e0 + g;
            if (e < np) es = max(es, fget(S.pred[r.z + e]));
        }
        es = group_max<G>(es);
        uint32_t rq[NW];
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            rq[w] = S.prq[q * NW + w];
            any |= rq[w];
        }
        int s = es;
        if (any != 0 && d > 0) {
            int t = es, c = 0;  // c: free units just before t
            s = -1;
            while (t < fr) {
                const int x = t + g;
                bool ok = true;
                if (x < fr) {
                    const uint32_t *P = prof + x * NW;
#pragma unroll
                    for (int w = 0; w < NW; ++w) ok = ok && (((P[w] - rq[w]) & Gd[w]) == Gd[w]);
                }
                const unsigned long long m = (__ballot(ok) >> gbase) & gm;
                const uint32_t mz = (uint32_t)(~m & gm);          // units that do not fit
                const uint32_t below = mz & ((2u << g) - 1u);     // ... at or below this lane's unit
                const int run = below ? g - (31 - __clz(below)) : c + g + 1;
                const unsigned long long hm = (__ballot(run >= d) >> gbase) & gm;
                if (hm != 0ull) {
                    s = t + (__ffsll(hm) - 1) - d + 1;
                    break;
                }
                c = mz ? (G - 1) - (31 - __clz(mz)) : c + G;
                t += G;
            }
            if (s < 0) s = t - c;  // reached the frontier: every later unit is free
            if (s + d > L) {
                ovf = true;
                return -1;
            }
            if (COUNT && g == 0) {
                w_ops += (s + d - es) + d;
                w_cells += (s + d - es) + d;
            }
            const int lo = min(s, fr), hi = s + d;
            for (int x0 = lo; x0 < hi; x0 += G) {
                const int x = x0 + g;
                if (x < hi) {
                    uint32_t *P = prof + x * NW;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        const uint32_t A = (x < fr) ? P[w] : FULL[w];
                        P[w] = (x < s) ? FULL[w] : A - rq[w];
                    }
                }
            }
            fr = max(fr, hi);
        } else if (COUNT && g == 0) {
            w_ops += 2 * d;
            w_cells += 2 * d;
        }
        // 8-bit finish times hold at most 255 (an activity without requests
        // can finish past the profile): report overflow (group-uniform)
        if (FB == 8 && s + d > 255) {
            ovf = true;
            return -1;
        }
        if (COUNT && g == 0) w_ops += 1 + np;
        if (g == 0) fset(a, s + d);
        __builtin_amdgcn_wave_barrier();
    }
    front = fr;
    if (COUNT && g == 0) wk->add(Work{w_ops, w_cells});
    return p1 == D.n ? fget(D.n - 1) : 0;
}

// Capacity-indexed decode with G lanes per candidate (G in {4, 8, 16}):
// lane g owns resources g, g + G, ...  Eq. 7's lookups and Alg. 4's updates
// of different resources are independent, so the group runs them side by
// side and combines the lanes' starts (with the predecessors' finish times,
// also split over the lanes) by a group maximum.  State at cb: 16-bit
// finish times by activity (F0 dwords), the c_k arrays as in decode_ci,
// then one copy ring of copy_p entries per lane.  Each lane's loops run to
// completion before the group maximum, so the group is converged there.
// With COUNT, lane 0 counts one operation per activity and per predecessor
// read, every lane its own eq. 7 lookups and Alg. 4 loop steps (the sum over
// the group equals decode_ci's count).
template <int G, bool COUNT = false>
__device__ int decode_cg(const Sh &S, const InstDesc &D, uint32_t *cb, int u, int v, int p0, int p1,
                         Work *wk) {
    static_assert(G == 4 || G == 8 || G == 16, "lanes per candidate");
    const int g = threadIdx.x & (G - 1);
    const int Mr = D.m;
    const int F0 = (D.n + 1) >> 1, Cd = (D.sum_r + 1) >> 1;
    uint16_t *F = reinterpret_cast<uint16_t *>(cb);
    uint16_t *Cc = reinterpret_cast<uint16_t *>(cb + F0);
    uint16_t *ring = reinterpret_cast<uint16_t *>(cb + F0 + Cd) + g * D.copy_p;
    const int pmask = D.copy_p - 1;
    const uint4 *rec = reinterpret_cast<const uint4 *>(S.prec);
    long long w_ops = 0, w_cells = 0;
    // the update of decode_ci on one resource; leading units at or past the
    // finish are passed over by a binary search
    auto update = [&](int rk, uint16_t *ck, int Rk, int s, int d, int c0) {
        int left = rk * d, raised = 0, bound = s + d;
        // the search ends by unit Rk - rk (free from the eq. 7 start, which
        // s does not precede); about half of the updates pass over nothing,
        // so the first unit is tested on its own
        int lo = 0, hi = Rk - rk;
        if (c0 < bound) hi = 0;
        else lo = 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((int)ck[mid] < bound) hi = mid;
            else lo = mid + 1;
        }
        if (COUNT) {
            w_ops += lo;
            w_cells += lo;
        }
        // lo < Rk (unit Rk - rk is below the bound); if unit lo is free at s,
        // so is every later one (non-increasing): the loop's rk steps each
        // take d of the effort, raising rk units to s + d and reading no
        // copy (most updates)
        const int cl = lo == 0 ? c0 : (int)ck[lo];
        if (cl <= s) {
            for (int i = 0; i < rk; ++i) ck[lo + i] = (uint16_t)bound;
            if (COUNT) {
                w_ops += rk;
                w_cells += rk;
            }
            return;
        }
        for (int j = lo; j < Rk && left > 0; ++j) {
            if (COUNT) {
                ++w_ops;
                ++w_cells;
            }
            // the copy ring's entry is read together with the unit, by the
            // lanes that use it (once rk units were raised)
            const int cv = j == lo ? cl : (int)ck[j];
            int rb = bound;
            if (raised >= rk) rb = ring[(raised - rk) & pmask];
            if (cv >= bound) continue;
            bound = rb;
            const int from = max(cv, s);
            if (bound - from >= left) {
                ck[j] = (uint16_t)(from + left);
                left = 0;
            } else {
                left -= bound - from;
                ring[raised & pmask] = (uint16_t)cv;
                ++raised;
                ck[j] = (uint16_t)bound;
            }
        }
    };
    // with at most G resources a lane owns at most one (k = g): its capacity
    // and c_k offset are read once
    const bool one = Mr <= G;
    const bool own = one && g < Mr;
    const int Rk1 = own ? (int)S.res[2 * g] : 0;
    uint16_t *const ck1 = Cc + (own ? (int)S.res[2 * g + 1] : 0);
    auto qof = [&](int p) {
        p = min(p, D.n - 1);
        return (p == u) ? v : ((p == v) ? u : p);
    };
    // the positions are the same for every lane of the wave: a scalar loop;
    // each position's record is read while the previous one is placed
    p0 = __builtin_amdgcn_readfirstlane(p0);
    p1 = __builtin_amdgcn_readfirstlane(p1);
    uint4 r = rec[qof(p0)];
    for (int p = p0; p < p1; ++p) {
        const int d = r.y & 0xffff, np = r.y >> 16, a = (int)r.w;
        const uint4 rn = rec[qof(p + 1)];
        int s = 0;
        for (int e = g; e < np; e += G) s = max(s, (int)F[S.pred[r.z + e]]);
        int rk1 = 0, c01 = 0;
        if (one) {
            if (own) {
                rk1 = S.reqk[a * Mr + g];
                if (rk1 > 0) {
                    // Alg. 4's first unit is read with the eq. 7 lookup
                    s = max(s, (int)ck1[Rk1 - rk1]);
                    c01 = ck1[0];
                    if (COUNT) {
                        ++w_ops;
                        ++w_cells;
                    }
                }
            }
        } else {
            for (int k = g; k < Mr; k += G) {
                const int rk = S.reqk[a * Mr + k];
                if (rk > 0) {
                    s = max(s, (int)Cc[(int)S.res[2 * k + 1] + (int)S.res[2 * k] - rk]);
                    if (COUNT) {
                        ++w_ops;
                        ++w_cells;
                    }
                }
            }
        }
        s = group_max<G>(s);
        if (d > 0) {
            if (one) {
                if (rk1 > 0) update(rk1, ck1, Rk1, s, d, c01);
            } else {
                for (int k = g; k < Mr; k += G) {
                    const int rk = S.reqk[a * Mr + k];
                    if (rk > 0) {
                        uint16_t *const ck = Cc + (int)S.res[2 * k + 1];
                        update(rk, ck, (int)S.res[2 * k], s, d, (int)ck[0]);
                    }
                }
            }
        }
        if (COUNT && g == 0) w_ops += 1 + np;
        if (g == 0) F[a] = (uint16_t)(s + d);
        __builtin_amdgcn_wave_barrier();
        r = rn;
    }
    if (COUNT) wk->add(Work{w_ops, w_cells});
    return p1 == D.n ? (int)F[D.n - 1] : 0;
}

// Group decode of either kind (time-indexed: decode_tg).
template <int NW, int DEC, int G, bool COUNT = false>
__device__ inline int decode_grp(const Sh &S, const InstDesc &D, uint32_t *cb, int L, int u, int v, int p0, int p1,
                                 int &front, bool &ovf, Work *wk) {
    if constexpr (DEC == kEvalCapacity) return decode_cg<G, COUNT>(S, D, cb, u, v, p0, p1, wk);
    else return decode_tg<NW, G, COUNT>(S, D, cb, L, u, v, p0, p1, front, ovf, wk);
}

// Group version of evaluate_moves: one candidate per group of G lanes,
// chunks of 64/G moves per wave.  Waves take chunks in canonical order from
// a counter and run independently, sharing one base decode (the prefix
// before the chunk's smallest u): chunk k's wave waits until chunk k - 1's
// wave has copied the base, extends it with its first group and copies it
// into its groups' states, then lets chunk k + 1 go on while it decodes.
// Candidates that overflow their profile are decoded afterwards by group 0
// over the whole candidate region (>= horizon units).
template <int NW, int T, int DEC, int G, bool COUNT = false>
__device__ unsigned long long evaluate_moves_g(const Sh &S, const InstDesc &D, const Layout &Ly, int nfeas,
                                               int L, int delta, TabuSrc tabu, int asp, int *out_mk,
                                               long long *ovf_total, Work *work_total = nullptr,
                                               bool share = true) {
    constexpr bool CAP = DEC == kEvalCapacity;
    const int tid = threadIdx.x, grp = tid / G, g = tid & (G - 1);
    unsigned long long best = ~0ull;
    Work lw{0, 0};
    constexpr int CW = 64 / G;   // candidates per wave chunk
    const int wv = tid >> 6, lane = tid & 63, gw = lane / G;
    int *ovf_n = S.scal;
    int *bstate = S.scal + 1;
    int *next_chunk = S.scal + 4, *copied = S.scal + 5;
    const bool use_base = share;
    const int F0 = (D.n + 1) >> 1, Cd = (D.sum_r + 1) >> 1;
    if (tid == 0) {
        *ovf_n = 0;
        bstate[0] = 0;
        bstate[1] = 0;
        bstate[2] = 0;
        *next_chunk = T / 64;
        *copied = -1;
    }
    // capacity-indexed states start with every c_k entry at zero
    if (CAP && use_base)
        for (int i = tid; i < Cd; i += T) S.bst[F0 + i] = 0u;
    __syncthreads();
    uint32_t *cb = S.region + grp * Ly.per_lane;
    for (int k = wv; k * CW < nfeas;) {
        const int j0 = k * CW;
        const int j = j0 + gw;
        const bool has = j < nfeas;
        const uint32_t mv = has ? S.moves[j] : 0u;
        int p0 = 0, front = 0;
        bool from_base = false;
        if (use_base) {
            // the base decode is chunk k's once chunk k - 1's copies are
            // done (every lane reads the flag: one load, one value)
            while (__hip_atomic_load(copied, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < k - 1)
                __builtin_amdgcn_s_sleep(1);
            const int ulo = S.moves[j0] & 0xffff;
            if (gw == 0 && !bstate[2] && bstate[0] < ulo) {
                bool bovf = false;
                int bf = bstate[1];
                Work bw{0, 0};
                decode_grp<NW, DEC, G, COUNT>(S, D, S.bst, L, 0, 0, bstate[0], ulo, bf, bovf, &bw);
                if (COUNT && !bovf) lw.add(bw);
                if (g == 0) {
                    bstate[0] = ulo;
                    bstate[1] = bf;
                    bstate[2] = bovf ? 1 : 0;
                }
            }
            __builtin_amdgcn_wave_barrier();
            from_base = !bstate[2];
            if (has && from_base) {
                p0 = bstate[0];
                front = bstate[1];
                const int nd = F0 + (CAP ? Cd : front * NW);
                const uint4 *src = reinterpret_cast<const uint4 *>(S.bst);
                uint4 *dst = reinterpret_cast<uint4 *>(cb);
                for (int i = g; i < (nd >> 2); i += G) dst[i] = src[i];
                for (int i = (nd & ~3) + g; i < nd; i += G) cb[i] = S.bst[i];
            }
            // this wave's reads of the base are done: chunk k + 1 may go on
            __builtin_amdgcn_wave_barrier();
            __hip_atomic_store(copied, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (has) {
            const int u = mv & 0xffff, v = mv >> 16;
            if (!from_base && CAP) {
                for (int i = g; i < Cd; i += G) cb[F0 + i] = 0u;
            }
            __builtin_amdgcn_wave_barrier();
            bool ovf = false;
            Work cw{0, 0};
            const int c = decode_grp<NW, DEC, G, COUNT>(S, D, cb, L, u, v, p0, D.n, front, ovf, &cw);
            // every lane adds its own count (a time-indexed group counts on lane 0 only)
            if (COUNT && !ovf) lw.add(cw);
            if (g == 0) {
                if (ovf) {
                    S.moves[j] = mv | 0x80000000u;
                    atomicAdd(ovf_n, 1);
                } else {
                    const unsigned long long key = move_key(c, u, v, tabu.get(u, v), asp);
                    best = key < best ? key : best;
                    if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        int nk = 0;
        if (lane == 0) nk = atomicAdd(next_chunk, 1);
        k = __builtin_amdgcn_readlane(nk, 0);
    }
    __syncthreads();
    // capacity-indexed states have no horizon and never overflow
    if (!CAP && *ovf_n > 0) {
        if (grp == 0) {
            for (int j = 0; j < nfeas; ++j) {
                const uint32_t mv = S.moves[j];
                if (mv & 0x80000000u) {
                    const int u = mv & 0xffff, v = (mv >> 16) & 0x7fff;
                    bool ovf = false;
                    int front = 0;
                    Work cw{0, 0};
                    const int c = decode_grp<NW, DEC, G, COUNT>(S, D, S.region, Ly.long_len, u, v, 0, D.n, front,
                                                                ovf, &cw);
                    if (g == 0) {
                        if (COUNT) lw.add(cw);
                        const unsigned long long k = move_key(c, u, v, tabu.get(u, v), asp);
                        best = k < best ? k : best;
                        if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                        S.moves[j] = mv & 0x7fffffffu;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            if (tid == 0 && ovf_total) *ovf_total += *ovf_n;
        }
        __syncthreads();
    }
    if (COUNT) {
        const long long ops = block_sum_i64<T>(lw.ops, S.red);
        const long long cells = block_sum_i64<T>(lw.cells, S.red);
        if (tid == 0) work_total->add(Work{ops, cells});
    }
    return block_min_u64<T>(best, S.red);
}

// ---------------------------------------------------------------------------
// Wave decode (layout kLayoutWave, time-indexed): one candidate per wave,
// its resource profile spread over the wave's registers.  Unit t lives in
// lane t & 63 of register chunk t >> 6: word w of chunk c in A[w][c] for
// c < CH, in B[w][c - CH] after that (NB = 2 banks), so the profile holds
// 64 * CH * NB units.  A single candidate makes every per-activity value
// wave-uniform (position, record, earliest start, start), so chunk indexes
// are scalars and index the register file directly (each bank is an array
// of at most 32 dwords, which the compiler keeps in VGPRs).  Finish times
// too: activity x in lane x & 63 of register x >> 6, with a 16-bit copy by
// activity at F in LDS for the predecessors past the first four (read by
// the lanes side by side).  The records of the next position are loaded
// while the current one is placed.
//
// Per activity: the earliest start from the predecessors' finish times;
// Alg. 5 walks chunks from the one holding the earliest start,
// every lane testing its unit for all resources with one subtract and mask
// per word, a ballot giving the chunk's units short of capacity and each
// lane the run of free units that ends at its unit (carried across chunks),
// and the first unit whose run reaches d closing the start; Alg. 6 writes
// the units of [s, s + d) with the lanes of the chunks covering them.  Units
// at or past the frontier fr were never written and count as free; units
// between fr and a start past it are set to full capacity when the frontier
// moves.  A start whose interval passes the profile reports overflow
// (wave-uniform).  COUNT counts as decode_tg does (on lane 0).
// (two banks: both are indexed and the value selected, so that no access
// goes through a pointer chosen between the arrays, which would move them
// to scratch memory)
template <int NW, int CH>
using WaveBanks = uint32_t[NW][CH];

template <int NW, int CH, int NB>
__device__ __attribute__((always_inline)) inline uint32_t tw_get(WaveBanks<NW, CH> &A, WaveBanks<NW, CH> &B, int w,
                                                                 int c) {
    if (NB == 1) return A[w][min(c, CH - 1)];
    const uint32_t x = A[w][min(c, CH - 1)], y = B[w][max(min(c - CH, CH - 1), 0)];
    return c < CH ? x : y;
}
template <int NW, int CH, int NB>
__device__ __attribute__((always_inline)) inline void tw_set(WaveBanks<NW, CH> &A, WaveBanks<NW, CH> &B, int w, int c,
                                                             uint32_t x) {
    if (NB == 1) {
        A[w][min(c, CH - 1)] = x;
        return;
    }
    const int ca = min(c, CH - 1), cb = max(min(c - CH, CH - 1), 0);
    const uint32_t xa = A[w][ca], xb = B[w][cb];
    A[w][ca] = c < CH ? x : xa;
    B[w][cb] = c < CH ? xb : x;
}

// Finish time of activity x from the wave's registers: lane x & 63 of
// register x >> 6 (x wave-uniform), and its update.
constexpr int kWaveFR = kWaveMaxN / 64;
__device__ __attribute__((always_inline)) inline int fr_get(const uint32_t (&FR)[kWaveFR], int x) {
    return __builtin_amdgcn_readlane((int)FR[min(x >> 6, kWaveFR - 1)], x & 63);
}
__device__ __attribute__((always_inline)) inline void fr_set(uint32_t (&FR)[kWaveFR], int x, int val) {
    const int i = min(x >> 6, kWaveFR - 1);
    const uint32_t old = FR[i];
    FR[i] = (int)(threadIdx.x & 63) == (x & 63) ? (uint32_t)val : old;
}

template <int NW, int CH, int NB, bool COUNT>
__device__ __attribute__((always_inline)) int decode_tw(const Sh &S, const InstDesc &D, uint16_t *F,
                                                        uint32_t (&FR)[kWaveFR], WaveBanks<NW, CH> &A,
                                                        WaveBanks<NW, CH> &B, int &fr, int u, int v, int p0, int p1,
                                                        bool &ovf, Work *wk) {
    constexpr int LW = 64 * CH * NB;
    const int lane = threadIdx.x & 63;
    uint32_t Gd[NW], FULL[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        Gd[w] = D.guard[w];
        FULL[w] = D.full[w];
    }
    // lanes at or below this lane (the run of free units ending at its unit)
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const uint4 *rec = reinterpret_cast<const uint4 *>(S.prec);
    const uint2 *pid = reinterpret_cast<const uint2 *>(S.pid);
    long long w_ops = 0, w_cells = 0;
    int f = __builtin_amdgcn_readfirstlane(fr);
    u = __builtin_amdgcn_readfirstlane(u);
    v = __builtin_amdgcn_readfirstlane(v);
    p0 = __builtin_amdgcn_readfirstlane(p0);
    p1 = __builtin_amdgcn_readfirstlane(p1);
    auto qof = [&](int p) {
        p = min(p, D.n - 1);
        return (p == u) ? v : ((p == v) ? u : p);
    };
    // the records of a position are loaded one position ahead
    int q = qof(p0);
    uint4 r = rec[q];
    uint2 pd = pid[q];
    uint32_t rqn[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) rqn[w] = S.prq[q * NW + w];
    for (int p = p0; p < p1; ++p) {
        const int d = __builtin_amdgcn_readfirstlane((int)(r.y & 0xffff));
        const int np = __builtin_amdgcn_readfirstlane((int)(r.y >> 16));
        const int po = __builtin_amdgcn_readfirstlane((int)r.z);
        const int a = __builtin_amdgcn_readfirstlane((int)r.w);
        const uint32_t i01 = __builtin_amdgcn_readfirstlane(pd.x), i23 = __builtin_amdgcn_readfirstlane(pd.y);
        uint32_t rq[NW];
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            rq[w] = __builtin_amdgcn_readfirstlane(rqn[w]);
            any |= rq[w];
        }
        q = qof(p + 1);
        r = rec[q];
        pd = pid[q];
#pragma unroll
        for (int w = 0; w < NW; ++w) rqn[w] = S.prq[q * NW + w];
        // earliest start: the first four predecessors from the registers,
        // further ones (lanes side by side) from the finish times in LDS
        int es = max(max(fr_get(FR, (int)(i01 & 0xffff)), fr_get(FR, (int)(i01 >> 16))),
                     max(fr_get(FR, (int)(i23 & 0xffff)), fr_get(FR, (int)(i23 >> 16))));
        if (np > 4) {
            int x = 0;
            for (int e0 = 4; e0 < np; e0 += 64) {
                const int e = e0 + lane;
                if (e < np) x = max(x, (int)F[S.pred[po + e]]);
            }
            x = np <= 20 ? __builtin_amdgcn_readlane(group_max<16>(x), 0) : wave_max_uniform(x);
            es = max(es, x);
        }
        int s = es;
        if (any != 0u && d > 0) {
            if (es < f) {
                // Alg. 5 over the written units, chunk by chunk (every chunk
                // visited starts below the frontier, so inside the profile)
                int c = es >> 6, run = 0;
                for (;;) {
                    const int tb = c << 6, t = tb + lane;
                    bool ok = true;
#pragma unroll
                    for (int w = 0; w < NW; ++w) ok = ok && (((tw_get<NW, CH, NB>(A, B, w, c) - rq[w]) & Gd[w]) == Gd[w]);
                    const bool fit = t >= es && (t >= f || ok);
                    const unsigned long long mz = ~__builtin_amdgcn_ballot_w64(fit);
                    const unsigned long long below = mz & upto;
                    const int rl = below ? lane - (63 - (int)__clzll(below)) : run + lane + 1;
                    const unsigned long long hm = __builtin_amdgcn_ballot_w64(rl >= d);
                    if (hm != 0ull) {
                        s = tb + (__ffsll(hm) - 1) - d + 1;
                        break;
                    }
                    run = mz ? (int)__clzll(mz) : run + 64;
                    if (tb + 64 >= f) {
                        // every unit past this chunk is free
                        s = tb + 64 - run;
                        break;
                    }
                    ++c;
                }
            }
            if (s + d > LW) {
                ovf = true;
                return -1;
            }
            if (COUNT && lane == 0) {
                w_ops += (s + d - es) + d;
                w_cells += (s + d - es) + d;
            }
            // Alg. 6 (and full capacity for the units between the frontier and s)
            const int lo = min(s, f), hi = s + d;
            for (int c = lo >> 6; c <= (hi - 1) >> 6; ++c) {
                const int x = (c << 6) + lane;
                const bool in = x >= lo && x < hi;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const uint32_t old = tw_get<NW, CH, NB>(A, B, w, c);
                    const uint32_t base = x < f ? old : FULL[w];
                    const uint32_t nv = x < s ? FULL[w] : base - rq[w];
                    tw_set<NW, CH, NB>(A, B, w, c, in ? nv : old);
                }
            }
            f = max(f, hi);
        } else if (COUNT && lane == 0) {
            w_ops += 2 * d;
            w_cells += 2 * d;
        }
        if (COUNT && lane == 0) w_ops += 1 + np;
        fr_set(FR, a, s + d);
        if (lane == 0) F[a] = (uint16_t)(s + d);
        __builtin_amdgcn_wave_barrier();
    }
    fr = f;
    if (COUNT && lane == 0) wk->add(Work{w_ops, w_cells});
    return p1 == D.n ? fr_get(FR, D.n - 1) : 0;
}

// Evaluation with one candidate per wave (layout kLayoutWave): wave w takes
// moves w, w + T/64, ... in canonical order (u ascending), so its own base
// decode (W itself, profile in the register bank Pb) only moves forward:
// before a candidate the wave extends it up to the candidate's u, copies
// the bank to P and decodes positions u.. of the candidate there.  Base and
// candidates share the wave's finish-time area: a candidate writes only the
// activities at positions u and later, which the base rewrites before it
// reads them.  Waves never wait for each other inside the loop.  A
// candidate that passes its bank (or comes after the wave's base passed
// its own) is decoded afterwards from scratch over both banks (twice the
// profile; the waves take these in turn), and one that passes both by
// lanes 0-15 with the group decode over the whole region (a profile of the
// full horizon).
template <int NW, int T, bool COUNT = false>
__device__ unsigned long long evaluate_moves_w(const Sh &S, const InstDesc &D, const Layout &Ly, int nfeas,
                                               int delta, TabuSrc tabu, int asp, int *out_mk, long long *ovf_total,
                                               Work *work_total = nullptr, bool share = true) {
    constexpr int CH = kWaveDwords / NW, NV = T / 64;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    unsigned long long best = ~0ull;
    Work lw{0, 0};
    int *ovf_n = S.scal;        // candidates flagged for a re-decode over both banks
    int *ovf2_n = S.scal + 1;   // ... and for the group decode
    if (tid == 0) {
        *ovf_n = 0;
        *ovf2_n = 0;
    }
    __syncthreads();
    uint16_t *F = reinterpret_cast<uint16_t *>(S.region + wv * Ly.per_lane);
    // both banks are set here so that their contents do not live on from
    // one evaluation to the next (registers held across the whole kernel)
    uint32_t Pb[NW][CH], P[NW][CH], FR[kWaveFR];
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int k = 0; k < CH; ++k) Pb[w][k] = P[w][k] = 0u;
#pragma unroll
    for (int k = 0; k < kWaveFR; ++k) FR[k] = 0u;
    // flags in the move list: bit 31 for a re-decode over both banks, bit 30
    // for the group decode (a candidate that passed both keeps bit 31, so
    // the list the waves deal from does not change under them)
    auto finish = [&](int j, uint32_t mv, int c, bool ovf, uint32_t flag, const Work &cw) {
        const int u = mv & 0xffff, v = (mv >> 16) & 0x3fff;
        if (lane == 0) {
            if (ovf) {
                S.moves[j] = mv | flag;
                atomicAdd((flag & 0x40000000u) ? ovf2_n : ovf_n, 1);
            } else {
                if (COUNT) lw.add(cw);
                const unsigned long long k = move_key(c, u, v, tabu.get(u, v), asp);
                best = k < best ? k : best;
                if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
            }
        }
    };
    int bpos = 0, bfr = 0;
    bool bdead = !share;
    for (int j = wv; j < nfeas; j += NV) {
        const uint32_t mv = __builtin_amdgcn_readfirstlane(S.moves[j]);
        const int u = mv & 0xffff, v = (mv >> 16) & 0x3fff;
        if (!bdead && bpos < u) {
            bool bo = false;
            Work bw{0, 0};
            decode_tw<NW, CH, 1, COUNT>(S, D, F, FR, Pb, Pb, bfr, 0, 0, bpos, u, bo, &bw);
            if (bo) bdead = true;
            else if (COUNT) lw.add(bw);
            bpos = u;
        }
        bool ovf = false;
        Work cw{0, 0};
        int c;
        if (!bdead) {
#pragma unroll
            for (int w = 0; w < NW; ++w)
#pragma unroll
                for (int k = 0; k < CH; ++k) P[w][k] = Pb[w][k];
            int fr = bfr;
            c = decode_tw<NW, CH, 1, COUNT>(S, D, F, FR, P, P, fr, u, v, bpos, D.n, ovf, &cw);
            finish(j, mv, c, ovf, 0x80000000u, cw);
        } else {
            // no base: decoded from scratch over both banks after the loop
            finish(j, mv, 0, true, 0x80000000u, cw);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    if (*ovf_n > 0) {
        // over both banks, from scratch: flagged candidates dealt to the waves in turn
        int rank = 0;
        for (int j0 = 0; j0 < nfeas; j0 += 64) {
            const int jj = j0 + lane;
            const bool flagged = jj < nfeas && (S.moves[jj] & 0x80000000u) != 0u;
            unsigned long long m = __builtin_amdgcn_ballot_w64(flagged);
            while (m != 0ull) {
                const int j = j0 + __ffsll(m) - 1;
                m &= m - 1ull;
                if (rank++ % NV != wv) continue;
                const uint32_t mv = __builtin_amdgcn_readfirstlane(S.moves[j]);
                const int u = mv & 0xffff, v = (mv >> 16) & 0x3fff;
                bool ovf = false;
                int fr = 0;
                Work cw{0, 0};
                const int c = decode_tw<NW, CH, 2, COUNT>(S, D, F, FR, Pb, P, fr, u, v, 0, D.n, ovf, &cw);
                finish(j, mv, c, ovf, 0x40000000u, cw);
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
    }
    if (*ovf2_n > 0) {
        // past both banks: the group decode over the whole region
        if (tid < 16) {
            constexpr unsigned long long gm = 0xffffull;
            for (int j0 = 0; j0 < nfeas; j0 += 16) {
                const int jj = j0 + tid;
                const bool flagged = jj < nfeas && (S.moves[jj] & 0x40000000u) != 0u;
                unsigned long long m = __builtin_amdgcn_ballot_w64(flagged) & gm;
                while (m != 0ull) {
                    const int j = j0 + __ffsll(m) - 1;
                    m &= m - 1ull;
                    const uint32_t mv = S.moves[j];
                    const int u = mv & 0xffff, v = (mv >> 16) & 0x3fff;
                    bool o = false;
                    int front = 0;
                    Work cw{0, 0};
                    const int c = decode_tg<NW, 16, COUNT>(S, D, S.region, Ly.long_len, u, v, 0, D.n, front, o, &cw);
                    if (tid == 0) {
                        if (COUNT) lw.add(cw);
                        const unsigned long long k = move_key(c, u, v, tabu.get(u, v), asp);
                        best = k < best ? k : best;
                        if (out_mk) out_mk[canon_index(D.n, delta, u, v)] = c;
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
        }
        __syncthreads();
    }
    // clear the flags, count the decodes that left the register profile
    if (*ovf_n > 0 || *ovf2_n > 0) {
        for (int j = tid; j < nfeas; j += T) S.moves[j] &= 0x3fffffffu;
        if (tid == 0 && ovf_total) *ovf_total += *ovf_n + *ovf2_n;
        __syncthreads();
    }
    if (COUNT) {
        const long long ops = block_sum_i64<T>(lw.ops, S.red);
        const long long cells = block_sum_i64<T>(lw.cells, S.red);
        if (tid == 0) work_total->add(Work{ops, cells});
    }
    return block_min_u64<T>(best, S.red);
}

// Lane-per-candidate (G = 1) or group decode (G > 2).
// Layout codes: G = 1 one candidate per lane with 16-bit finish times,
// G = 2 one candidate per lane with 8-bit finish times (lane profiles of at
// most 255 units), G = 16 one candidate per 16 lanes (time-indexed), G = 8
// one candidate per 8 lanes (capacity-indexed, a lane per resource),
// G = 64 one time-indexed candidate per wave, profile in registers.
template <int NW, int T, int DEC, int G, bool COUNT = false>
__device__ inline unsigned long long evaluate_any(const Sh &S, const InstDesc &D, const Layout &Ly, int nfeas, int L,
                                                  int delta, TabuSrc tabu, int asp, int *out_mk, long long *ovf_total,
                                                  Work *work_total = nullptr, bool share = true) {
    if constexpr (G == kLayoutWave) {
        static_assert(DEC == kEvalTime, "the wave layout is time-indexed");
        return evaluate_moves_w<NW, T, COUNT>(S, D, Ly, nfeas, delta, tabu, asp, out_mk, ovf_total, work_total,
                                              share);
    } else if constexpr (layout_is_group(G)) {
        return evaluate_moves_g<NW, T, DEC, G, COUNT>(S, D, Ly, nfeas, L, delta, tabu, asp, out_mk, ovf_total,
                                                      work_total, share);
    } else {
        return evaluate_moves<NW, T, DEC, COUNT, layout_finish_bits(G), G == kLayoutRegs>(
            S, D, Ly, nfeas, L, delta, tabu, asp, out_mk, ovf_total, work_total, share);
    }
}

// Finish-time bits of the lane records for a layout code.
template <int G>
constexpr int records_fb() { return layout_finish_bits(G); }

// ---------------------------------------------------------------------------
// rcpsp_evaluate_neighbourhood

template <int NW, int T, int DEC, int G>
__global__ __launch_bounds__(T, G == kLayoutRegs ? 2 : 1) void k_eval(EvalArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    const InstDesc &D = A.D;
    const Layout &Ly = A.Ly;
    Sh S = make_sh(lds, D, Ly);
    const int N = D.n, tid = threadIdx.x;
    stage_blob<T>(lds, D, Ly);
    __shared__ int err;
    if (tid == 0) err = 0;
    for (int p = tid; p < N; p += T) S.fs[p] = 0;
    __syncthreads();
    // the order must be a permutation with w_0 = 0, w_{N-1} = N-1 ...
    for (int p = tid; p < N; p += T) {
        const int a = A.order[p];
        if (a < 0 || a >= N) err = 1;
        else S.W[p] = (uint16_t)a;
    }
    __syncthreads();
    if (!err) {
        // every id seen exactly once: 16-bit counters, two per dword
        for (int p = tid; p < N; p += T) {
            const int a = S.W[p];
            const unsigned int prev =
                atomicAdd(reinterpret_cast<unsigned int *>(S.fs + (a & ~1)), (a & 1) ? 0x10000u : 1u);
            if (((prev >> ((a & 1) * 16)) & 0xffffu) != 0u) err = 1;
        }
        if (tid == 0 && (S.W[0] != 0 || S.W[N - 1] != N - 1)) err = 1;
    }
    __syncthreads();
    // ... and respect every precedence arc
    if (!err) {
        for (int p = tid; p < N; p += T) S.pos[S.W[p]] = (uint16_t)p;
        __syncthreads();
        for (int i = tid; i < N; i += T)
            for (int e = S.succoff[i]; e < S.succoff[i + 1]; ++e)
                if (S.pos[i] >= S.pos[S.succ[e]]) err = 1;
    }
    __syncthreads();
    if (err) {
        if (tid == 0) A.best[3] = -5;  // RCPSP_E_ORDER
        return;
    }
    const int nf = build_moves<T, records_fb<G>()>(S, D, A.delta);
    if (A.makespan) {
        for (int i = tid; i < A.P; i += T) A.makespan[i] = -1;
    }
    __syncthreads();
    TabuSrc tb{nullptr, A.tabu, 0, N};
    const unsigned long long k =
        evaluate_any<NW, T, DEC, G>(S, D, Ly, nf, A.L, A.delta, tb, A.aspiration, A.makespan, nullptr);
    if (tid == 0) {
        if (nf == 0) {
            A.best[0] = 0; A.best[1] = 0; A.best[2] = -1; A.best[3] = 0;
        } else {
            A.best[0] = (int)((k >> 16) & 0xffff);
            A.best[1] = (int)(k & 0xffff);
            A.best[2] = (int)((k >> 32) & 0x7fffffff);
            A.best[3] = nf;
        }
    }
}

// ---------------------------------------------------------------------------
// Tabu search
//
// The steps below are device functions so that one search plan (one
// instance, kernels launched per iteration) and a batch (many instances, one
// persistent workgroup per instance at a time) share them.  Global memory a
// step writes and a later step of the same workgroup reads is published with
// a fence before the closing barrier.

// Reset search i (if i < B) and working-set record i (if i < NF) of a plan.
// Initial orders (Section 4.1): the level order (levels ascending, ids
// ascending) with every level shuffled by Fisher-Yates on the stream
// (seed, i).  w: N 16-bit entries of LDS scratch.
template <int T>
__device__ void reset_unit(const SearchArgs &A, int i, uint16_t *w) {
    const InstDesc &D = A.D;
    const int tid = threadIdx.x, N = D.n, N2 = n2(N);
    const uint16_t *base = reinterpret_cast<const uint16_t *>(D.blob + D.off_base);
    const uint16_t *lvl = reinterpret_cast<const uint16_t *>(D.blob + D.off_lvl);
    const bool has_search = i < A.B, has_rec = i < A.NF;
    for (int p = tid; p < N; p += T) w[p] = base[p];
    __syncthreads();
    if (tid == 0) {
        uint64_t ctr = 0;
        for (int l = 0; l < D.n_levels; ++l) {
            const int b0 = lvl[l], len = lvl[l + 1] - lvl[l];
            for (int j = len - 1; j >= 1; --j) {
                const int r = (int)rng_below(A.seed, kStreamInit + (uint64_t)i, ctr++, (uint32_t)(j + 1));
                const uint16_t t = w[b0 + j];
                w[b0 + j] = w[b0 + r];
                w[b0 + r] = t;
            }
        }
    }
    __syncthreads();
    const int tcn = N * A.tcw;
    if (has_search) {
        if (A.NF == 0)
            for (int p = tid; p < N2; p += T) A.Wcur[(size_t)i * N2 + p] = p < N ? w[p] : 0;
        for (int x = tid; x < A.tl; x += T) A.ring[(size_t)i * A.tl + x] = 0;
        for (int x = tid; x < tcn; x += T) A.tc[(size_t)i * tcn + x] = 0;
        if (A.record && A.traj) {
            const size_t n4 = (size_t)A.iters * 4;
            for (size_t x = tid; x < n4; x += T) A.traj[(size_t)i * n4 + x] = -1;
        }
        if (tid == 0) {
            SearchScalars s = {};
            s.C_cur = 0x7fffffff; s.C_best = 0x7fffffff; s.C_imp = 0x7fffffff; s.C_read = 0x7fffffff;
            s.flags = A.NF == 0 ? kFlagInitDecode : 0;
            A.sc[i] = s;
        }
    }
    if (has_rec) {
        for (int p = tid; p < N2; p += T) A.Fw[(size_t)i * N2 + p] = p < N ? w[p] : 0;
        for (int x = tid; x < A.tl; x += T) A.Fring[(size_t)i * A.tl + x] = 0;
        for (int x = tid; x < tcn; x += T) A.Ftc[(size_t)i * tcn + x] = 0;
        if (tid == 0) {
            A.Fwidx[i] = 0;
            A.Fmeta[i].IC = 0; A.Fmeta[i].reads = 0; A.Fmeta[i].buf = 0; A.Fmeta[i].C = 0x7fffffff;
        }
    }
    if (i == 0 && tid == 0) {
        A.g->Cstar = 0x7fffffff;
        A.g->gstop = 0;
        A.g->queue = 0;
        // a time budget runs from the start of the run's first kernel
        A.g->deadline = A.budget_ticks > 0 ? (long long)wall_clock64() + A.budget_ticks : 0;
    }
    __threadfence();
    __syncthreads();
}

#ifdef RCPSP_PLAIN_KERNELS
__global__ __launch_bounds__(64) void k_reset(SearchArgs A) {
    __shared__ uint16_t w[kMaxN];
    reset_unit<64>(A, blockIdx.x, w);
}
#endif  // RCPSP_PLAIN_KERNELS

// Makespan of the order in S.W decoded from scratch over the whole decode
// region (at least the horizon): time-indexed by lanes 0-15 together,
// capacity-indexed by lanes 0-7 (group decodes).  Every thread of the
// workgroup calls it; the value is that of thread 0.
template <int NW, int DEC>
__device__ inline int decode_order(const Sh &S, const InstDesc &D, const Layout &Ly) {
    int c = 0;
    if constexpr (DEC == kEvalTime) {
        if (threadIdx.x < 16) {
            bool ovf = false;
            int front = 0;
            c = decode_tg<NW, 16, false, 16>(S, D, S.region, Ly.long_len, 0, 0, 0, D.n, front, ovf, nullptr);
        }
    } else {
        if (threadIdx.x < 8) {
            const int F0 = (D.n + 1) >> 1, Cd = (D.sum_r + 1) >> 1;
            for (int i = threadIdx.x; i < Cd; i += 8) S.region[F0 + i] = 0u;
            __builtin_amdgcn_wave_barrier();
            c = decode_cg<8>(S, D, S.region, 0, 0, 0, D.n, nullptr);
        }
    }
    return c;
}

// Activities in decreasing order of key (16-bit, by activity), ties by
// decreasing position in S.W, written to out[]: each thread ranks its
// activities by counting those ordered before them (keys and positions make
// the order strict).
template <int T>
__device__ inline void sort_desc(const Sh &S, const InstDesc &D, const uint16_t *key, uint16_t *out) {
    const int N = D.n;
    for (int p = threadIdx.x; p < N; p += T) S.pos[S.W[p]] = (uint16_t)p;
    __syncthreads();
    for (int a = threadIdx.x; a < N; a += T) {
        const int ka = key[a], pa = S.pos[a];
        int rank = 0;
        for (int b = 0; b < N; ++b) {
            const int kb = key[b], pb = S.pos[b];
            rank += (kb > ka) || (kb == ka && pb > pa);
        }
        out[rank] = (uint16_t)a;
    }
    __syncthreads();
}

// Forward-backward improvement of the activity list in S.W (in place): the
// backward pass is the serial SGS on the project with every arc reversed
// (successor lists taken as predecessor lists) over the activities by
// decreasing finish time; its finish times are measured back from the end,
// so the activities by decreasing backward finish are in increasing order of
// their right-justified starts, and the forward pass is the serial SGS over
// that list.  Ties: the later list position first (which keeps every list
// precedence-feasible for its pass).  Repeated while the forward makespan
// strictly decreases; the last list that decreased it stays.  Both passes use
// the search's decoder, decoding whole lists over the decode region (finish
// times as 16-bit values at its start).
template <int NW, int T, int DEC>
__device__ void fbi_order(const Sh &S, const InstDesc &D, const Layout &Ly, int *shc) {
    Sh R = S;
    R.pred = S.succ;
    R.predoff = S.succoff;
    const int N = D.n, N2h = n2(N) / 2;
    const uint16_t *fin = reinterpret_cast<const uint16_t *>(S.region);
    uint32_t *Wd = reinterpret_cast<uint32_t *>(S.W);
    uint32_t *Wk = reinterpret_cast<uint32_t *>(S.Wimp);   // the best list so far
    build_records<T>(S, D);
    __syncthreads();
    int c = decode_order<NW, DEC>(S, D, Ly);
    if (threadIdx.x == 0) shc[0] = c;
    __syncthreads();
    int C = shc[0];
    for (int i = threadIdx.x; i < N2h; i += T) Wk[i] = Wd[i];
    for (;;) {
        __syncthreads();
        // backward list: by decreasing finish time of the current schedule
        sort_desc<T>(S, D, fin, S.fs);
        for (int p = threadIdx.x; p < N; p += T) S.W[p] = S.fs[p];
        __syncthreads();
        build_records<T>(R, D);
        __syncthreads();
        decode_order<NW, DEC>(R, D, Ly);
        __syncthreads();
        // forward list: by decreasing backward finish time
        sort_desc<T>(S, D, fin, S.fs);
        for (int p = threadIdx.x; p < N; p += T) S.W[p] = S.fs[p];
        __syncthreads();
        build_records<T>(S, D);
        __syncthreads();
        c = decode_order<NW, DEC>(S, D, Ly);
        if (threadIdx.x == 0) shc[0] = c;
        __syncthreads();
        const int c2 = shc[0];
        if (c2 >= C) break;
        C = c2;
        for (int i = threadIdx.x; i < N2h; i += T) Wk[i] = Wd[i];
    }
    for (int i = threadIdx.x; i < N2h; i += T) Wd[i] = Wk[i];
    __syncthreads();
}

// Forward-backward improvement of every second initial solution: workgroup
// g takes unit 2g + 1 (a search's order without a working set, else a
// working-set record), right after the reset kernel wrote it.
template <int NW, int T, int DEC>
__global__ __launch_bounds__(T) void k_fbi(SearchArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ int shc[1];
    const InstDesc &D = A.D;
    Sh S = make_sh(lds, D, A.Ly);
    stage_blob<T>(lds, D, A.Ly);
    const int i = 2 * blockIdx.x + 1, N2h = n2(D.n) / 2;
    uint32_t *g = reinterpret_cast<uint32_t *>((A.NF > 0 ? A.Fw : A.Wcur) + (size_t)i * n2(D.n));
    uint32_t *Wd = reinterpret_cast<uint32_t *>(S.W);
    for (int x = threadIdx.x; x < N2h; x += T) Wd[x] = g[x];
    __syncthreads();
    fbi_order<NW, T, DEC>(S, D, A.Ly, shc);
    for (int x = threadIdx.x; x < N2h; x += T) g[x] = Wd[x];
    __threadfence();
}

// Makespan of initial working-set record k (buffer 0); the blob is staged.
template <int NW, int T, int DEC>
__device__ void decode_record(const SearchArgs &A, const Sh &S, int k) {
    const InstDesc &D = A.D;
    const int N2 = n2(D.n);
    const uint32_t *src = reinterpret_cast<const uint32_t *>(A.Fw + (size_t)k * N2);
    for (int i = threadIdx.x; i < N2 / 2; i += T) reinterpret_cast<uint32_t *>(S.W)[i] = src[i];
    __syncthreads();
    build_records<T>(S, D);
    __syncthreads();
    const int c = decode_order<NW, DEC>(S, D, A.Ly);
    if (threadIdx.x == 0) A.Fmeta[k].C = c;
    __threadfence();
    __syncthreads();
}

template <int NW, int T, int DEC>
__global__ __launch_bounds__(T) void k_decode_records(SearchArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    Sh S = make_sh(lds, A.D, A.Ly);
    stage_blob<T>(lds, A.D, A.Ly);
    __syncthreads();
    decode_record<NW, T, DEC>(A, S, blockIdx.x);
}

template <int T>
__device__ inline void copy_dw(uint32_t *dst, const uint32_t *src, int n) {
    for (int i = threadIdx.x; i < n; i += T) dst[i] = src[i];
}

// Per-workgroup scratch of a search step.
struct StepShared {
    SearchScalars sc;
    int dirty_best, dirty_imp;
    int expired;   // independent searches: the time budget has passed
};

// Search b, iterations [it0, it0 + n_it): complete a pending read (record
// or export, diversification), then iterate (neighbourhood, decode, best
// admissible move, Alg. 3), then export for the next exchange round.  The
// instance blob must be staged.  COUNT adds the algorithmic operations of
// every decode to the search's work counter.
template <int NW, int T, int DEC, int G, bool COUNT>
__device__ __attribute__((always_inline)) void search_step(const SearchArgs &A, const Sh &S, StepShared &ss, int b, int it0,
                                                         int n_it) {
    const InstDesc &D = A.D;
    const Layout &Ly = A.Ly;
    SearchScalars &sc = ss.sc;
    const int tid = threadIdx.x, N = D.n, N2 = n2(N);
    const int tcn = N * A.tcw;
    const bool coop = A.NF > 0;
    if (tid == 0) {
        sc = A.sc[b];
        ss.dirty_best = 0;
        ss.dirty_imp = 0;
    }
    __syncthreads();
    // control flow below depends on the flags as loaded; thread 0 rewrites
    // sc.flags later, so every thread takes its copy before that can happen.
    // After a global stop (the working set reached the critical path) a
    // read chosen by the last round is still completed, then nothing runs.
    const int flags0 = sc.flags;
    const bool gstop = A.g->gstop != 0;
    const bool skip = sc.stopped || (gstop && !(flags0 & (kFlagReadPending | kFlagInitDecode)));
    const int it_end = gstop ? it0 : it0 + n_it;
    __syncthreads();
    if (skip) return;
    uint32_t *Wd = reinterpret_cast<uint32_t *>(S.W);
    if (flags0 & kFlagReadPending) {
        const uint32_t *sw, *sr, *st;
        int swidx;
        if (sc.src_kind == kSrcRecord) {
            const size_t r = (size_t)sc.src_buf * A.NF + sc.src_idx;
            sw = reinterpret_cast<const uint32_t *>(A.Fw + r * N2);
            sr = A.Fring + r * A.tl;
            st = A.Ftc + r * tcn;
            swidx = A.Fwidx[r];
        } else {
            const size_t r = (size_t)sc.src_buf * A.B + sc.src_idx;
            sw = reinterpret_cast<const uint32_t *>(A.Xw + r * N2);
            sr = A.Xring + r * A.tl;
            st = A.Xtc + r * tcn;
            swidx = A.Xwidx[r];
        }
        copy_dw<T>(Wd, sw, N2 / 2);
        copy_dw<T>(S.ring, sr, A.tl);
        copy_dw<T>(S.tc, st, tcn);
        __syncthreads();
        if (tid == 0) {
            sc.widx = swidx;
            sc.C_cur = sc.src_C;
        }
        if (flags0 & kFlagDiversify) {
            // Section 6.1: phi_steps random feasible swaps, tabu list untouched
            for (int step = 0; step < A.phi_steps; ++step) {
                const int nf = random_swap<T>(S, D, A.delta, A.seed, kStreamDiversify + (uint64_t)b, &sc.rng_ctr);
                if (nf == 0) break;
            }
            build_records<T>(S, D);
            __syncthreads();
            const int c = decode_order<NW, DEC>(S, D, Ly);
            if (tid == 0) sc.C_cur = c;
        }
        __syncthreads();
        copy_dw<T>(reinterpret_cast<uint32_t *>(S.Wimp), Wd, N2 / 2);
        if (tid == 0) {
            sc.C_imp = sc.C_cur;
            if (sc.C_cur < sc.C_best) {
                sc.C_best = sc.C_cur;
                ss.dirty_best = 1;
            }
            sc.flags &= ~(kFlagReadPending | kFlagDiversify);
        }
        __syncthreads();
    } else {
        copy_dw<T>(Wd, reinterpret_cast<const uint32_t *>(A.Wcur + (size_t)b * N2), N2 / 2);
        copy_dw<T>(S.ring, A.ring + (size_t)b * A.tl, A.tl);
        copy_dw<T>(S.tc, A.tc + (size_t)b * tcn, tcn);
        if (coop) copy_dw<T>(reinterpret_cast<uint32_t *>(S.Wimp),
                             reinterpret_cast<const uint32_t *>(A.Wimp + (size_t)b * N2), N2 / 2);
        __syncthreads();
        if (flags0 & kFlagInitDecode) {
            build_records<T>(S, D);
            __syncthreads();
            const int c = decode_order<NW, DEC>(S, D, Ly);
            if (tid == 0) {
                sc.C_cur = c;
                sc.C_best = sc.C_cur;
                ss.dirty_best = 1;
                sc.flags &= ~kFlagInitDecode;
            }
            __syncthreads();
        }
    }
    const int dirty0 = ss.dirty_best;
    __syncthreads();
    if (dirty0) copy_dw<T>(reinterpret_cast<uint32_t *>(A.Wbest + (size_t)b * N2), Wd, N2 / 2);
    if (tid == 0) ss.dirty_best = 0;
    __syncthreads();

    TabuSrc tb{S.tc, nullptr, A.tcw, N};
    for (int it = it0; it < it_end; ++it) {
        // independent searches check a time budget at every iteration
        // boundary (one reading of the clock, shared by the workgroup); with
        // a working set the exchange round does
        bool past = false;
        if (!coop && A.budget_ticks > 0) {
            if (tid == 0) ss.expired = (long long)wall_clock64() >= A.g->deadline;
            __syncthreads();
            past = ss.expired != 0;
        }
        bool stop = sc.it_done >= A.iters || (!coop && sc.C_best == D.cp) || past;
        const int asp = coop ? min(sc.C_best, A.g->Cstar) : sc.C_best;
        __syncthreads();
        if (stop) {
            if (tid == 0 && sc.it_done < A.iters) sc.stopped = 1;
            break;
        }
        const int nf = build_moves<T, records_fb<G>()>(S, D, A.delta);
        if (nf == 0) {
            if (tid == 0) sc.stopped = 1;
            break;
        }
        Work wk{0, 0};
        const unsigned long long key =
            evaluate_any<NW, T, DEC, G, COUNT>(S, D, Ly, nf, A.L, A.delta, tb, asp, nullptr, &sc.overflow, &wk,
                                              !A.full_decode);
        if (tid == 0) {
            if (COUNT) {
                sc.work += wk.ops;
                sc.cells += wk.cells;
            }
            const int u = (int)((key >> 16) & 0xffff), v = (int)(key & 0xffff);
            const int c = (int)((key >> 32) & 0x7fffffff);
            const uint16_t t = S.W[u];
            S.W[u] = S.W[v];
            S.W[v] = t;
            // Alg. 3: evict the oldest entry, insert (u,v), advance the write index
            const uint32_t old = S.ring[sc.widx];
            if (old != 0u) {
                const int uo = old & 0xffff, vo = old >> 16, o = vo - uo - 1;
                S.tc[uo * A.tcw + (o >> 5)] &= ~(1u << (o & 31));
            }
            S.ring[sc.widx] = (uint32_t)u | ((uint32_t)v << 16);
            {
                const int o = v - u - 1;
                S.tc[u * A.tcw + (o >> 5)] |= 1u << (o & 31);
            }
            sc.widx = (sc.widx + 1) % A.tl;
            sc.C_cur = c;
            sc.evals += nf;
            if (c < sc.C_best) {
                sc.C_best = c;
                ss.dirty_best = 1;
            }
            if (A.record) {
                int *rec = A.traj + ((size_t)b * A.iters + it) * 4;
                rec[0] = u; rec[1] = v; rec[2] = c; rec[3] = sc.C_best;
            }
            sc.it_done++;
            if (coop) {
                sc.it_read++;
                if (c < sc.C_imp) {
                    sc.C_imp = c;
                    ss.dirty_imp = 1;
                }
                sc.fired = (sc.C_imp < sc.C_read) || (sc.it_read > sc.I_assigned);
            }
        }
        __syncthreads();
        const int db = ss.dirty_best, di = ss.dirty_imp;
        if (db) copy_dw<T>(reinterpret_cast<uint32_t *>(A.Wbest + (size_t)b * N2), Wd, N2 / 2);
        if (di) copy_dw<T>(reinterpret_cast<uint32_t *>(S.Wimp), Wd, N2 / 2);
        __syncthreads();
        if (tid == 0) {
            ss.dirty_best = 0;
            ss.dirty_imp = 0;
        }
        __syncthreads();
    }
    // export for the exchange round (two buffers by the parity of the block
    // of iterations between rounds: readers of this round's exports run in
    // the next block, while their writers may export again)
    if (coop && sc.fired && sc.C_imp < sc.C_read) {
        const int par = (it0 / A.every) & 1;
        const size_t r = (size_t)par * A.B + b;
        copy_dw<T>(reinterpret_cast<uint32_t *>(A.Xw + r * N2), reinterpret_cast<uint32_t *>(S.Wimp), N2 / 2);
        copy_dw<T>(A.Xring + r * A.tl, S.ring, A.tl);
        copy_dw<T>(A.Xtc + r * tcn, S.tc, tcn);
        if (tid == 0) A.Xwidx[r] = sc.widx;
    }
    copy_dw<T>(reinterpret_cast<uint32_t *>(A.Wcur + (size_t)b * N2), Wd, N2 / 2);
    copy_dw<T>(A.ring + (size_t)b * A.tl, S.ring, A.tl);
    copy_dw<T>(A.tc + (size_t)b * tcn, S.tc, tcn);
    if (coop)
        copy_dw<T>(reinterpret_cast<uint32_t *>(A.Wimp + (size_t)b * N2), reinterpret_cast<uint32_t *>(S.Wimp),
                   N2 / 2);
    __syncthreads();
    if (tid == 0) A.sc[b] = sc;
    __threadfence();
    __syncthreads();
}

// Iterations [it0, it0 + n_it) of every search of a plan: as many
// workgroups as fit the GPU at once, each taking searches from a queue
// (A.g->queue, zeroed by the reset kernel and after every exchange round), so
// no CU idles while searches remain and the slowest search of a fixed group
// no longer sets the pace.  Each search's step reads and writes only its own
// state, so results do not depend on which workgroup runs it.
template <int NW, int T, int DEC, int G, bool COUNT>
__global__ __launch_bounds__(T, G == kLayoutRegs ? 2 : 1) void k_search(SearchArgs A) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ StepShared ss;
    __shared__ int next;
    Sh S = make_sh(lds, A.D, A.Ly);
    stage_blob<T>(lds, A.D, A.Ly);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) next = atomicAdd(&A.g->queue, 1);
        __syncthreads();
        const int b = next;
        if (b >= A.B) break;
        search_step<NW, T, DEC, G, COUNT>(A, S, ss, b, A.it0, A.n_it);
    }
}

// eq. 8, read as floor(I_block (4 E[a] + E[b]) / (25 * 2^24)) >= 1 with the
// decay table E[j] ~ 2^24 exp(-j/256).
__device__ inline int iterations_assigned(int iblock, int ck, int cstar, int ic, const uint32_t *E, int elen) {
    const long long a = cstar > 0 ? (25600ll * (ck - cstar)) / cstar : 0;
    const long long bq = iblock > 0 ? (1024ll * ic) / iblock : 0;
    const long long ea = (a >= 0 && a < elen) ? E[a] : 0;
    const long long eb = (bq >= 0 && bq < elen) ? E[bq] : 0;
    const long long ia = ((long long)iblock * (4 * ea + eb)) / (25ll << 24);
    return ia < 1 ? 1 : (int)ia;
}

// Working-set exchange round (Section 6.1).  Searches whose exchange
// condition fired are taken in ascending id: each writes its best solution
// since its last read to the record it read (if it improved that solution and
// beats the record's current content) and reads the next record.  The
// bookkeeping is sequential; the data moves are done by the readers
// themselves in their next step, from the record buffer or from the writer's
// export buffer they were pointed at.  rs: 6B + 5NF ints of LDS scratch.
//
// The fired searches are first listed in ascending id (wave ballots); one
// thread then walks the list touching LDS only, and leaves per search what
// its read saw (source, record makespan, C* and the record's iteration count
// at that moment); eq. 8's table lookups and the searches' scalars in global
// memory are done afterwards by all threads.
template <int T>
__device__ void exchange_round(const SearchArgs &A, int parity, int init, int *rs) {
    const int B = A.B, NF = A.NF, tid = threadIdx.x, N2 = n2(A.D.n), tcn = A.D.n * A.tcw;
    // per search b (in order of use): fired flag, then the read's source;
    // slot; iterations since the read, then the record's count at the read;
    // C_imp, then the record's makespan; C_read, then C* at the read
    int *fired = rs, *slot = rs + B, *itr = rs + 2 * B, *cimp = rs + 3 * B, *cread = rs + 4 * B;
    int *list = rs + 5 * B;
    int *fC = rs + 6 * B, *fIC = fC + NF, *fR = fIC + NF, *fB = fR + NF, *content = fB + NF;
    __shared__ int wcnt[T / 64];
    __shared__ int nfired, cstar_s;
    for (int b = tid; b < B; b += T) {
        const SearchScalars &s = A.sc[b];
        if (init) {
            fired[b] = 1;
            slot[b] = (b + NF - 1) % NF;
            itr[b] = 0;
            cimp[b] = 0x7fffffff;
            cread[b] = 0x7fffffff;
        } else {
            fired[b] = s.fired && !s.stopped;
            slot[b] = s.slot;
            itr[b] = s.it_read;
            cimp[b] = s.C_imp;
            cread[b] = s.C_read;
        }
    }
    for (int k = tid; k < NF; k += T) {
        fC[k] = A.Fmeta[k].C;
        fIC[k] = A.Fmeta[k].IC;
        fR[k] = A.Fmeta[k].reads;
        fB[k] = A.Fmeta[k].buf;
        content[k] = -1;
    }
    __syncthreads();
    // list of the fired searches in ascending id
    {
        const int w = tid >> 6, lane = tid & 63;
        int base = 0;
        for (int b0 = 0; b0 < B; b0 += T) {
            const int b = b0 + tid;
            const bool f = b < B && fired[b] != 0;
            const unsigned long long m = __ballot(f);
            if (lane == 0) wcnt[w] = __popcll(m);
            __syncthreads();
            int off = base, tot = 0;
#pragma unroll
            for (int j = 0; j < T / 64; ++j) {
                off += j < w ? wcnt[j] : 0;
                tot += wcnt[j];
            }
            if (f) list[off + __popcll(m & ((1ull << lane) - 1ull))] = b;
            base += tot;
            __syncthreads();
        }
        if (tid == 0) nfired = base;
    }
    if (tid == 0) {
        int cstar = 0x7fffffff;
        for (int k = 0; k < NF; ++k) cstar = min(cstar, fC[k]);
        const int nf = nfired;
        for (int i = 0; i < nf; ++i) {
            const int b = list[i];
            const int k = slot[b];
            const int ci = cimp[b], cr = cread[b];
            fIC[k] += itr[b];
            if (ci < cr && ci < fC[k]) {
                fC[k] = ci;
                fIC[k] = 0;
                fR[k] = 0;
                content[k] = b;
                cstar = min(cstar, ci);
            }
            const int k2 = (k + 1) % NF;
            const int reads = fR[k2] + 1;
            fR[k2] = reads;
            // the source: bits 0-23 index (searches and records number far
            // fewer: 6B ints of scratch fit in LDS), bit 24 export, bit 25
            // buffer, bit 26 diversify
            const int w = content[k2];
            const int src = w < 0 ? (k2 | (fB[k2] << 25)) : (w | (1 << 24) | (parity << 25));
            fired[b] = src | (reads > A.phi_max ? 1 << 26 : 0);
            cimp[b] = fC[k2];
            cread[b] = cstar;
            itr[b] = fIC[k2];
        }
        cstar_s = cstar;
    }
    __syncthreads();
    for (int i = tid; i < nfired; i += T) {
        const int b = list[i];
        const int src = fired[b];
        SearchScalars &s = A.sc[b];
        s.src_kind = (src >> 24) & 1 ? kSrcExport : kSrcRecord;
        s.src_idx = src & 0xffffff;
        s.src_buf = (src >> 25) & 1;
        s.src_C = cimp[b];
        s.C_read = cimp[b];
        s.I_assigned = iterations_assigned(A.iters, cimp[b], cread[b], itr[b], A.decay, A.decay_len);
        s.flags |= kFlagReadPending | ((src >> 26) & 1 ? kFlagDiversify : 0);
        s.slot = (slot[b] + 1) % NF;
        s.it_read = 0;
        s.fired = 0;
    }
    __syncthreads();
    // final content of each written record -> its other buffer
    for (int k = 0; k < NF; ++k) {
        const int w = content[k];
        if (w < 0) continue;
        const size_t src = (size_t)parity * B + w;
        const size_t dst = (size_t)(fB[k] ^ 1) * NF + k;
        for (int i = tid; i < N2 / 2; i += T)
            reinterpret_cast<uint32_t *>(A.Fw + dst * N2)[i] = reinterpret_cast<const uint32_t *>(A.Xw + src * N2)[i];
        for (int i = tid; i < A.tl; i += T) A.Fring[dst * A.tl + i] = A.Xring[src * A.tl + i];
        for (int i = tid; i < tcn; i += T) A.Ftc[dst * tcn + i] = A.Xtc[src * tcn + i];
        if (tid == 0) A.Fwidx[dst] = A.Xwidx[src];
    }
    __syncthreads();
    for (int k = tid; k < NF; k += T) {
        A.Fmeta[k].C = fC[k];
        A.Fmeta[k].IC = fIC[k];
        A.Fmeta[k].reads = fR[k];
        A.Fmeta[k].buf = content[k] >= 0 ? (fB[k] ^ 1) : fB[k];
    }
    if (tid == 0) {
        A.g->Cstar = cstar_s;
        A.g->gstop = cstar_s == A.D.cp;
    }
    __threadfence();
    __syncthreads();
}

#ifdef RCPSP_PLAIN_KERNELS
__global__ __launch_bounds__(256) void k_round(SearchArgs A, int parity, int init) {
    extern __shared__ int rs[];
    // a time budget that has passed ends the run at this iteration boundary:
    // no round, and every later iteration launch finds the stop flag
    if (!init && A.budget_ticks > 0) {
        __shared__ int past;
        if (threadIdx.x == 0) past = (long long)wall_clock64() >= A.g->deadline;
        __syncthreads();
        if (past) {
            if (threadIdx.x == 0) {
                A.g->gstop = 1;
                A.g->queue = 0;
            }
            return;
        }
    }
    exchange_round<256>(A, parity, init, rs);
    if (threadIdx.x == 0) A.g->queue = 0;   // the next iteration launch starts from search 0
}
#endif  // RCPSP_PLAIN_KERNELS

// ---------------------------------------------------------------------------
// Batches: many instances, each with its own search plan, in one persistent
// launch per class (decoder, profile width, threads, workgroups per CU).
// Work is split into tasks taken from a queue in a fixed order: first one
// set-up task per instance (reset, initial working-set records, first
// exchange round), then, iteration by iteration, one task per (instance,
// search) running that search's iteration.  A search task waits until the
// instance's previous exchange round is done; the task that completes the
// last search of an iteration runs the instance's next round.  Every task a
// task waits for comes earlier in the queue and is held by a running
// workgroup, so the waits always end; a wait that exceeds a time limit sets
// the abort flag, and every workgroup then leaves.  Every instance's result
// equals that of its own plan: the searches and rounds see the same states
// in the same order.

struct BatchQueue {
    unsigned long long next;
    int abort;
    int pad[13];
};

__device__ inline int upper_index_ll(const long long *a, int n, long long x) {
    // largest i in [0, n) with a[i] <= x (a ascending, a[0] <= x)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline int upper_index(const int *a, int n, int x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

static_assert(sizeof(SearchArgs) + sizeof(StepShared) + 4 * sizeof(int) + 64 <= kBatchStaticLds,
              "batch kernel static LDS");

template <int NW, int T, int DEC, int G>
__global__ __launch_bounds__(T, G == kLayoutRegs ? 2 : 1) void k_batch(BatchClassArgs C) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ SearchArgs A;
    __shared__ StepShared ss;
    __shared__ int task[4];
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const long long t = (long long)atomicAdd(&C.q->next, 1ull);
            int ok = t < C.total && __hip_atomic_load(&C.q->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
            int j = 0, it = -1, b = 0;
            if (ok && t >= C.count) {
                it = upper_index_ll(C.off, C.max_steps + 1, t);
                const int r = (int)(t - C.off[it]);
                j = upper_index(C.cumB, C.act[it] + 1, r);
                b = r - C.cumB[j];
                // the instance's previous exchange round (or its set-up)
                const long long t0 = (long long)wall_clock64();
                while (__hip_atomic_load(&C.epoch[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < it + 1) {
                    if ((long long)wall_clock64() - t0 > C.wait_ticks ||
                        __hip_atomic_load(&C.q->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        atomicExch(&C.q->abort, 1);
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            } else if (ok) {
                j = (int)t;
            }
            task[0] = ok; task[1] = j; task[2] = it; task[3] = b;
        }
        __syncthreads();
        const int ok = task[0], j = task[1], it = task[2], b = task[3];
        if (!ok) break;
        __threadfence();
        {
            const uint32_t *src = reinterpret_cast<const uint32_t *>(C.items + C.order[j]);
            uint32_t *dst = reinterpret_cast<uint32_t *>(&A);
            for (int i = tid; i < (int)(sizeof(SearchArgs) / 4); i += T) dst[i] = src[i];
        }
        __syncthreads();
        Sh S = make_sh(lds, A.D, A.Ly);
        const int steps = A.NF > 0 ? (A.iters > 0 ? A.iters : 1) : 1;
        if (it < 0) {
            // set-up: reset every search and record, decode the records, first round
            uint16_t *scratch16 = reinterpret_cast<uint16_t *>(S.region);
            const int units = A.B > A.NF ? A.B : A.NF;
            for (int i = 0; i < units; ++i) reset_unit<T>(A, i, scratch16);
            stage_blob<T>(lds, A.D, A.Ly);
            __syncthreads();
            if (A.NF > 0) {
                for (int k = 0; k < A.NF; ++k) decode_record<NW, T, DEC>(A, S, k);
                exchange_round<T>(A, 0, 1, reinterpret_cast<int *>(S.region));
            }
            if (tid == 0) __hip_atomic_store(&C.epoch[j], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            continue;
        }
        stage_blob<T>(lds, A.D, A.Ly);
        __syncthreads();
        if (A.NF > 0) search_step<NW, T, DEC, G, false>(A, S, ss, b, it, A.iters > 0 ? 1 : 0);
        else search_step<NW, T, DEC, G, false>(A, S, ss, b, 0, A.iters);
        if (tid == 0) {
            const int old = __hip_atomic_fetch_add(&C.done[j], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            task[0] = old + 1 == (it + 1) * A.B && A.NF > 0 && it < steps - 1;
        }
        __syncthreads();
        const int last = task[0];
        __syncthreads();
        if (last) {
            __threadfence();
            exchange_round<T>(A, it & 1, 0, reinterpret_cast<int *>(S.region));
            if (tid == 0) __hip_atomic_store(&C.epoch[j], it + 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
        }
    }
}

#ifdef RCPSP_PLAIN_KERNELS
// Clear n ints (a kernel, so that graph replays never record a memset).
__global__ void k_fill_zero(int *p, long long n) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
#endif  // RCPSP_PLAIN_KERNELS

// ---------------------------------------------------------------------------
// Serving: requests arrive over time; each keeps its search state in device
// memory and advances in time slices.  A slice is one persistent launch per
// class over a task queue that grows while it runs: the host seeds it with
// the tasks left from the previous slice and a set-up task per new request;
// the task that completes the last search of an iteration ends the request
// (allowance, deadline, global stop, cancel) or runs its exchange round and
// queues the next iteration's tasks.  Workgroups take no task after the
// slice's end time, and a finished task's slot is marked done, so the host
// carries every queued task that did not run over to the next slice: a slice
// ends one task duration after its end time, whatever the backlog.  A task
// is counted in `pending` from being queued until it finishes, so pending = 0
// means no task can be queued any more.  Tasks only ever wait for the queue,
// never for each other.

template <int NW, int T, int DEC, int G>
__global__ __launch_bounds__(T, G == kLayoutRegs ? 2 : 1) void k_serve(ServeArgs C) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ SearchArgs A;
    __shared__ StepShared ss;
    __shared__ long long tk, hslot;
    __shared__ int flag;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            long long task = -1;
            unsigned long long h = ~0ull;
            if ((long long)wall_clock64() < C.slice_end) h = atomicAdd(&C.q->head, 1ull);
            if (h < (unsigned long long)C.cap) {
                const long long t0 = (long long)wall_clock64();
                for (;;) {
                    const unsigned long long v =
                        __hip_atomic_load(&C.tasks[h], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    if (v != 0ull) {
                        task = (long long)(v - 1ull);
                        break;
                    }
                    // nothing can arrive any more, or the slice is over (a task
                    // that lands here later is carried over by the host)
                    if (__hip_atomic_load(&C.q->pending, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) break;
                    const long long now = (long long)wall_clock64();
                    if (now >= C.slice_end) break;
                    if (now - t0 > C.wait_ticks ||
                        __hip_atomic_load(&C.q->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        atomicExch(&C.q->abort, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            tk = task;
            hslot = (long long)h;
        }
        __syncthreads();
        const long long task = tk;
        const long long my_slot = hslot;
        __syncthreads();
        if (task < 0) break;
        __threadfence();
        const int slot = (int)((unsigned long long)task >> 44);
        const int kind = (int)(((unsigned long long)task >> 43) & 1ull);
        const int b = (int)(((unsigned long long)task >> 27) & 0xffffull);
        const int it = (int)((unsigned long long)task & 0x7ffffffull);
        {
            const uint32_t *src = reinterpret_cast<const uint32_t *>(C.items + slot);
            uint32_t *dst = reinterpret_cast<uint32_t *>(&A);
            for (int i = tid; i < (int)(sizeof(SearchArgs) / 4); i += T) dst[i] = src[i];
        }
        __syncthreads();
        Sh S = make_sh(lds, A.D, A.Ly);
        ServeReq *R = C.req + slot;
        int next = -1;
        if (kind == 0) {
            uint16_t *scratch16 = reinterpret_cast<uint16_t *>(S.region);
            const int units = A.B > A.NF ? A.B : A.NF;
            for (int i = 0; i < units; ++i) reset_unit<T>(A, i, scratch16);
            stage_blob<T>(lds, A.D, A.Ly);
            __syncthreads();
            if (A.NF > 0) {
                for (int k = 0; k < A.NF; ++k) decode_record<NW, T, DEC>(A, S, k);
                exchange_round<T>(A, 0, 1, reinterpret_cast<int *>(S.region));
            }
            // a request whose budget ran out during set-up (it waited for a
            // workgroup) runs no iteration: its searches only finish their
            // set-up, and it ends with its initial solutions
            if (tid == 0) {
                const int cancel = __hip_atomic_load(&R->cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                flag = ((long long)wall_clock64() >= R->deadline || cancel) ? 1 : 0;
            }
            __syncthreads();
            next = flag ? kServeNoIteration : 0;
            __syncthreads();
        } else {
            const bool none = it == kServeNoIteration;
            stage_blob<T>(lds, A.D, A.Ly);
            __syncthreads();
            search_step<NW, T, DEC, G, false>(A, S, ss, b, none ? 0 : it, none ? 0 : 1);
            if (tid == 0) {
                const int old = __hip_atomic_fetch_add(&R->done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                int fin = -1;
                if (old + 1 == A.B) {
                    // every search finished iteration `it`: end here or continue
                    R->done = 0;
                    const long long now = (long long)wall_clock64();
                    int all_stopped = 1, best = 0x7fffffff;
                    long long evals = 0;
                    for (int s = 0; s < A.B; ++s) {
                        all_stopped &= A.sc[s].stopped != 0;
                        best = min(best, A.sc[s].C_best);
                        evals += A.sc[s].evals;
                    }
                    for (int k = 0; k < A.NF; ++k) best = min(best, A.Fmeta[k].C);
                    const int gstop = A.NF > 0 && A.g->gstop != 0;
                    const int cancel = __hip_atomic_load(&R->cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    fin = none || it + 1 >= R->max_iters || now >= R->deadline || all_stopped || gstop || cancel;
                    if (fin) {
                        R->best = best;
                        R->evals = evals;
                        R->replay_iters = none ? 0 : it + 1;
                        R->done_ticks = now;
                        R->next_iter = -1;
                        __hip_atomic_store(&R->finished, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                flag = fin;
            }
            __syncthreads();
            const int fin = flag;
            __syncthreads();
            if (fin == 0) {
                __threadfence();
                if (A.NF > 0) exchange_round<T>(A, it & 1, 0, reinterpret_cast<int *>(S.region));
                next = it + 1;
            }
        }
        if (tid == 0) {
            if (next >= 0) {
                // queue the next iteration (the host seeds it if the queue is full)
                const unsigned long long t = atomicAdd(&C.q->tail, (unsigned long long)A.B);
                if ((long long)(t + A.B) <= C.cap) {
                    R->next_iter = -2;
                    __hip_atomic_fetch_add(&C.q->pending, (long long)A.B, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                    for (int s = 0; s < A.B; ++s)
                        __hip_atomic_store(&C.tasks[t + s], serve_task(slot, 1, s, next) + 1ull, __ATOMIC_RELEASE,
                                           __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    R->next_iter = next;
                }
            }
            __threadfence();
            __hip_atomic_store(&C.tasks[my_slot], kServeTaskDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&C.q->pending, -1ll, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// Slice start: queue header (n0 tasks already copied to tasks[0, n0)) and the
// rest of the task array cleared.
#ifdef RCPSP_PLAIN_KERNELS
__global__ void k_serve_begin(ServeQueue *q, unsigned long long *tasks, long long cap, long long n0) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n0 && i < cap) tasks[i] = 0ull;
    if (i == 0) {
        q->head = 0ull;
        q->tail = (unsigned long long)n0;
        q->pending = n0;
        q->abort = 0;
    }
}
#endif  // RCPSP_PLAIN_KERNELS

#ifdef RCPSP_PLAIN_KERNELS
// Device wall clock (ticks) for the host's clock mapping.
__global__ void k_clock(long long *out) {
    if (threadIdx.x == 0) out[0] = (long long)wall_clock64();
}
#endif  // RCPSP_PLAIN_KERNELS

// ---------------------------------------------------------------------------
// Launch-shape dispatch shared by the launchers

#define RCPSP_DISPATCH(NWV, TV, DECV, GV, CALL)                                                                      \
    switch (DECV) {                                                                                                  \
    case kEvalCapacity:                                                                                              \
        switch ((TV) * 128 + (GV)) {                                                                                 \
        case 64 * 128 + 1: { constexpr int T_ = 64, NW_ = 1, DEC_ = kEvalCapacity, G_ = 1; CALL; } break;            \
        case 128 * 128 + 1: { constexpr int T_ = 128, NW_ = 1, DEC_ = kEvalCapacity, G_ = 1; CALL; } break;          \
        case 256 * 128 + 1: { constexpr int T_ = 256, NW_ = 1, DEC_ = kEvalCapacity, G_ = 1; CALL; } break;          \
        case 64 * 128 + 8: { constexpr int T_ = 64, NW_ = 1, DEC_ = kEvalCapacity, G_ = 8; CALL; } break;            \
        case 128 * 128 + 8: { constexpr int T_ = 128, NW_ = 1, DEC_ = kEvalCapacity, G_ = 8; CALL; } break;          \
        case 256 * 128 + 8: { constexpr int T_ = 256, NW_ = 1, DEC_ = kEvalCapacity, G_ = 8; CALL; } break;          \
        case 512 * 128 + 8: { constexpr int T_ = 512, NW_ = 1, DEC_ = kEvalCapacity, G_ = 8; CALL; } break;          \
        default: return hipErrorInvalidValue;                                                                        \
        }                                                                                                            \
        break;                                                                                                       \
    default:                                                                                                         \
        switch (((TV) * 16 + (NWV)) * 128 + (GV)) {                                                                  \
        case (64 * 16 + 1) * 128 + 1: { constexpr int T_ = 64, NW_ = 1, DEC_ = kEvalTime, G_ = 1; CALL; } break;     \
        case (64 * 16 + 1) * 128 + 2: { constexpr int T_ = 64, NW_ = 1, DEC_ = kEvalTime, G_ = 2; CALL; } break;     \
        case (64 * 16 + 1) * 128 + 16: { constexpr int T_ = 64, NW_ = 1, DEC_ = kEvalTime, G_ = 16; CALL; } break;   \
        case (64 * 16 + 2) * 128 + 1: { constexpr int T_ = 64, NW_ = 2, DEC_ = kEvalTime, G_ = 1; CALL; } break;     \
        case (64 * 16 + 2) * 128 + 2: { constexpr int T_ = 64, NW_ = 2, DEC_ = kEvalTime, G_ = 2; CALL; } break;     \
        case (64 * 16 + 2) * 128 + 16: { constexpr int T_ = 64, NW_ = 2, DEC_ = kEvalTime, G_ = 16; CALL; } break;   \
        case (64 * 16 + 4) * 128 + 1: { constexpr int T_ = 64, NW_ = 4, DEC_ = kEvalTime, G_ = 1; CALL; } break;     \
        case (64 * 16 + 4) * 128 + 2: { constexpr int T_ = 64, NW_ = 4, DEC_ = kEvalTime, G_ = 2; CALL; } break;     \
        case (64 * 16 + 4) * 128 + 16: { constexpr int T_ = 64, NW_ = 4, DEC_ = kEvalTime, G_ = 16; CALL; } break;   \
        case (128 * 16 + 1) * 128 + 1: { constexpr int T_ = 128, NW_ = 1, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (128 * 16 + 1) * 128 + 2: { constexpr int T_ = 128, NW_ = 1, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (128 * 16 + 1) * 128 + 16: { constexpr int T_ = 128, NW_ = 1, DEC_ = kEvalTime, G_ = 16; CALL; } break; \
        case (128 * 16 + 2) * 128 + 1: { constexpr int T_ = 128, NW_ = 2, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (128 * 16 + 2) * 128 + 2: { constexpr int T_ = 128, NW_ = 2, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (128 * 16 + 2) * 128 + 16: { constexpr int T_ = 128, NW_ = 2, DEC_ = kEvalTime, G_ = 16; CALL; } break; \
        case (128 * 16 + 4) * 128 + 1: { constexpr int T_ = 128, NW_ = 4, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (128 * 16 + 4) * 128 + 2: { constexpr int T_ = 128, NW_ = 4, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (128 * 16 + 4) * 128 + 16: { constexpr int T_ = 128, NW_ = 4, DEC_ = kEvalTime, G_ = 16; CALL; } break; \
        case (192 * 16 + 1) * 128 + 1: { constexpr int T_ = 192, NW_ = 1, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (192 * 16 + 1) * 128 + 2: { constexpr int T_ = 192, NW_ = 1, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (192 * 16 + 2) * 128 + 1: { constexpr int T_ = 192, NW_ = 2, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (192 * 16 + 2) * 128 + 2: { constexpr int T_ = 192, NW_ = 2, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (192 * 16 + 4) * 128 + 1: { constexpr int T_ = 192, NW_ = 4, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (192 * 16 + 4) * 128 + 2: { constexpr int T_ = 192, NW_ = 4, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (256 * 16 + 1) * 128 + 1: { constexpr int T_ = 256, NW_ = 1, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (256 * 16 + 1) * 128 + 2: { constexpr int T_ = 256, NW_ = 1, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (256 * 16 + 1) * 128 + 16: { constexpr int T_ = 256, NW_ = 1, DEC_ = kEvalTime, G_ = 16; CALL; } break; \
        case (256 * 16 + 1) * 128 + 4: { constexpr int T_ = 256, NW_ = 1, DEC_ = kEvalTime, G_ = 4; CALL; } break;   \
        case (256 * 16 + 2) * 128 + 1: { constexpr int T_ = 256, NW_ = 2, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (256 * 16 + 2) * 128 + 2: { constexpr int T_ = 256, NW_ = 2, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (256 * 16 + 2) * 128 + 16: { constexpr int T_ = 256, NW_ = 2, DEC_ = kEvalTime, G_ = 16; CALL; } break; \
        case (256 * 16 + 4) * 128 + 1: { constexpr int T_ = 256, NW_ = 4, DEC_ = kEvalTime, G_ = 1; CALL; } break;   \
        case (256 * 16 + 4) * 128 + 2: { constexpr int T_ = 256, NW_ = 4, DEC_ = kEvalTime, G_ = 2; CALL; } break;   \
        case (256 * 16 + 4) * 128 + 16: { constexpr int T_ = 256, NW_ = 4, DEC_ = kEvalTime, G_ = 16; CALL; } break; \
        case (512 * 16 + 1) * 128 + 64: { constexpr int T_ = 512, NW_ = 1, DEC_ = kEvalTime, G_ = 64; CALL; } break;\
        case (512 * 16 + 2) * 128 + 64: { constexpr int T_ = 512, NW_ = 2, DEC_ = kEvalTime, G_ = 64; CALL; } break;\
        case (512 * 16 + 4) * 128 + 64: { constexpr int T_ = 512, NW_ = 4, DEC_ = kEvalTime, G_ = 64; CALL; } break;\
        default: return hipErrorInvalidValue;                                                                        \
        }                                                                                                            \
    }

template <typename K>
static hipError_t set_lds(K kernel, size_t lds) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds);
}

}  // namespace rcpsp
