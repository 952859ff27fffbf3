// Library-internal definitions shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rcpsp {

constexpr int kMaxM = 16;        // resources
constexpr int kMaxN = 2048;      // activities incl. dummies (positions fit in 16 bits)
constexpr int kMaxNW = 4;        // dwords per packed time slot of the time-indexed profile
constexpr int kMaxDelta = 64;    // swap range
constexpr int kMaxHorizon = 32767;  // times are stored in 16 bits
constexpr int kMaxLds = 160 * 1024; // LDS per workgroup on gfx950

constexpr int kEvalTime = 1;
constexpr int kEvalCapacity = 2;

// Candidate layouts (the template argument G of the kernels):
//   1  one candidate per lane, 16-bit finish times, profile in LDS
//   2  one candidate per lane, 8-bit finish times, profile in LDS
//   4  one candidate per lane, 8-bit finish times, time-indexed profile of
//      kRegUnits time units in registers (one dword per unit)
//   8  one capacity-indexed candidate per 8 lanes (a lane per resource)
//   16 one time-indexed candidate per 16 lanes
//   64 one time-indexed candidate per wave, its profile spread over the
//      wave's registers (kWaveDwords dwords per lane: 64 * kWaveDwords / NW
//      time units), kWaveThreads threads
constexpr int kLayoutRegs = 4;
constexpr int kRegUnits = 160;
constexpr int kLayoutWave = 64;
constexpr int kWaveDwords = 32;
constexpr int kWaveThreads = 512;
constexpr int kWaveMaxN = 1024;  // finish times in registers: 16 per lane
__host__ __device__ constexpr int wave_profile_units(int nw) { return 64 * (kWaveDwords / nw); }
// A layout instantiated at T threads for decoder dec, for the set-up kernels
// (which depend on T only): 512 threads exist for one candidate per wave
// (time-indexed) and 8 lanes per candidate (capacity-indexed).
__host__ __device__ constexpr int setup_layout(int T, int dec) {
    return T == 512 ? (dec == kEvalTime ? kLayoutWave : 8) : 1;
}
__host__ __device__ constexpr bool layout_is_group(int G) { return G == 8 || G == 16; }
__host__ __device__ constexpr int layout_finish_bits(int G) { return (G == 2 || G == kLayoutRegs) ? 8 : 16; }

// Dwords of n finish times of fb bits at the start of a candidate state.
__host__ __device__ constexpr int finish_dwords(int n, int fb) { return fb == 8 ? (n + 3) >> 2 : (n + 1) >> 1; }

// Packed instance, passed by value to every kernel.  The arrays live in one
// device blob (dword sections) that kernels copy into LDS.
struct InstDesc {
    int n, m, n_arcs, horizon, cp;
    int nw;          // dwords per time slot (time-indexed profile)
    int fbits;       // 8 or 16 bits per resource field
    int sum_r;       // sum of R_k: capacity-indexed state size (16-bit entries)
    int copy_p;      // capacity-indexed copy ring length (power of two >= max request)
    int n_levels;
    uint32_t guard[kMaxNW];  // top bit of every field
    uint32_t full[kMaxNW];   // R_k of every field, with its guard bit set
    int R[kMaxM];
    int cbase[kMaxM];        // first entry of c_k in the capacity-indexed state
    // blob sections (dword offsets)
    int off_dur, off_predoff, off_pred, off_succoff, off_succ, off_rq, off_reqk, off_base, off_lvl, off_res;
    int blob_dwords;
    const uint32_t *blob;
};

// Dword offsets of the workgroup's LDS areas.
struct Layout {
    int blob, W, Wimp, pos, fs, lp, cnt, tc, ring, moves, prec, prq, predT, pin, pid, bst, red, scal, region;
    int per_lane;    // dwords of private decode state per candidate slot
    int base_stride; // dwords of the workgroup's base decode (one-candidate-per-lane layouts)
    int cands;       // candidate slots per round (threads, or threads / lanes per candidate)
    int long_len;    // time slots available to the single-thread long-profile decode
    int total;       // dwords
};

// Per-search scalar state in device memory.
struct SearchScalars {
    int C_cur, C_best, C_imp, C_read;
    int it_done, it_read, I_assigned, slot;
    int fired, stopped, widx, flags;
    int src_kind, src_idx, src_buf, src_C;
    unsigned long long rng_ctr;
    long long evals;
    long long overflow;
    long long work;      // algorithmic operations of all decodes (counting runs only)
    long long cells;     // resource-state cells among them (profile units / capacity entries)
};

enum : int {
    kFlagInitDecode = 1,   // decode the initial order at the first launch
    kFlagReadPending = 2,  // take the record chosen by the last exchange round
    kFlagDiversify = 4     // and diversify it
};
enum : int { kSrcRecord = 0, kSrcExport = 1 };

struct SlotMeta {
    int C, IC, reads, buf;
};

struct Global {
    int Cstar;
    int gstop;
    int queue;     // next search of the current iteration launch (plain plans)
    int pad;
    long long deadline;   // device wall-clock tick after which no iteration starts (time budget)
};

constexpr uint64_t kStreamInit = 0ull;
constexpr uint64_t kStreamDiversify = 1ull << 32;

// Search plan arguments for the kernels.
struct SearchArgs {
    InstDesc D;
    Layout Ly;
    int delta, tl, iters, B, NF, phi_max, phi_steps, tcw, L, record, count_work, full_decode;
    int it0, n_it;
    int grid;      // iteration-kernel workgroups (each takes searches from A.g->queue)
    int decay_len;
    int every;     // iterations between exchange rounds (>= 1)
    int pad_every;
    long long budget_ticks;   // time budget in device wall-clock ticks (0 = none)
    unsigned long long seed;
    SearchScalars *sc;
    uint16_t *Wcur, *Wimp, *Wbest;       // [B][N2] (N2 = N rounded up to even)
    uint32_t *ring;                      // [B][tl]
    uint32_t *tc;                        // [B][N*tcw]
    uint16_t *Xw; uint32_t *Xring; uint32_t *Xtc; int *Xwidx;   // exports [2][B]
    uint16_t *Fw; uint32_t *Fring; uint32_t *Ftc; int *Fwidx;   // working set [2][NF]
    SlotMeta *Fmeta;                     // [NF]
    Global *g;
    int *traj;                           // [B][iters][4]
    const uint32_t *decay;               // eq. 8 table
};

__host__ __device__ inline int n2(int n) { return (n + 1) & ~1; }

}  // namespace rcpsp
