// Internal interface of the matrix-core (tiled) search path and of the
// low-precision index copy it reads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace osann {

// A wave tile holds 16*G queries (G MFMA B operand groups).  G = 4 or 2
// for R <= 8 (wide tiles amortise each row load over more queries, narrow
// ones stream fewer cones that only some of their queries probe; the tuner
// picks), G = 2 for R = 16 (LDS and register budget of the top-R lists).
inline int tile_groups(int R) { return R <= 8 ? 4 : 2; }  // default
inline bool tile_groups_ok(int R, int G) { return G == 2 || (G == 4 && R <= 8); }
constexpr int kChunk = 512;  // cones a screen wave lists at a time (a multiple of 64)
constexpr int kWalkCache = 16;  // probed non-empty cones a query lane keeps from one walk decode (no bitmaps)
constexpr int kXcd = 8;      // chiplets (each with its own L2) the blocks of a launch are dealt to in turn
constexpr size_t kLdsPerBlock = 160 * 1024;  // LDS of one compute unit, all usable by one block

struct TiledArgs {
    // low-precision index
    const uint16_t* xl;
    int dk;
    const float* nrm;
    const uint32_t* prow;   // original row of each padded row (0xFFFFFFFF: padding)
    const uint32_t* poff;
    const uint32_t* offsets;
    const uint32_t* ne_id;
    const uint32_t* ne_cone;
    int64_t n_ne;
    // walk tables
    const uint8_t* lexsub;
    const uint8_t* maskord;
    const uint32_t* binom;
    int64_t n_sub;
    int D, L;
    // queries
    const uint16_t* ql;     // [Q][dk]
    int64_t Q;
    const uint32_t* qorder; // tile slot -> query
    const uint8_t* order;   // [Q][D]
    const uint8_t* sbit;    // [Q][D]
    const uint32_t* jstop;  // [Q]
    // probed cones: per-query bitmap over the non-empty cones (or null:
    // the kernel regenerates each query's walk)
    const uint64_t* qbits;  // [Q][nw]
    int64_t nw;
    // schedule
    int64_t T;              // wave tiles
    int S;                  // splits of the non-empty cones
    int64_t span;           // non-empty cones per split (multiple of 64)
    uint32_t* counter;      // [kXcd] work-queue heads, zero before the launch
    // output
    uint2* part;            // [Q][S][R] (FP32 bits of d~, original row), ascending
    uint32_t* cmin;         // [R][Q] by tile slot: smallest order-preserving d~ bits kept per class
                            // (padded position mod R), 0xFFFFFFFF before the launch
};

// Bound seeding before the screen: d~ of the rows of the first cones of each
// query's walk (its own cone first) on the vector units, raised by an
// accumulation-order error bound; the R-th smallest goes into every class.
struct SeedArgs {
    const uint16_t* xl;
    const float* nrm;
    const uint32_t* poff;
    int dk;
    const uint16_t* ql;      // [Q][dk]
    const uint32_t* qorder;  // tile slot -> query
    int64_t Q;
    uint32_t* cmin;          // [R][Q] by tile slot, as in the screen
    int rows;                // padded rows seeded per query (at most; a multiple of 64, <= 1024)
    // walk state and tables (the walk's first positions are the cones seeded)
    const uint8_t* order;    // [Q][D]
    const uint8_t* sbit;     // [Q][D]
    const uint32_t* jstop;   // [Q] walk positions taken (kWalkAll: every cone)
    const uint8_t* lexsub;
    const uint8_t* maskord;
    const uint32_t* binom;
    int64_t n_sub, n_cones;
    int D, L;
};

struct FinishArgs {
    const uint2* part;
    int S;
    int64_t Q;
    const void* planes;
    int dtype;
    int64_t N;
    int nch;
    const uint32_t* ppos;   // sorted position of each padded row
    const uint32_t* ipos;   // padded position of each original row
    const float* yf;
    int dpad;
    // Row-major low-precision copy ([padded position][dk] codes) where it
    // holds the table's values exactly: xl_codes 1 for FP16 codes of an FP16
    // table, 2 for BF16 codes of a uint8 table (BF16 holds 0..255 exactly),
    // 0 to read the chunk-major planes instead.
    const uint16_t* xl;
    int dk;
    int xl_codes;
    int64_t* out_idx;
    float* out_dist;
};

hipError_t launch_binom_table(uint32_t* tab, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_lowp_layout(const uint32_t* offsets, int64_t n_cones, uint32_t* psz_tmp, uint32_t* nef_tmp,
                              uint32_t* scan_tmp, uint32_t* poff, uint32_t* ne_id, uint32_t* ne_cone,
                              hipStream_t s);
hipError_t launch_lowp_rows(const void* planes, int dtype, int64_t N, int D, int nch, const uint32_t* sorted_cone,
                            const uint32_t* offsets, int64_t n_cones, const uint32_t* poff, const uint32_t* perm,
                            int dk, int to_f16, uint16_t* xl, uint32_t* ppos, uint32_t* prow, uint32_t* ipos,
                            float* nrm, int64_t np_total, hipStream_t s);
hipError_t launch_tiled_screen(const TiledArgs& a, int R, int G, int f16in, int blocks, hipStream_t s);
size_t tiled_screen_lds();                      // dynamic LDS bytes of one screen block
size_t tiled_screen_static_lds(int R, int G);          // static LDS bytes (upper bound) of one screen block
hipError_t launch_tiled_finish(const FinishArgs& f, int R, hipStream_t s);
// Cone-major screen (needs the probe bitmaps; a.S must equal a.nw: one list
// per (query, 64-cone word)); dk of 32, 64 or 128.
bool cone_screen_ok(int dk, int R);
size_t cone_screen_lds(int dk);
hipError_t launch_cone_screen(const TiledArgs& a, int R, int f16in, hipStream_t s);
hipError_t cone_screen_max_lds();
hipError_t launch_tiled_seed(const SeedArgs& a, int R, int f16in, hipStream_t s);
hipError_t tiled_screen_max_lds();
int tiled_screen_occupancy(int R, int G, int f16in, int ks, size_t lds);

}  // namespace osann
