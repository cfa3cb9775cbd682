// Internal layout shared by the device kernels and the host runtime of
// libgrainenv.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ge {

// ---------------------------------------------------------------- layout --
// Particle record, 16 bytes, stored as uint4:
//   x: travel s since the departure site (float bits)
//   y: grain << 3 | direction (0..5 = +x,-x,+y,-y,+z,-z of the crystal frame)
//   z: site x (int16, low half) | site y (int16, high half)
//   w: site z (int16, low half) | flags (high half)
// Flags: bits 0-1 state, bit 2 spawner this step, bit 3 kept (active,
// forwarded), bits 8-13 child-direction mask.
enum : uint32_t { ST_ACTIVE = 0, ST_STOPPED = 1, ST_RETIRED = 2 };
enum : uint32_t { FL_SPAWN = 4, FL_KEEP = 8 };

// Site states.
enum : uint32_t { SITE_DORMANT = 0, SITE_FIRED = 1, SITE_ENGULFED = 2 };

// Error bits of the sticky error word.
enum : uint32_t { ERR_CAPACITY = 1, ERR_NUMERIC = 2, ERR_CFL = 4 };
// Held context (not an error): every kernel of a step returns at once.
constexpr uint32_t HOLD = 0x100u;

// Grain table row: 24 floats.
//   [0..2] centre, [3] spare (site tables: nucleation undercooling),
//   [4..12] R row-major (crystal -> world), [13..21] lambda0 * R, [22..23] spare.
constexpr int GT_STRIDE = 24;

// Cells are grouped in bricks of 4^3; cell storage is brick-major
// (cell index = brick * 64 + local index), so a brick's 64 cells are
// contiguous and one wave64 lane serves one cell of a brick.
constexpr int BRICK = 4;
constexpr int BRICK_CELLS = 64;

// Streaming kernels run on a fixed grid; per-block lists (spawners, newly
// stopped particles) live in the block's own region of a particle-sized array.
constexpr int STREAM_GRID = 2048;

// Claim hash: 8^3 lattice sites per slot, three 512-bit masks per slot
// (claimed as target, reached, reached during the current step).
constexpr uint64_t CLAIM_EMPTY = ~0ull;
// Claim slot bricks per block along each axis: 2^CLAIM_BLOCK_BITS.
constexpr int CLAIM_BLOCK_BITS = 1;
constexpr uint64_t CLAIM_BLOCK_SLOTS = 1ull << (3 * CLAIM_BLOCK_BITS);
// Slots in the pool per slot brick asked for (blocks at the fringe of a
// grain are partly used).
constexpr uint64_t CLAIM_POOL_FACTOR = 2;
constexpr uint32_t NIL = 0xFFFFFFFFu;
constexpr uint32_t MIXED = 0xFFFFFFFEu;  // owner word: particles of several grains
constexpr uint32_t BOWN_CELLS = 0xFFFFFFFDu;  // brick owner word: see the cells' words
// Owner word of a particle with periodic axes: grain | image code << 26, the
// code holding the period index of the unwrapped position, two bits per
// axis (two's complement); without periodic axes the code is zero.
constexpr uint32_t OWNER_SHIFT = 26;
constexpr uint32_t GRAIN_MASK = (1u << OWNER_SHIFT) - 1u;

// Tunable kernels (index into Dev::sched).
enum : int { TK_ADVANCE = 0, TK_BRANCH, TK_CELLSCAN, TK_SCATTER, TK_CHILDREN, TK_DIRTY,
             TK_CONTAIN, TK_STOPLINK, TK_N };

// Field kinds.
enum : int32_t { F_UNIFORM = 0, F_LINEAR = 1, F_GRID = 2, F_ROSENTHAL = 3 };

struct Counters {
  uint32_t n_active;   // records in A (sorted region + nucleated tail)
  uint32_t n_out;      // records written by the scatter = sorted region of B
  uint32_t n_occ;      // occupied bricks this step
  uint32_t n_stopped;  // stopped store length
  uint32_t n_sorted;   // cell-sorted prefix of the stopped store
  uint32_t n_socc;     // bricks holding sorted stopped particles
  uint32_t n_grains;
  uint32_t claim_used; // occupied claim slots
  uint32_t err;        // sticky error bits
  uint32_t n_cand;     // nucleation candidates this step
  uint32_t max_step;   // float bits of max v dt (non-negative floats order as uints)
  uint32_t n_fired;    // sites fired this step
  uint32_t n_live;     // active particles (A also holds records stopped at the end of a step)
  uint32_t n_newstop;  // particles stopped by containment this step
  uint32_t n_dpart;    // particles of dirty bricks this step
  unsigned long long advanced, exited, spawners, children, contained, nucleated;
  unsigned long long pair_tests;  // candidate particles examined by containment
  unsigned long long dirty_tests; // active particles in dirty bricks
  // melting (walk-back): sites melted, particles removed, particles
  // re-activated, grains melted entirely
  unsigned long long melted, removed, reactivated, grains_melted;
  uint32_t n_melt_slots;  // claim slots with sites melted this step
  uint32_t n_resorted;    // live records counted by the stopped-store re-sort
  // step state, advanced on the device by k_finish (so that a captured
  // sequence of steps replays without host involvement)
  uint32_t par;        // 1: the active-store roles of A and B (and their tags) are swapped
  uint32_t spar;       // 1: the roles of S, PS and S2, PS2 are swapped
  uint32_t epoch;      // step stamp of occupied bricks (starts at 1)
  uint32_t dir_used;   // occupied entries of the claim-block directory
  double t;            // time
  unsigned long long step;  // steps taken
};

// Rosenthal moving point source over a linear background (field kind 3).
struct Rosenthal {
  double dT0, grad[3], rate, q, U, alpha, x_start, x_end, ys, zs, r_min, dT_min;
  double o[3], sp[3];
};

// Everything a kernel needs, passed by value.  It does not change from step
// to step: the roles of the double-buffered stores, the step stamp and the
// time live in the counters (device memory), so a recorded sequence of steps
// replays without host involvement.
struct Dev {
  // geometry
  float lo[3], hi[3];
  float inv_h;
  int32_t n[3];      // cells per axis
  int32_t nb[3];     // bricks per axis
  uint32_t n_bricks;
  int32_t stencil8;  // rc <= h/2: 2x2x2 cell stencil, else 3x3x3
  int32_t periodic;  // bit a: axis a periodic with period L[a] = hi[a] - lo[a]
  float L[3], invL[3];
  float lambda0, rc2, rc_half;
  float ka[2], kb[2];
  int32_t kin_poly;
  float theta;
  int32_t branching, box_exit;
  // field
  int32_t fkind;
  float fdT, fgrad[3];
  double fdT0, frate;  // LINEAR: dT0 + rate t, evaluated in FP64 on the device
  Rosenthal ros;
  int32_t fn[3];
  float fo[3], finv[3];
  float* fgrid;
  // mushy-zone deposition grid (gcnt null: off): reached sites per
  // node-centred cell
  uint32_t* gcnt;
  int32_t gn[3];
  float go[3], ginv[3];
  // melting (walk-back; melting = 0: off)
  int32_t melting;
  float* fcmin;        // [field cells] least node value of each cell of a node grid
  float* fcoarse;      // [coarse cells] least of fcmin over blocks of 4 x 4 x 4 cells
  uint32_t* mslots;    // [claim slots] slots with sites melted this step
  uint32_t* greach;    // [cap_grains] reached sites of each grain (kept while melting)
  int32_t* gsite;      // [cap_grains] nucleation site of each grain, -1: none
  uint32_t* gdead;     // [cap_grains] 1: the grain has melted entirely
  // grains
  float* gtab;     // [cap_grains][GT_STRIDE]
  int32_t* gbox;   // [cap_grains][6] lattice bbox of claims: lo xyz, hi xyz
  uint32_t cap_grains;
  // active store: A is this step's input, B its cell-sorted output, P the
  // positions (xyz, grain bits) of B
  uint4* A;
  uint4* B;
  float4* P;
  uint32_t cap_p;
  uint32_t* spawn;        // [cap_p], per-block regions
  uint32_t* spslot;       // [cap_p] claim slot of each spawner's reached site, at
                          //  the spawner's position in the per-block regions
  uint32_t* spawn_cnt;    // [STREAM_GRID]
  uint32_t* spawn_off;    // [STREAM_GRID + 1] exclusive prefix of spawn_cnt
  uint32_t* newstop;      // [cap_p], per-block regions
  uint32_t* newstop_cnt;  // [STREAM_GRID]
  // stopped store: records S, positions PS; [0, n_sorted) cell-sorted
  // (sstart, bsinfo), the rest in linked cell lists (shead, snext)
  uint4* S;
  float4* PS;
  uint4* S2;
  float4* PS2;
  uint32_t* snext;
  uint32_t cap_s;
  uint32_t* shead;     // [cells]
  uint32_t* sstart;    // [cells]
  uint2* bsinfo;       // [bricks] start, count of the sorted stopped particles
  // per-step cell list of the active particles
  uint32_t* ccnt;      // [cells] counts, back to zero after the scatter
  uint32_t* cstart;    // [cells]
  uint32_t* bcnt;      // [bricks] counts, reset by the scan
  uint2* binfo;        // [bricks] start, count of the step's active particles
  uint4* bmeta;        // [bricks] {step at which the brick was last occupied by active
                       //  particles, their least and greatest owner word that step,
                       //  owner word of the stopped particles}: what the neighbour
                       //  tests read, in one 16-byte load
  uint32_t* dlist;     // [bricks] dirty bricks, per-block regions of the occupied list
  uint32_t* dlist_cnt; // [STREAM_GRID]
  uint32_t* dpart;     // [cap_p] particles of dirty bricks (indices into B, P)
  unsigned long long* dmask;  // [bricks] per listed brick: cells whose particles need the test
  uint32_t* doff;      // [bricks] per listed brick: offset in the block's stretch of dpart
  uint2* bown;         // [bricks] {step, owner word of the active particles: the grain of a
                       //  single-grain brick, or BOWN_CELLS for a dirty brick}
  uint2* cown;         // [cells] {owner word of the active particles (dirty bricks, this
                       //  step), owner word of the stopped particles}
  uint32_t* smask;     // [cells] slabs (eighths of the cell per axis, 8 bits per axis)
                       //  that hold stopped particles
  uint32_t* occ;       // [bricks] occupied-brick list
  uint64_t* scan_tmp;  // block partial sums of the brick scan
  // claims: the slot bricks of a grain in cubic blocks of CLAIM_BLOCK_SLOTS
  // consecutive slots; a hash directory of the blocks
  unsigned long long* ckeys;   // [slots] key of each taken slot, else CLAIM_EMPTY
  unsigned long long* cbits;   // [slots][3][8]: claimed, reached, now
  unsigned long long* clist;   // [slots] keys of the occupied slots in insertion order
                               //  (claim_used of them)
  unsigned long long* dirkeys; // [blocks] block key of each directory entry
  uint64_t cmask;              // slots - 1
  uint64_t dirmask;            // blocks - 1 (slots = CLAIM_BLOCK_SLOTS blocks)
  uint32_t claim_limit;        // slots that can be taken
  uint32_t dir_limit;          // occupancy limit of the directory
  // sites
  float* stab;         // [cap_sites][GT_STRIDE], [3] = nucleation undercooling
  uint32_t* sstate;    // [cap_sites]
  uint32_t* cand;      // [cap_sites]
  uint32_t* sgrain;    // [cap_sites] with melting: grain whose claims covered the site at its
                       //  last test (a hint; NIL or stale values only cost the full search)
  uint32_t n_sites;
  // counters
  Counters* cnt;
  // adjoint recording (all null when off): tags travel with the records of
  // A and B (tag = index into the tracked set, NIL for untracked particles)
  uint32_t* tagA;
  uint32_t* tagB;
  uint4* adj_rec;      // [tracked] records at the start of the recorded run
  int32_t* adj_nact;   // [tracked] steps in which the particle advanced
  float* adj_sfin;     // [tracked] travel at the end of the run (or at its stop)
  float* adj_ck;       // [checkpoints][adj_ncap] travel at steps c * adj_K
  float* adj_linc;      // [steps] LINEAR field constant of each recorded step
  uint32_t adj_ncap;
  int32_t adj_K;        // checkpoint interval
  unsigned long long adj_step0;  // step count at the start of the recorded run
  int32_t resort_every;  // steps between re-sorts of the stopped store
  // launch schedule: blocks per launch of each tunable kernel.  The spawn
  // lists have sched[TK_ADVANCE] regions, the stop lists sched[TK_CONTAIN].
  uint32_t sched[9];
};

// Every pointer member of Dev (a batched launch stores them as offsets from
// the batch workspace and rebuilds them on the device).
#define GE_DEV_POINTERS(X)                                                                   \
  X(fgrid) X(gcnt) X(fcmin) X(fcoarse) X(mslots) X(greach) X(gsite) X(gdead) X(gtab) X(gbox) X(A) X(B) X(P) X(spawn) X(spslot) X(spawn_cnt) X(spawn_off) X(newstop)      \
  X(newstop_cnt) X(S) X(PS) X(S2) X(PS2) X(snext) X(shead) X(sstart) X(bsinfo)      \
  X(ccnt) X(cstart) X(bcnt) X(binfo) X(bmeta) X(dlist) X(dlist_cnt) X(dpart) X(dmask)       \
  X(doff) X(bown)                                                                             \
  X(cown) X(smask) X(occ) X(scan_tmp) X(ckeys) X(cbits) X(clist) X(dirkeys) X(stab) X(sstate) X(cand) X(sgrain) X(cnt) X(tagA)      \
  X(tagB) X(adj_rec) X(adj_nact) X(adj_sfin) X(adj_ck) X(adj_linc)
constexpr uintptr_t NULL_OFFSET = ~(uintptr_t)0;

// Batched launches: for each launch site, the blocks of every context
// (map: per block, context | virtual block << 12; gsz: per context, its
// blocks; total: blocks of the launch).
enum : int {
  BS_RESAMPLE = 0, BS_ADVANCE, BS_ONE, BS_BRANCH, BS_TILES, BS_CELLSCAN,
  BS_SCATTER, BS_CHILDREN, BS_DIRTY, BS_CONTAIN, BS_STOPLINK, BS_NUCTEST, BS_NUCFIRE,
  BS_RESORT, BS_N
};
constexpr uint32_t BATCH_MAX = 4096;  // contexts per batch (12 bits of a map entry)
constexpr uint64_t SCAN_TILE_HOST = 2048;  // bricks per tile of the brick scan
struct BatchSite {
  const uint32_t* map;
  const uint32_t* gsz;
  uint32_t total;
};
struct BatchLaunch {
  const Dev* tab;  // per context: Dev with pointers stored as offsets from base
  char* base;
  BatchSite site[BS_N];
  int32_t any_periodic;  // some context has periodic axes
};

// -------------------------------------------------- host-side launchers --
hipError_t resident_grids(Dev& d);  // default schedule for the current device
void launch_advance(const Dev& d, float dt, hipStream_t s);
void launch_branch(const Dev& d, hipStream_t s);
void launch_scan(const Dev& d, hipStream_t s);
void launch_scatter(const Dev& d, hipStream_t s);
void launch_scatter_children(const Dev& d, hipStream_t s);
void launch_dirty(const Dev& d, hipStream_t s);
void launch_contain(const Dev& d, hipStream_t s);
void launch_stoplink(const Dev& d, hipStream_t s);
void launch_nucleate(const Dev& d, hipStream_t s);
void launch_finish(const Dev& d, double dt, hipStream_t s);
void launch_reset_stats(const Dev& d, hipStream_t s);
void launch_stopped_rebuild(const Dev& d, hipStream_t s);  // S -> S2 (caller swaps)
void launch_resample(const Dev& d, hipStream_t s);
// Melting by walk-back, run at the start of a step when enabled: least node
// value per field cell, melted sites, walk-back particles, melted grains,
// stopped particles of melted sites.  launch_count_reached recounts the
// reached sites of every grain (grains with none are marked melted).
void launch_melt(const Dev& d, hipStream_t s);
void launch_count_reached(const Dev& d, hipStream_t s);
// Mushy-zone deposition: counts of every reached site (counts cleared
// first), and g^m = min(1, count lambda0^3 / cell volume) per cell.
void launch_deposit_all(const Dev& d, hipStream_t s);
void launch_mushy_fraction(const uint32_t* cnt, uint64_t n, double site_over_cell, float* out,
                           hipStream_t s);
// Node undercooling liq_T + liq_m w - T of a SOLUTE field (FP64 in, FP32 out).
void launch_solute_nodes(const double* T, const double* w, double liq_T, double liq_m,
                         uint64_t n, float* out, hipStream_t s);
void launch_init_workspace(const Dev& d, hipStream_t s);
// exit_rule: particles outside the box (box exit on) start stopped (new
// envelopes); off for loaded states, whose particles keep their states.
void launch_classify_new(const Dev& d, uint32_t first, uint32_t count, bool exit_rule,
                         hipStream_t s);
void launch_claim_ball(const Dev& d, uint32_t grain, int32_t r, hipStream_t s);
void launch_claim_list(const Dev& d, const int32_t* grain, const int32_t* site,
                       const uint8_t* flags, uint32_t n, hipStream_t s);
// Claim bricks of a saved state (144-byte records, see k_export_slots):
// into the claim hash, and out of it (every slot with a claimed or reached
// site; counter: device uint32, zeroed by the caller).
void launch_claim_slots(const Dev& d, const void* slots, uint32_t n, hipStream_t s);
void launch_export_slots(const Dev& d, uint32_t* counter, void* out, uint32_t cap_out,
                         hipStream_t s);
void launch_export_particles(const Dev& d, uint32_t* counter, void* out, uint32_t cap_out,
                             const float* window /* lo xyz, hi xyz or null */, hipStream_t s);
// Allocation-free particle export: records staged in a static device array
// of NOALLOC_RECORDS records (48 bytes each) after a 256-byte header whose
// first word counts the records the window holds.  noalloc_scratch gives the
// array's address on the current device (looked up once per device).
constexpr size_t NOALLOC_RECORDS = 1u << 20;
constexpr size_t NOALLOC_RECORDS_OFFSET = 256;
hipError_t noalloc_scratch(void** out);
void launch_export_particles_staged(const Dev& d, void* scratch_ptr, const float* window,
                                    hipStream_t s);
void launch_export_claims(const Dev& d, uint32_t* counter, void* out, uint32_t cap_out,
                          const float* window, hipStream_t s);
void launch_grain_map(const Dev& d, const int32_t n[3], const float origin[3],
                      const float spacing[3], uint32_t* out, hipStream_t s);
void launch_batch_reset_stats(const BatchLaunch& L, hipStream_t s);
void launch_batch_step(const BatchLaunch& L, double dt, hipStream_t s);
void launch_digest(const Dev& d, unsigned long long* out /*[3], zeroed*/, hipStream_t s);
void launch_adj_init(const Dev& d, uint32_t n, int32_t n_steps, hipStream_t s);
void launch_adj_final(const Dev& d, hipStream_t s);
void launch_adj_positions(const Dev& d, uint32_t n, float* xN, hipStream_t s);
// Reverse sweep and reduction; grad_out: 3 doubles (device), mismatch: 1 uint32 (device).
constexpr uint32_t ADJ_BLOCKS = 4096;
void launch_adj_backward(const Dev& d, uint32_t n, int32_t n_steps, int32_t K, const float* linc,
                         float dt, const float* dLdx, float* seg, double* part, double* grad_out,
                         uint32_t* mismatch, hipStream_t s);

}  // namespace ge
