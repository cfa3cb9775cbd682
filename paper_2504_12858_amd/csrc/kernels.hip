// Device kernels of the grain-envelope step for gfx950 (wave64).
//
// One step (Sec. 2.1.2 growth and branching, Sec. 2.3 cell partitioning and
// collision detection, Sec. 2.1.1 nucleation) runs as:
//   k_resample   moving point-source field sampled onto the node grid
//   k_melt_*, k_walkback   melting by walk-back, when enabled (Sec. 2.1.3)
//   k_advance    undercooling at each active particle, kinetic law Eq. (2),
//                advance along R e_d, box exit, spawner list, per-cell and
//                per-brick counts of the particles that stay active; marks
//                each spawner's reached site as reached this step
//   k_branch     outer directions of each spawner against the grain's claims;
//                same-step competitors for one target resolved by lowest
//                direction; counts of the children
//   k_scan_*     exclusive scan of brick counts -> brick starts, occupied list
//   k_cellscan   one wave per occupied brick, one lane per cell: cell starts
//   k_scatter    records and positions -> cell-sorted arrays (ranks from
//                wave-aggregated decrements of the cell counts)
//   k_dirty      bricks whose particles can meet another grain; their cells'
//                owner words and the list of particles to test
//   k_contain    cell-stencil test against other grains' particles
//   k_stoplink   moves newly stopped particles to the stopped store
//   k_nuc_test / k_nuc_fire   nucleation of liquid sites past threshold
//   k_finish     counters for the next step
// Every few steps the stopped store is re-sorted by cell with the same
// counting machinery (k_srb_*), so that containment reads it as contiguous
// cell ranges; particles stopped since the last re-sort sit in short linked
// cell lists.
//
// Particle positions are recomputed from the record (grain, departure site,
// direction, travel) with one function everywhere, so binning, containment
// and export see identical FP32 values.  With periodic axes (Sec. 3.4) the
// binned and stored position is that one wrapped into the box, its period
// index kept in the owner word.
#include "internal.h"

#include <math.h>

#include <algorithm>
#include <initializer_list>
#include <mutex>

namespace ge {

constexpr int TPB = 256;

enum : int { CB_CLAIMED = 0, CB_REACHED = 8, CB_NOW = 16 };
enum : uint32_t { M_CLAIMED = 1, M_REACHED = 2, M_NOW = 4 };

// ------------------------------------------------------------- records ----
__device__ __forceinline__ uint32_t rec_grain(uint4 r) { return r.y >> 3; }
__device__ __forceinline__ int rec_dir(uint4 r) { return (int)(r.y & 7u); }
__device__ __forceinline__ float rec_s(uint4 r) { return __uint_as_float(r.x); }
__device__ __forceinline__ int rec_sx(uint4 r) { return (int)(int16_t)(r.z & 0xFFFFu); }
__device__ __forceinline__ int rec_sy(uint4 r) { return (int)(int16_t)(r.z >> 16); }
__device__ __forceinline__ int rec_sz(uint4 r) { return (int)(int16_t)(r.w & 0xFFFFu); }
__device__ __forceinline__ uint32_t rec_fl(uint4 r) { return r.w >> 16; }
__device__ __forceinline__ uint4 make_rec(float s, uint32_t g, int d, int sx, int sy, int sz,
                                          uint32_t fl) {
  return make_uint4(__float_as_uint(s), (g << 3) | (uint32_t)d,
                    ((uint32_t)(uint16_t)sx) | ((uint32_t)(uint16_t)sy << 16),
                    ((uint32_t)(uint16_t)sz) | (fl << 16));
}
__device__ __forceinline__ uint4 with_fl(uint4 r, uint32_t fl) {
  r.w = (r.w & 0xFFFFu) | (fl << 16);
  return r;
}

struct P3 {
  float x, y, z;
};

// World position of departure site (sx, sy, sz) plus travel s along d:
// x = c + (lambda0 R) site + s R e_d, with explicit FMAs (no contraction
// freedom is left to the compiler, so every kernel gets the same bits).
__device__ __forceinline__ P3 lattice_pos(const float* __restrict__ G, int sx, int sy, int sz,
                                          int d, float s) {
  const float fx = (float)sx, fy = (float)sy, fz = (float)sz;
  const int a = d >> 1;
  const float ss = (d & 1) ? -s : s;
  P3 p;
  p.x = fmaf(ss, G[4 + a], fmaf(G[13], fx, fmaf(G[14], fy, fmaf(G[15], fz, G[0]))));
  p.y = fmaf(ss, G[7 + a], fmaf(G[16], fx, fmaf(G[17], fy, fmaf(G[18], fz, G[1]))));
  p.z = fmaf(ss, G[10 + a], fmaf(G[19], fx, fmaf(G[20], fy, fmaf(G[21], fz, G[2]))));
  return p;
}


// A grain's table row held in registers (six 16-byte loads), for kernels
// that place several positions of one grain around atomics: a wave's memory
// operations retire in order, so a load issued after an atomic waits for
// the atomic's round trip.
struct GRow {
  float v[24];
};
__device__ __forceinline__ GRow load_grow(const float* G) {
  GRow g;
  const float4* q = reinterpret_cast<const float4*>(G);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float4 t = q[k];
    g.v[4 * k] = t.x;
    g.v[4 * k + 1] = t.y;
    g.v[4 * k + 2] = t.z;
    g.v[4 * k + 3] = t.w;
  }
  return g;
}
// Site S of a grain as lattice_pos builds it: the site's position
// c + lambda0 R S and the columns of R, from which the positions at travel s
// along each direction follow with the same FMAs (hence the same bits).
struct SiteFrame {
  P3 o;
  float e[9];  // R e_a for a = 0, 1, 2: x components, then y, then z
};
__device__ __forceinline__ SiteFrame site_frame(const GRow& G, int sx, int sy, int sz) {
  const float fx = (float)sx, fy = (float)sy, fz = (float)sz;
  SiteFrame f;
  f.o.x = fmaf(G.v[13], fx, fmaf(G.v[14], fy, fmaf(G.v[15], fz, G.v[0])));
  f.o.y = fmaf(G.v[16], fx, fmaf(G.v[17], fy, fmaf(G.v[18], fz, G.v[1])));
  f.o.z = fmaf(G.v[19], fx, fmaf(G.v[20], fy, fmaf(G.v[21], fz, G.v[2])));
#pragma unroll
  for (int k = 0; k < 9; ++k) f.e[k] = G.v[4 + k];
  return f;
}
// lattice_pos(G, S, d, s) from the frame of S.
__device__ __forceinline__ P3 frame_pos(const SiteFrame& f, int d, float s) {
  const int a = d >> 1;
  const float ss = (d & 1) ? -s : s;
  return {fmaf(ss, f.e[a], f.o.x), fmaf(ss, f.e[3 + a], f.o.y), fmaf(ss, f.e[6 + a], f.o.z)};
}

__device__ __forceinline__ P3 rec_pos(const Dev& D, uint4 r) {
  return lattice_pos(D.gtab + (size_t)rec_grain(r) * GT_STRIDE, rec_sx(r), rec_sy(r), rec_sz(r),
                     rec_dir(r), rec_s(r));
}

// ---------------------------------------------------------------- cells ---
// Single-rounded FP32 binning: floor((x - lo) * inv_h), clamped to [0, n-1].
__device__ __forceinline__ int cell_axis(float x, float lo, float inv_h, int n) {
  float u = (x - lo) * inv_h;
  float f = floorf(u);
  f = fmaxf(f, 0.0f);
  f = fminf(f, (float)(n - 1));
  return (int)f;
}

struct C3 {
  int x, y, z;
};

__device__ __forceinline__ C3 cell_of(const Dev& D, P3 p) {
  C3 c;
  c.x = cell_axis(p.x, D.lo[0], D.inv_h, D.n[0]);
  c.y = cell_axis(p.y, D.lo[1], D.inv_h, D.n[1]);
  c.z = cell_axis(p.z, D.lo[2], D.inv_h, D.n[2]);
  return c;
}

// ------------------------------------------------ periodic boundaries ---
// On a periodic axis (period L = hi - lo) positions stay lattice-anchored
// and unwrapped; the cell, the field and the contact tests take the position
// wrapped into [lo, hi) together with its period index k (x = wrapped + k L).
// A position already inside the box is returned unchanged, so wrapping is
// idempotent.
struct Placed {
  P3 p;
  uint32_t code;  // period index per periodic axis, two bits each (two's complement)
};
__device__ __forceinline__ float wrap_axis(float x, float lo, float hi, float L, float invL,
                                          int& k) {
  k = 0;
  if (x >= lo && x < hi) return x;
  float f = floorf((x - lo) * invL);
  float y = fmaf(-f, L, x);
  if (!(y >= lo)) {
    y = lo;
  } else if (!(y < hi)) {
    y = lo;
    f += 1.0f;
  }
  k = (int)f;
  return y;
}
__device__ __forceinline__ Placed place(const Dev& D, P3 x) {
  Placed o = {x, 0u};
  if (!D.periodic) return o;
  int k;
  if (D.periodic & 1) {
    o.p.x = wrap_axis(x.x, D.lo[0], D.hi[0], D.L[0], D.invL[0], k);
    o.code |= (uint32_t)k & 3u;
  }
  if (D.periodic & 2) {
    o.p.y = wrap_axis(x.y, D.lo[1], D.hi[1], D.L[1], D.invL[1], k);
    o.code |= ((uint32_t)k & 3u) << 2;
  }
  if (D.periodic & 4) {
    o.p.z = wrap_axis(x.z, D.lo[2], D.hi[2], D.L[2], D.invL[2], k);
    o.code |= ((uint32_t)k & 3u) << 4;
  }
  return o;
}
__device__ __forceinline__ uint32_t owner_id(uint32_t g, uint32_t code) {
  return g | (code << OWNER_SHIFT);
}
// Period index of axis a in an owner word.
__device__ __forceinline__ int owner_image(uint32_t own, int a) {
  const int v = (int)((own >> (OWNER_SHIFT + 2 * a)) & 3u);
  return v >= 2 ? v - 4 : v;
}
// Inside the box along every axis that is not periodic.
template <int PM = 2>
__device__ __forceinline__ bool in_box(const Dev& D, P3 x) {
  const int per = PM == 0 ? 0 : D.periodic;
  return ((per & 1) || (x.x >= D.lo[0] && x.x < D.hi[0])) &&
         ((per & 2) || (x.y >= D.lo[1] && x.y < D.hi[1])) &&
         ((per & 4) || (x.z >= D.lo[2] && x.z < D.hi[2]));
}
// Wrapped position and owner word of a particle of grain g at x.
__device__ __forceinline__ float4 placed4(const Dev& D, P3 x, uint32_t g) {
  const Placed pl = place(D, x);
  return make_float4(pl.p.x, pl.p.y, pl.p.z, __uint_as_float(owner_id(g, pl.code)));
}
// Cell index along a periodic axis, wrapped (stencil cells past a face).
__device__ __forceinline__ int wrap_cell(int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); }

__device__ __forceinline__ uint32_t brick_index(const Dev& D, int cx, int cy, int cz) {
  return ((uint32_t)(cz >> 2) * (uint32_t)D.nb[1] + (uint32_t)(cy >> 2)) * (uint32_t)D.nb[0] +
         (uint32_t)(cx >> 2);
}

__device__ __forceinline__ uint32_t local_index(int cx, int cy, int cz) {
  return (uint32_t)((cx & 3) | ((cy & 3) << 2) | ((cz & 3) << 4));
}

// Brick-major cell index: the 64 cells of a brick are contiguous.
__device__ __forceinline__ uint32_t cell_index(const Dev& D, int cx, int cy, int cz) {
  return brick_index(D, cx, cy, cz) * (uint32_t)BRICK_CELLS + local_index(cx, cy, cz);
}

__device__ __forceinline__ float dist2(P3 a, P3 b) {
  float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ P3 p3_of(float4 q) { return P3{q.x, q.y, q.z}; }
__device__ __forceinline__ uint32_t grain_of(float4 q) { return __float_as_uint(q.w); }
__device__ __forceinline__ float4 pos4(P3 p, uint32_t g) {
  return make_float4(p.x, p.y, p.z, __uint_as_float(g));
}

// Cells that can hold a particle within rc of p along one axis: with
// rc <= h/2 the cell of p and its neighbour on the side of the nearer face,
// otherwise the cell and both neighbours; clamped to the grid.
__device__ __forceinline__ void stencil_axis(const Dev& D, float x, int a, int& c0, int& c1) {
  const int n = D.n[a];
  const float u = (x - D.lo[a]) * D.inv_h;
  const float fl = floorf(u);
  const int c = (int)fminf(fmaxf(fl, 0.0f), (float)(n - 1));
  if (D.stencil8) {
    const bool up = (u - fl) >= 0.5f;
    c0 = up ? c : c - 1;
    c1 = up ? c + 1 : c;
  } else {
    c0 = c - 1;
    c1 = c + 1;
  }
  // On a periodic axis the stencil runs past the face (its cells wrap).
  if ((D.periodic >> a) & 1) return;
  c0 = max(c0, 0);
  c1 = min(c1, n - 1);
}

// ---------------------------------------------------------------- field ---
__device__ __forceinline__ float trilinear(const Dev& D, P3 p) {
  float u[3] = {(p.x - D.fo[0]) * D.finv[0], (p.y - D.fo[1]) * D.finv[1],
                (p.z - D.fo[2]) * D.finv[2]};
  int i0[3];
  float f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float fl = floorf(u[a]);
    fl = fmaxf(fl, 0.0f);
    fl = fminf(fl, (float)(D.fn[a] - 2));
    i0[a] = (int)fl;
    float w = u[a] - fl;
    w = fminf(fmaxf(w, 0.0f), 1.0f);
    f[a] = w;
  }
  const size_t sy = (size_t)D.fn[0], sz = (size_t)D.fn[0] * (size_t)D.fn[1];
  const size_t b = (size_t)i0[2] * sz + (size_t)i0[1] * sy + (size_t)i0[0];
  const float* __restrict__ g = D.fgrid;
  float c000 = g[b], c100 = g[b + 1], c010 = g[b + sy], c110 = g[b + sy + 1];
  float c001 = g[b + sz], c101 = g[b + sz + 1], c011 = g[b + sz + sy], c111 = g[b + sz + sy + 1];
  float c00 = fmaf(f[0], c100 - c000, c000);
  float c10 = fmaf(f[0], c110 - c010, c010);
  float c01 = fmaf(f[0], c101 - c001, c001);
  float c11 = fmaf(f[0], c111 - c011, c011);
  float c0 = fmaf(f[1], c10 - c00, c00);
  float c1 = fmaf(f[1], c11 - c01, c01);
  return fmaf(f[2], c1 - c0, c0);
}

// Undercooling at p (without theta).  lin_c = dT0 + rate t for LINEAR.
// PM (periodic mode): 0 for a context without periodic axes, 1 with them,
// 2 as the context has them; kernels on the hot path are instantiated for 0
// and 1 so that the plain case carries no periodic code.
template <int PM = 2>
__device__ __forceinline__ float field_at(const Dev& D, P3 p, float lin_c) {
  if (D.fkind == F_UNIFORM) return D.fdT;
  if constexpr (PM != 0) p = place(D, p).p;
  if (D.fkind == F_LINEAR)
    return ((lin_c + D.fgrad[0] * p.x) + D.fgrad[1] * p.y) + D.fgrad[2] * p.z;
  return trilinear(D, p);
}

// Kinetic law, Eq. (2): v = a0 dT^b0 + a1 dT^b1 for dT > 0, else 0.
__device__ __forceinline__ float velocity(const Dev& D, float dT) {
  if (!(dT > 0.0f)) return 0.0f;
  if (D.kin_poly) return dT * dT * fmaf(D.ka[1], dT, D.ka[0]);
  float l = log2f(dT);
  return D.ka[0] * exp2f(D.kb[0] * l) + D.ka[1] * exp2f(D.kb[1] * l);
}

// --------------------------------------------------------------- claims ---
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ uint64_t claim_key(uint32_t g, int sx, int sy, int sz) {
  const uint64_t bx = (uint64_t)((sx >> 3) + 2048) & 0xFFFull;
  const uint64_t by = (uint64_t)((sy >> 3) + 2048) & 0xFFFull;
  const uint64_t bz = (uint64_t)((sz >> 3) + 2048) & 0xFFFull;
  return ((uint64_t)g << 36) | (bx << 24) | (by << 12) | bz;
}

__device__ __forceinline__ uint32_t site_bit(int sx, int sy, int sz) {
  return (uint32_t)((sx & 7) | ((sy & 7) << 3) | ((sz & 7) << 6));
}

constexpr uint32_t MAX_PROBE = 4096;

__device__ __forceinline__ unsigned long long load_relaxed(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A plain load, which the L2 of the reading chiplet may serve.  Each kernel
// starts with the caches invalidated, so it returns the word as it was at the
// kernel's start or a later value; the readers below take it for words whose
// updates during the kernel do not change their outcome.
__device__ __forceinline__ unsigned long long load_cached(const unsigned long long* p) {
  return *p;
}

// Claim slots.  The slot bricks of a grain are grouped into cubic blocks
// (2^CLAIM_BLOCK_BITS slot bricks per axis) of consecutive slots, so that the
// claim words of nearby sites lie close together in memory (few pages, hence
// few address translations, per wave).  A hash directory (open addressing,
// linear probing) places the blocks: slot = CLAIM_BLOCK_SLOTS * (directory
// entry of the block) + position in the block.
constexpr uint64_t CB_LOW = (1ull << CLAIM_BLOCK_BITS) - 1ull;
__device__ __forceinline__ uint64_t claim_block_key(uint64_t key) {
  return key & ~((CB_LOW << 24) | (CB_LOW << 12) | CB_LOW);
}
__device__ __forceinline__ uint64_t claim_fine(uint64_t key) {
  return ((key >> 24) & CB_LOW) | (((key >> 12) & CB_LOW) << CLAIM_BLOCK_BITS) |
         ((key & CB_LOW) << (2 * CLAIM_BLOCK_BITS));
}

// Directory entry of a block, or -1; through the cache or not.
template <bool CACHED>
__device__ __forceinline__ int64_t block_find(const Dev& D, uint64_t bkey) {
  const uint64_t h = mix64(bkey) & D.dirmask;
  for (uint32_t p = 0; p < MAX_PROBE; ++p) {
    const uint64_t idx = (h + p) & D.dirmask;
    const uint64_t k = CACHED ? load_cached(&D.dirkeys[idx]) : load_relaxed(&D.dirkeys[idx]);
    if (k == bkey) return (int64_t)idx;
    if (k == CLAIM_EMPTY) return -1;
  }
  return -1;
}

// Read-only probe: slot or -1.
__device__ int64_t claim_find(const Dev& D, uint64_t key) {
  const int64_t b = block_find<false>(D, claim_block_key(key));
  if (b < 0) return -1;
  const uint64_t slot = (uint64_t)b * CLAIM_BLOCK_SLOTS + claim_fine(key);
  return load_relaxed(&D.ckeys[slot]) == key ? (int64_t)slot : -1;
}

// Find or insert: slot or -1 (capacity error raised).  Keys never change
// once inserted, so the probes read through the cache: a stale empty entry
// only sends the insertion to the compare-and-swap, whose result decides.
// A slot can only ever hold its own key.
__device__ int64_t claim_get(const Dev& D, uint64_t key) {
  const uint64_t bkey = claim_block_key(key);
  const uint64_t h = mix64(bkey) & D.dirmask;
  int64_t blk = -1;
  for (uint32_t p = 0; p < MAX_PROBE && blk < 0; ++p) {
    const uint64_t idx = (h + p) & D.dirmask;
    const unsigned long long k = load_cached(&D.dirkeys[idx]);
    if (k == bkey) {
      blk = (int64_t)idx;
    } else if (k == CLAIM_EMPTY) {
      if (__hip_atomic_load(&D.cnt->dir_used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
          D.dir_limit) {
        atomicOr(&D.cnt->err, ERR_CAPACITY);
        return -1;
      }
      const unsigned long long prev =
          atomicCAS(&D.dirkeys[idx], CLAIM_EMPTY, (unsigned long long)bkey);
      if (prev == CLAIM_EMPTY) atomicAdd(&D.cnt->dir_used, 1u);
      if (prev == CLAIM_EMPTY || prev == bkey) blk = (int64_t)idx;
    }
  }
  if (blk < 0) {
    atomicOr(&D.cnt->err, ERR_CAPACITY);
    return -1;
  }
  const uint64_t slot = (uint64_t)blk * CLAIM_BLOCK_SLOTS + claim_fine(key);
  if (load_cached(&D.ckeys[slot]) != key &&
      atomicCAS(&D.ckeys[slot], CLAIM_EMPTY, (unsigned long long)key) == CLAIM_EMPTY) {
    // One count per slot taken, so the list index stays below the slots.
    D.clist[atomicAdd(&D.cnt->claim_used, 1u)] = key;
  }
  return (int64_t)slot;
}

__device__ __forceinline__ void claim_or(const Dev& D, uint32_t g, int sx, int sy, int sz,
                                         uint32_t which) {
  int64_t slot = claim_get(D, claim_key(g, sx, sy, sz));
  if (slot < 0) return;
  const uint32_t b = site_bit(sx, sy, sz);
  const unsigned long long m = 1ull << (b & 63);
  unsigned long long* w = D.cbits + (size_t)slot * 24 + (b >> 6);
  if (which & M_CLAIMED) atomicOr(w + CB_CLAIMED, m);
  if (which & M_REACHED) atomicOr(w + CB_REACHED, m);
  if (which & M_NOW) atomicOr(w + CB_NOW, m);
}

// True if the site is in any of the masks selected by `which`.
__device__ __forceinline__ bool claim_test(const Dev& D, uint32_t g, int sx, int sy, int sz,
                                           uint32_t which) {
  int64_t slot = claim_find(D, claim_key(g, sx, sy, sz));
  if (slot < 0) return false;
  const uint32_t b = site_bit(sx, sy, sz);
  const unsigned long long m = 1ull << (b & 63);
  const unsigned long long* w = D.cbits + (size_t)slot * 24 + (b >> 6);
  unsigned long long v = 0;
  if (which & M_CLAIMED) v |= load_relaxed(w + CB_CLAIMED);
  if (which & M_REACHED) v |= load_relaxed(w + CB_REACHED);
  if (which & M_NOW) v |= load_relaxed(w + CB_NOW);
  return (v & m) != 0;
}

// Grows grain g's lattice bounding box to include the site.  Plain reads
// first: the box changes only at its extremes, and skipping the atomics in
// the common case keeps thousands of spawners of one grain off six hot words.
// Grows grain g's lattice bounding box to hold the box [lo, hi] of sites.
__device__ __forceinline__ void bbox_add_box(const Dev& D, uint32_t g, const int lo[3],
                                             const int hi[3]) {
  int32_t* b = D.gbox + (size_t)g * 6;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (lo[a] < __hip_atomic_load(b + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMin(b + a, lo[a]);
    if (hi[a] > __hip_atomic_load(b + 3 + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(b + 3 + a, hi[a]);
  }
}
__device__ __forceinline__ void bbox_add(const Dev& D, uint32_t g, int sx, int sy, int sz) {
  const int s[3] = {sx, sy, sz};
  bbox_add_box(D, g, s, s);
}

// Mushy-zone deposition: a lattice site that a grain has reached adds its
// crystal-frame cube (lambda0^3) to the deposition cell holding its centre;
// cell (i, j, k) is the node-centred box of node (i, j, k) of the deposition
// grid.  FP32, single-rounded: i = floor((x - origin) * inv_spacing + 1/2).
// Deposition cell of a site, or NIL outside the grid.
__device__ __forceinline__ uint32_t deposit_cell(const Dev& D, const float* __restrict__ G, int sx,
                                                 int sy, int sz) {
  const P3 x = place(D, lattice_pos(G, sx, sy, sz, 0, 0.0f)).p;
  const float xs[3] = {x.x, x.y, x.z};
  uint32_t idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float f = floorf((xs[a] - D.go[a]) * D.ginv[a] + 0.5f);
    if (!(f >= 0.0f && f < (float)D.gn[a])) return NIL;
    idx[a] = (uint32_t)f;
  }
  return (idx[2] * (uint32_t)D.gn[1] + idx[1]) * (uint32_t)D.gn[0] + idx[0];
}
__device__ __forceinline__ void deposit_site(const Dev& D, const float* __restrict__ G, int sx,
                                             int sy, int sz) {
  const uint32_t c = deposit_cell(D, G, sx, sy, sz);
  if (c != NIL) atomicAdd(&D.gcnt[c], 1u);
}

// Whether the undercooling field minus theta can be negative somewhere in
// the box [lo, hi]: false only when a lower bound of the field over the box
// (with a margin for the rounding of the evaluation) is at least theta.  For
// a node grid the bound is the least node value of the cells the box meets
// (a trilinear interpolant lies between the least and the greatest node of
// its cell), taken first over blocks of 4 x 4 x 4 cells from a table small
// enough to stay in cache, then cell by cell.  Clamped coordinates and boxes
// reaching beyond the grid are handled as the interpolation handles them.
__device__ __forceinline__ float bound_margin(float m) { return m - 1e-5f * fabsf(m) - 1e-6f; }
template <int PM = 2>
__device__ bool may_melt(const Dev& D, P3 lo, P3 hi, float lin_c) {
  if (D.fkind == F_UNIFORM) return D.fdT - D.theta < 0.0f;
  float l[3] = {lo.x, lo.y, lo.z}, h[3] = {hi.x, hi.y, hi.z};
  // On a periodic axis the box is moved into the period of its low end
  // (with a margin for the rounding of the move); a box that then reaches
  // past the face, or spans a period, takes the whole axis.
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (PM == 0 || !((D.periodic >> a) & 1)) continue;
    int k;
    const float ln = wrap_axis(l[a], D.lo[a], D.hi[a], D.L[a], D.invL[a], k);
    const float m = 1e-6f * D.L[a];
    const float hn = fmaf(-(float)k, D.L[a], h[a]) + m;
    if (!(h[a] - l[a] < D.L[a]) || !(hn < D.hi[a])) {
      l[a] = D.lo[a];
      h[a] = D.hi[a];
    } else {
      l[a] = ln - m;
      h[a] = hn;
    }
  }
  if (D.fkind == F_LINEAR) {
    float v = lin_c, mag = fabsf(lin_c);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v += fminf(D.fgrad[a] * l[a], D.fgrad[a] * h[a]);
      mag += fmaxf(fabsf(D.fgrad[a] * l[a]), fabsf(D.fgrad[a] * h[a]));
    }
    return v - 1e-5f * mag - 1e-6f - D.theta < 0.0f;
  }
  int c0[3], c1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float top = (float)(D.fn[a] - 2);
    c0[a] = (int)fminf(fmaxf(floorf((l[a] - D.fo[a]) * D.finv[a]), 0.0f), top);
    c1[a] = (int)fminf(fmaxf(floorf((h[a] - D.fo[a]) * D.finv[a]), 0.0f), top);
  }
  const size_t cx = (size_t)D.fn[0] - 1, cy = (size_t)D.fn[1] - 1;
  const size_t kx = (cx + 3) >> 2, ky = (cy + 3) >> 2;
  float m = INFINITY;
  for (int k = c0[2] >> 2; k <= c1[2] >> 2; ++k)
    for (int j = c0[1] >> 2; j <= c1[1] >> 2; ++j)
      for (int i = c0[0] >> 2; i <= c1[0] >> 2; ++i)
        m = fminf(m, D.fcoarse[((size_t)k * ky + j) * kx + i]);
  if (bound_margin(m) - D.theta >= 0.0f) return false;
  m = INFINITY;
  for (int k = c0[2]; k <= c1[2]; ++k)
    for (int j = c0[1]; j <= c1[1]; ++j)
      for (int i = c0[0]; i <= c1[0]; ++i) m = fminf(m, D.fcmin[((size_t)k * cy + j) * cx + i]);
  return bound_margin(m) - D.theta < 0.0f;
}

// Undercooling at the departure site of a record is negative (the site
// melted), tested first against the bound of its cell neighbourhood.
template <int PM = 2>
__device__ __forceinline__ bool departure_melted(const Dev& D, const float* __restrict__ G,
                                                 int sx, int sy, int sz, float lin_c) {
  const P3 x = lattice_pos(G, sx, sy, sz, 0, 0.0f);
  return may_melt<PM>(D, x, x, lin_c) && field_at<PM>(D, x, lin_c) - D.theta < 0.0f;
}

// Rounded lattice position of world point y in grain G (crystal frame).
__device__ __forceinline__ void lattice_round(const float* __restrict__ G, float inv_lambda, P3 y,
                                              int out[3]) {
  const float dx = y.x - G[0], dy = y.y - G[1], dz = y.z - G[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float l = fmaf(G[10 + k], dz, fmaf(G[7 + k], dy, G[4 + k] * dx));
    out[k] = (int)rintf(l * inv_lambda);
  }
}

// ----------------------------------------------------------- wave tools ---
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Appends for lanes with pred; one atomic per wave.  Returns the slot or NIL.
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
  const int lane = lane_id();
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return NIL;
  const int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  return pred ? base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull)) : NIL;
}

// Groups runs of equal keys in consecutive lanes.
struct Run {
  int head, off, len;
};
__device__ __forceinline__ Run wave_run(uint32_t key) {
  const int lane = lane_id();
  const uint32_t prev = __shfl_up(key, 1u);
  const bool head = (lane == 0) || (prev != key);
  const unsigned long long H = __ballot(head);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long below = H & upto;
  const unsigned long long above = H & ~upto;
  Run r;
  r.head = 63 - __clzll((long long)below);
  const int next = above ? (__ffsll((long long)above) - 1) : 64;
  r.len = next - r.head;
  r.off = lane - r.head;
  return r;
}

// Contiguous chunk of [0, n) per block; blocks on one XCD (round-robin
// dispatch: block b runs on XCD b % 8) get neighbouring chunks so that they
// share that XCD's L2.
struct Chunk {
  uint32_t begin, end;
};
// Block index and grid size of a launch as seen by one context: the real
// ones for a plain launch, the context's share of the blocks for a batched
// launch.
struct VGrid {
  uint32_t b, G;
};
__device__ __forceinline__ uint32_t logical_block(const VGrid& V) {
  const uint32_t G = V.G, b = V.b;
  return ((G & 7u) == 0u) ? (b & 7u) * (G >> 3) + (b >> 3) : b;
}
// Chunk of [0, n) of logical block lb on a grid of G blocks (whole granules).
__device__ __forceinline__ Chunk chunk_at(uint32_t n, uint32_t granule, uint32_t G, uint32_t lb) {
  uint32_t per = (n + G - 1u) / G;
  per = (per + granule - 1u) / granule * granule;
  const uint64_t b = (uint64_t)lb * per;
  Chunk c;
  c.begin = (uint32_t)(b < n ? b : n);
  const uint64_t e = b + per;
  c.end = (uint32_t)(e < n ? e : n);
  return c;
}
__device__ __forceinline__ Chunk chunk_of(const VGrid& V, uint32_t n, uint32_t granule) {
  return chunk_at(n, granule, V.G, logical_block(V));
}
// Regions of a per-block list written by a kernel of G_w blocks, as read by
// this block: an even share [lb G_w / G, (lb + 1) G_w / G) of them, so that
// with grids that are multiples of 8 a region is read on the XCD that wrote it.
__device__ __forceinline__ Chunk regions_of(const VGrid& V, uint32_t G_w) {
  const uint64_t lb = logical_block(V), G = V.G;
  Chunk c;
  c.begin = (uint32_t)(lb * G_w / G);
  c.end = (uint32_t)((lb + 1u) * G_w / G);
  return c;
}

// A context whose state must not change: a capacity error, or held.
__device__ __forceinline__ bool dead(const Dev& D) {
  return (__hip_atomic_load(&D.cnt->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
          (ERR_CAPACITY | HOLD)) != 0u;
}

// The context as seen by a kernel of the current step: the launch argument
// (the same for every step) with the roles of the double-buffered stores set
// by the step state in the counters.
// Step state read from the counters is the same for every lane: kept in
// scalar registers.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ double uniform_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = uniform_u32((uint32_t)b), hi = uniform_u32((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ uint32_t step_epoch(const Dev& D) { return uniform_u32(D.cnt->epoch); }

__device__ __forceinline__ Dev dev_view(const Dev& Dv) {
  Dev D = Dv;
  if (uniform_u32(D.cnt->par) & 1u) {
    uint4* r = D.A;
    D.A = D.B;
    D.B = r;
    uint32_t* t = D.tagA;
    D.tagA = D.tagB;
    D.tagB = t;
  }
  if (uniform_u32(D.cnt->spar) & 1u) {
    uint4* r = D.S;
    D.S = D.S2;
    D.S2 = r;
    float4* p = D.PS;
    D.PS = D.PS2;
    D.PS2 = p;
  }
  return D;
}

// Launch bindings.  Plain: one context, passed by value.  Batch: many
// contexts in one launch; block b serves context map[b] & 0xFFF as its
// virtual block map[b] >> 12 of gsz[context] blocks.  The contexts' tables
// hold offsets from `base` (their common workspace) in place of pointers,
// so that the rebuilt pointers stay global-memory pointers.
struct Plain {
  Dev d;
  __device__ __forceinline__ void bind(Dev& D, VGrid& V) const {
    D = dev_view(d);
    V.b = blockIdx.x;
    V.G = gridDim.x;
  }
};

struct Batch {
  const Dev* __restrict__ tab;
  char* __restrict__ base;
  const uint32_t* __restrict__ map;
  const uint32_t* __restrict__ gsz;
  __device__ __forceinline__ void bind(Dev& D, VGrid& V) const {
    const uint32_t e = map[blockIdx.x];
    const uint32_t m = e & 0xFFFu;
    V.b = e >> 12;
    V.G = gsz[m];
    Dev t = tab[m];
#define GE_REBASE(f)                                                                 \
  t.f = ((uintptr_t)t.f == NULL_OFFSET) ? nullptr : (decltype(t.f))(base + (uintptr_t)t.f);
    GE_DEV_POINTERS(GE_REBASE)
#undef GE_REBASE
    D = dev_view(t);
  }
};

// LINEAR field constant dT0 + rate t of the current step (FP64, then FP32).
__device__ __forceinline__ float lin_const(const Dev& D) {
  return D.fkind == F_LINEAR ? (float)(D.fdT0 + D.frate * uniform_f64(D.cnt->t)) : 0.0f;
}

// The stopped store is re-sorted after every resort_every-th step (the
// re-sort kernels run after k_finish has counted the step).
__device__ __forceinline__ bool resort_due(const Dev& D) {
  return uniform_u32((uint32_t)(D.cnt->step % (unsigned long long)D.resort_every)) == 0u;
}

// Block-wide exclusive scan of one uint32 per thread (TPB threads).
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
  const int lane = lane_id(), wid = (int)(threadIdx.x >> 6);
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, (unsigned)o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < TPB / 64; ++w) {
    uint32_t s = wsum[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

__device__ __forceinline__ unsigned long long block_excl_scan64(unsigned long long v,
                                                                unsigned long long* wsum,
                                                                unsigned long long& total) {
  const int lane = lane_id(), wid = (int)(threadIdx.x >> 6);
  unsigned long long incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    unsigned long long y = __shfl_up(incl, (unsigned)o);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  unsigned long long off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < TPB / 64; ++w) {
    unsigned long long s = wsum[w];
    if (w < wid) off += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

// Orders the LDS accesses of this wave's lanes: every access before it
// (by any lane of the wave) is complete and visible to every access after it.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t& total) {
  const int lane = lane_id();
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, (unsigned)o);
    if (lane >= o) incl += y;
  }
  total = __shfl(incl, 63);
  return incl - v;
}


// One-entry cache of claim slots: the sites a spawner claims lie within one
// lattice step of its reached site, mostly in the same 8^3 slot brick.
struct SlotCache {
  uint64_t key;
  int64_t slot;
};
// One-entry cache of claim blocks for the tests: the sites a spawner tests
// lie within two lattice steps of its reached site, mostly in the same
// block of slot bricks.  A slot of a known block that was never
// taken has all its words zero, so the tests read it without checking.
struct BlockCache {
  uint64_t bkey;
  int64_t blk;
};

__device__ __forceinline__ bool cached_test(const Dev& D, BlockCache& c, uint32_t g, int sx,
                                            int sy, int sz, uint32_t which) {
  const uint64_t key = claim_key(g, sx, sy, sz);
  const uint64_t bkey = claim_block_key(key);
  if (bkey != c.bkey) {
    c.bkey = bkey;
    c.blk = block_find<true>(D, bkey);
  }
  if (c.blk < 0) return false;
  const uint64_t slot = (uint64_t)c.blk * CLAIM_BLOCK_SLOTS + claim_fine(key);
  const uint32_t b = site_bit(sx, sy, sz);
  const unsigned long long m = 1ull << (b & 63);
  const unsigned long long* w = D.cbits + (size_t)slot * 24 + (b >> 6);
  unsigned long long v = 0;
  if (which & M_CLAIMED) v |= load_cached(w + CB_CLAIMED);
  if (which & M_REACHED) v |= load_cached(w + CB_REACHED);
  if (which & M_NOW) v |= load_cached(w + CB_NOW);
  return (v & m) != 0;
}

// Claim words of the reached site S's slot around S: the z-layers
// (S.z & 7) - 2 .. + 1.  Every target S + e and every same-step competitor
// T - e' of a target T lies in them or in another slot.  No update made
// during k_branch changes the outcome of its tests (a target is claimed only
// by its winner, after that spawner's own test, and this step's marks do not
// change), so the words are read once, through the cache: one probe and
// twelve independent loads.  The same holds for the tests outside the window.
struct SlotWin {
  int bx, by, bz, z0;
  unsigned long long a0, a1, a2, a3;  // claimed | reached | this step's marks
  unsigned long long n0, n1, n2, n3;  // this step's marks
};

__device__ __forceinline__ SlotWin load_win(const Dev& D, uint32_t slot, int sx, int sy, int sz) {
  SlotWin w;
  w.bx = sx >> 3;
  w.by = sy >> 3;
  w.bz = sz >> 3;
  w.z0 = (sz & 7) - 2;
  const unsigned long long* q = D.cbits + (size_t)(slot == NIL ? 0u : slot) * 24;
  auto layer = [&](int z, unsigned long long& any, unsigned long long& now) {
    unsigned long long c = 0, r = 0, m = 0;
    if (slot != NIL && z >= 0 && z < 8) {
      c = load_cached(q + CB_CLAIMED + z);
      r = load_cached(q + CB_REACHED + z);
      m = load_cached(q + CB_NOW + z);
    }
    any = c | r | m;
    now = m;
  };
  layer(w.z0, w.a0, w.n0);
  layer(w.z0 + 1, w.a1, w.n1);
  layer(w.z0 + 2, w.a2, w.n2);
  layer(w.z0 + 3, w.a3, w.n3);
  return w;
}

// Bit of a site in the window (false: the site is outside it).
__device__ __forceinline__ bool win_bit(const SlotWin& w, int sx, int sy, int sz, bool now_only,
                                        bool& hit) {
  if ((sx >> 3) != w.bx || (sy >> 3) != w.by || (sz >> 3) != w.bz) return false;
  const int j = (sz & 7) - w.z0;
  if (j < 0 || j > 3) return false;
  // Word j by masks (a select chain would be turned into an indexed table
  // in scratch memory).
  const unsigned long long m0 = 0ull - (unsigned long long)(j == 0);
  const unsigned long long m1 = 0ull - (unsigned long long)(j == 1);
  const unsigned long long m2 = 0ull - (unsigned long long)(j == 2);
  const unsigned long long m3 = 0ull - (unsigned long long)(j == 3);
  const unsigned long long v =
      now_only ? ((w.n0 & m0) | (w.n1 & m1) | (w.n2 & m2) | (w.n3 & m3))
               : ((w.a0 & m0) | (w.a1 & m1) | (w.a2 & m2) | (w.a3 & m3));
  hit = ((v >> ((sx & 7) | ((sy & 7) << 3))) & 1ull) != 0ull;
  return true;
}

// claim_or through a one-entry find-or-insert cache.
__device__ __forceinline__ void cached_or(const Dev& D, SlotCache& c, uint32_t g, int sx, int sy,
                                          int sz, uint32_t which) {
  const uint64_t key = claim_key(g, sx, sy, sz);
  if (key != c.key || c.slot < 0) {
    c.key = key;
    c.slot = claim_get(D, key);
  }
  if (c.slot < 0) return;
  const uint32_t b = site_bit(sx, sy, sz);
  const unsigned long long m = 1ull << (b & 63);
  unsigned long long* w = D.cbits + (size_t)c.slot * 24 + (b >> 6);
  if (which & M_CLAIMED) atomicOr(w + CB_CLAIMED, m);
  if (which & M_REACHED) atomicOr(w + CB_REACHED, m);
  if (which & M_NOW) atomicOr(w + CB_NOW, m);
}

// Owner word of a cell: NIL (empty), the one grain of its particles, or MIXED.
__device__ __forceinline__ uint32_t owner_merge(uint32_t own, uint32_t g) {
  return own == NIL ? g : (own == g ? g : MIXED);
}

// ------------------------------------------------------- stopped store ----
// Slab bits of a position in its cell: bit 8 a + k for the k-th eighth of
// the cell along axis a (the cell coordinate as in cell_of).
__device__ __forceinline__ uint32_t slab_bits(const Dev& D, P3 p) {
  const float x[3] = {p.x, p.y, p.z};
  uint32_t bits = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float u = (x[a] - D.lo[a]) * D.inv_h;
    const float f = u - floorf(u);
    const bool inside = u >= 0.0f && u < (float)D.n[a];
    const uint32_t k = min((uint32_t)(f * 8.0f), 7u);
    bits |= (inside ? (1u << k) : 0xFFu) << (8 * a);
  }
  return bits;
}

// Writes record r (state STOPPED) and its placed position pw (wrapped
// position, owner word) at slot j of the stopped store and links it into the
// cell list of recently stopped particles.  Callers run in kernels that
// never read those lists.
__device__ __forceinline__ void stopped_put(const Dev& D, uint32_t j, uint4 r, float4 pw) {
  if (j >= D.cap_s) {
    atomicOr(&D.cnt->err, ERR_CAPACITY);
    return;
  }
  const uint32_t g = grain_of(pw);
  D.S[j] = r;
  D.PS[j] = pw;
  const C3 c = cell_of(D, p3_of(pw));
  const uint32_t ci = cell_index(D, c.x, c.y, c.z);
  const uint32_t old = atomicExch(&D.shead[ci], j);
  D.snext[j] = old;
  // The slab of each axis that holds the particle (all eight of an axis
  // whose position lies outside the grid, clamped into its outer cell).
  const uint32_t bits = slab_bits(D, p3_of(pw));
  if ((D.smask[ci] & bits) != bits) atomicOr(&D.smask[ci], bits);
  // Owner word of the cell's stopped particles; it only moves from NIL to a
  // grain to MIXED, so a stale read costs one failed compare-and-swap.
  uint32_t* sown = &D.cown[ci].y;
  uint32_t own = *sown;
  for (;;) {
    const uint32_t nw = owner_merge(own, g);
    if (nw == own) break;
    const uint32_t prev = atomicCAS(sown, own, nw);
    if (prev == own) break;
    own = prev;
  }
  // The same for the brick's stopped owner word.
  uint32_t* bown_s = &D.bmeta[ci / (uint32_t)BRICK_CELLS].w;
  own = *bown_s;
  for (;;) {
    const uint32_t nw = owner_merge(own, g);
    if (nw == own) break;
    const uint32_t prev = atomicCAS(bown_s, own, nw);
    if (prev == own) break;
    own = prev;
  }
}

// ==================================================================== step
template <class Bind, int PM>
__global__ __launch_bounds__(TPB, 8) void k_advance(Bind Bd, float dt) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const float lin_c = lin_const(D);
  // Step of an adjoint recording (tagged particles only).
  const int32_t adj_k = D.tagA ? (int32_t)(D.cnt->step - D.adj_step0) : 0;
  if (D.tagA && V.b == 0 && threadIdx.x == 0) D.adj_linc[adj_k] = lin_c;
  if (dead(D)) return;
  __shared__ uint32_t s_nsp, s_adv, s_exit, s_bad, s_max;
  if (threadIdx.x == 0) {
    s_nsp = 0;
    s_adv = 0;
    s_exit = 0;
    s_bad = 0;
    s_max = 0;
  }
  __syncthreads();
  const uint32_t n = D.cnt->n_active;
  const Chunk ch = chunk_of(V, n, TPB);
  const int lane = lane_id();
  float max_step = 0.0f;
  uint32_t nadv = 0, nexit = 0, bad = 0, nrm = 0;
  for (uint32_t base = ch.begin; base < ch.end; base += TPB) {
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < ch.end;
    uint4 r = valid ? D.A[i] : make_uint4(0u, 0u, 0u, 0u);
    const bool act = valid && ((rec_fl(r) & 3u) == ST_ACTIVE);
    uint32_t ckey = NIL, bkey = NIL;
    bool spawn = false, exited = false;
    P3 x2 = {0.0f, 0.0f, 0.0f};
    uint32_t tag = NIL;
    bool gone = false;
    if (act && D.melting) {
      // Melting: a particle whose departure site melted this step goes, and
      // its target is released.
      const uint32_t g = rec_grain(r);
      const float* G = D.gtab + (size_t)g * GT_STRIDE;
      gone = departure_melted<PM>(D, G, rec_sx(r), rec_sy(r), rec_sz(r), lin_c);
      if (gone) {
        const int d = rec_dir(r);
        int T[3] = {rec_sx(r), rec_sy(r), rec_sz(r)};
        T[d >> 1] += (d & 1) ? -1 : 1;
        const int64_t slot = claim_find(D, claim_key(g, T[0], T[1], T[2]));
        if (slot >= 0) {
          const uint32_t b = site_bit(T[0], T[1], T[2]);
          atomicAnd(D.cbits + (size_t)slot * 24 + CB_CLAIMED + (b >> 6), ~(1ull << (b & 63)));
        }
        r = with_fl(r, ST_RETIRED);
        D.A[i] = r;
        nrm += 1;
      }
    }
    if (act && !gone) {
      const uint32_t g = rec_grain(r);
      const int d = rec_dir(r);
      const int sx = rec_sx(r), sy = rec_sy(r), sz = rec_sz(r);
      const float s = rec_s(r);
      if (D.tagA) {  // adjoint recording: checkpoint of the travel every adj_K steps
        tag = D.tagA[i];
        if (tag != NIL && adj_k % D.adj_K == 0)
          D.adj_ck[(size_t)(adj_k / D.adj_K) * D.adj_ncap + tag] = s;
      }
      const float* G = D.gtab + (size_t)g * GT_STRIDE;
      const P3 x = lattice_pos(G, sx, sy, sz, d, s);
      const float dT = field_at<PM>(D, x, lin_c) - D.theta;
      float delta = velocity(D, dT) * dt;
      // velocity() maps a NaN undercooling to rest: test both.
      if (!isfinite(dT) || !isfinite(delta)) {
        bad |= ERR_NUMERIC;
        delta = 0.0f;
      }
      if (delta > D.rc_half) bad |= ERR_CFL;
      max_step = fmaxf(max_step, delta);
      const float s2 = s + delta;
      x2 = lattice_pos(G, sx, sy, sz, d, s2);
      nadv += 1;
      const bool inside = in_box<PM>(D, x2);
      uint32_t fl;
      if (D.box_exit && !inside) {
        exited = true;
        fl = ST_STOPPED;
        nexit += 1;
      } else if (D.branching && s2 >= D.lambda0) {
        spawn = true;
        fl = ST_ACTIVE | FL_SPAWN;
        if (s2 >= 2.0f * D.lambda0) bad |= ERR_CFL;
      } else {
        fl = ST_ACTIVE | FL_KEEP;
        const C3 c = cell_of(D, PM == 0 ? x2 : place(D, x2).p);
        ckey = cell_index(D, c.x, c.y, c.z);
        bkey = ckey / (uint32_t)BRICK_CELLS;
      }
      r = make_rec(s2, g, d, sx, sy, sz, fl);
      D.A[i] = r;
    }
    // Cell and brick counts of the particles that stay active: one atomic
    // per run of equal keys in consecutive lanes (the input is cell-sorted).
    const Run rc = wave_run(ckey);
    if (ckey != NIL && rc.off == 0) atomicAdd(&D.ccnt[ckey], (uint32_t)rc.len);
    const Run rb = wave_run(bkey);
    if (bkey != NIL && rb.off == 0) atomicAdd(&D.bcnt[bkey], (uint32_t)rb.len);
    // Spawners go to the block's region of the spawner list.
    const unsigned long long m = __ballot(spawn);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      uint32_t wb = 0;
      if (lane == leader) wb = atomicAdd(&s_nsp, (uint32_t)__popcll(m));
      wb = __shfl(wb, leader);
      if (spawn) D.spawn[ch.begin + wb + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = i;
    }
    const uint32_t sj = wave_append(exited, &D.cnt->n_stopped);
    if (exited) {
      stopped_put(D, sj, r, PM == 0 ? pos4(x2, rec_grain(r)) : placed4(D, x2, rec_grain(r)));
      if (tag != NIL) {
        D.adj_nact[tag] = adj_k + 1;
        D.adj_sfin[tag] = rec_s(r);
      }
    }
  }
  if (nadv) atomicAdd(&s_adv, nadv);
  if (nexit) atomicAdd(&s_exit, nexit);
  if (nrm) atomicAdd(&D.cnt->removed, (unsigned long long)nrm);
  if (bad) atomicOr(&s_bad, bad);
  if (max_step > 0.0f) atomicMax(&s_max, __float_as_uint(max_step));
  __syncthreads();
  // The reached sites of the block's spawners, marked as reached this step
  // (the mark the same-step competition of the branching reads), with the
  // claim slot of each kept next to the spawner's index.  The records were
  // written by this block before the barrier.
  for (uint32_t k = threadIdx.x; k < s_nsp; k += TPB) {
    const uint32_t pos = ch.begin + k;
    const uint4 r = D.A[D.spawn[pos]];
    const int d = rec_dir(r), a = d >> 1, e = (d & 1) ? -1 : 1;
    const int sx = rec_sx(r) + (a == 0 ? e : 0), sy = rec_sy(r) + (a == 1 ? e : 0),
              sz = rec_sz(r) + (a == 2 ? e : 0);
    const int64_t slot = claim_get(D, claim_key(rec_grain(r), sx, sy, sz));
    D.spslot[pos] = slot < 0 ? NIL : (uint32_t)slot;
    if (slot < 0) continue;
    const uint32_t b = site_bit(sx, sy, sz);
    atomicOr(D.cbits + (size_t)slot * 24 + CB_NOW + (b >> 6), 1ull << (b & 63));
  }
  if (threadIdx.x == 0) {
    D.spawn_cnt[logical_block(V)] = s_nsp;
    if (s_adv) atomicAdd(&D.cnt->advanced, (unsigned long long)s_adv);
    if (s_exit) atomicAdd(&D.cnt->exited, (unsigned long long)s_exit);
    if (s_bad) atomicOr(&D.cnt->err, s_bad);
    if (s_max) atomicMax(&D.cnt->max_step, s_max);
  }
}

// Exclusive prefix of the per-block spawner counts (one block): spawner i
// of the step is in the region r with spawn_off[r] <= i < spawn_off[r + 1].
template <class Bind>
__global__ __launch_bounds__(1024) void k_spawn_scan(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  __shared__ uint32_t s_w[16];
  const uint32_t G = D.sched[TK_ADVANCE];
  const uint32_t per = (G + 1023u) / 1024u;  // regions per thread, G <= STREAM_GRID
  const uint32_t r0 = threadIdx.x * per;
  uint32_t v[2] = {0u, 0u};
  for (uint32_t k = 0; k < per && k < 2u; ++k) v[k] = r0 + k < G ? D.spawn_cnt[r0 + k] : 0u;
  uint32_t tot;
  const uint32_t ex = wave_excl_scan(v[0] + v[1], tot);
  if (lane_id() == 0) s_w[threadIdx.x >> 6] = tot;
  __syncthreads();
  uint32_t wbase = 0;
  for (uint32_t w = 0; w < (threadIdx.x >> 6); ++w) wbase += s_w[w];
  uint32_t acc = wbase + ex;
  for (uint32_t k = 0; k < per && k < 2u; ++k) {
    if (r0 + k < G) D.spawn_off[r0 + k] = acc;
    acc += v[k];
  }
  if (threadIdx.x == 1023u) D.spawn_off[G] = acc;
}

// The step's spawners as one list: this block's even share of them, and the
// lookup of spawner i (the region offsets are staged in LDS).
struct SpawnView {
  uint32_t n, G, total;
};
__device__ __forceinline__ SpawnView spawn_view(const Dev& D, uint32_t* s_off) {
  SpawnView v;
  v.n = D.cnt->n_active;
  v.G = D.sched[TK_ADVANCE];
  for (uint32_t r = threadIdx.x; r <= v.G; r += blockDim.x) s_off[r] = D.spawn_off[r];
  __syncthreads();
  v.total = s_off[v.G];
  return v;
}
// Position of spawner i of the step in the per-block regions of the
// spawner list (where the advance wrote its index and its claim slot).
__device__ __forceinline__ uint32_t spawn_pos(const SpawnView& v, const uint32_t* s_off,
                                              uint32_t i) {
  uint32_t lo = 0, hi = v.G;  // s_off[lo] <= i < s_off[hi]
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s_off[mid] <= i) lo = mid;
    else hi = mid;
  }
  return chunk_at(v.n, TPB, v.G, lo).begin + (i - s_off[lo]);
}

// At most 80 registers, for six waves per SIMD: more waves in flight hide
// more of the latency of the branching's loads and atomics.
template <class Bind>
__global__ __launch_bounds__(TPB, 6) void k_branch(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  __shared__ uint32_t s_sp, s_ch;
  if (threadIdx.x == 0) {
    s_sp = 0;
    s_ch = 0;
  }
  __syncthreads();
  __shared__ uint32_t s_off[STREAM_GRID + 1];
  const SpawnView v = spawn_view(D, s_off);
  const Chunk it = chunk_of(V, v.total, 1u);
  uint32_t nsp = 0, nch = 0;
  // The next round's spawner (index, record, claim slot) is loaded during
  // this round, off the chain of dependent loads.  Each record is read and
  // written only in its own spawner's round.
  uint32_t ni = 0, nslot = NIL;
  uint4 nr = make_uint4(0u, 0u, 0u, 0u);
  if (it.begin + threadIdx.x < it.end) {
    const uint32_t np = spawn_pos(v, s_off, it.begin + threadIdx.x);
    ni = D.spawn[np];
    nr = D.A[ni];
    nslot = D.spslot[np];
  }
  // The trip count is the same for the block's waves, so the deposition of
  // the reached sites can be added once per run of equal cells of a wave.
  for (uint32_t k0 = it.begin; k0 < it.end; k0 += TPB) {
    const uint32_t k = k0 + threadIdx.x;
    const uint32_t i = ni, slot = nslot;
    const uint4 r = nr;
    if (k + TPB < it.end) {
      const uint32_t np = spawn_pos(v, s_off, k + TPB);
      ni = D.spawn[np];
      nr = D.A[ni];
      nslot = D.spslot[np];
    }
    uint32_t dep = NIL, rg = NIL;
    // Children of this lane's spawner (mask 0 past the range), placed after
    // the tests so that the cell and brick counts of a direction are added
    // once per run of equal keys of the wave.
    uint32_t mask = 0, g = 0;
    int S[3] = {0, 0, 0};
    float sc2 = 0.0f;
    SlotCache wc{~0ull, -1};
    SiteFrame F{};
    if (k < it.end) {
      g = rec_grain(r);
      const int d = rec_dir(r);
      const float s2 = rec_s(r);
      // Reached site S = departure site + one step in direction d.
      const int dstep = (d & 1) ? -1 : 1;
      S[0] = rec_sx(r) + ((d >> 1) == 0 ? dstep : 0);
      S[1] = rec_sy(r) + ((d >> 1) == 1 ? dstep : 0);
      S[2] = rec_sz(r) + ((d >> 1) == 2 ? dstep : 0);
      BlockCache sc{~0ull, -1};
      const SlotWin win = load_win(D, slot, S[0], S[1], S[2]);
      for (int dd = 0; dd < 6; ++dd) {
        const int a = dd >> 1;
        const int sg = (dd & 1) ? -1 : 1;
        if (sg * (a == 0 ? S[0] : a == 1 ? S[1] : S[2]) < 0) continue;  // octant rule: outer only
        const int tx = S[0] + (a == 0 ? sg : 0), ty = S[1] + (a == 1 ? sg : 0),
                  tz = S[2] + (a == 2 ? sg : 0);
        bool taken;
        if (!win_bit(win, tx, ty, tz, false, taken))
          taken = cached_test(D, sc, g, tx, ty, tz, M_CLAIMED | M_REACHED | M_NOW);
        if (taken) continue;
        bool lose = false;
        for (int d2 = 0; d2 < dd && !lose; ++d2) {
          const int a2 = d2 >> 1;
          const int sg2 = (d2 & 1) ? -1 : 1;
          const int ux = tx - (a2 == 0 ? sg2 : 0), uy = ty - (a2 == 1 ? sg2 : 0),
                    uz = tz - (a2 == 2 ? sg2 : 0);
          if (sg2 * (a2 == 0 ? ux : a2 == 1 ? uy : uz) < 0) continue;
          bool rival;
          if (!win_bit(win, ux, uy, uz, true, rival)) rival = cached_test(D, sc, g, ux, uy, uz, M_NOW);
          if (rival) lose = true;
        }
        if (!lose) mask |= 1u << dd;
      }
      // The grain row for the children's positions, loaded before the
      // round's atomics.
      if (mask) F = site_frame(load_grow(D.gtab + (size_t)g * GT_STRIDE), S[0], S[1], S[2]);
      // The parent retires whether or not a child survives: without one, every
      // outer neighbour of S already belongs to the grain (interior point).
      D.A[i] = with_fl(r, ST_RETIRED | FL_SPAWN | (mask << 8));
      sc2 = s2 - D.lambda0;
      wc = SlotCache{claim_key(g, S[0], S[1], S[2]), slot == NIL ? -1 : (int64_t)slot};
      cached_or(D, wc, g, S[0], S[1], S[2], M_REACHED);
      // One bounding-box update for the reached site and the targets of its
      // children (each one step from S).
      int blo[3] = {S[0], S[1], S[2]}, bhi[3] = {S[0], S[1], S[2]};
#pragma unroll
      for (int dd = 0; dd < 6; ++dd) {
        if (!((mask >> dd) & 1u)) continue;
        const int a = dd >> 1;
        if (dd & 1) blo[a] = S[a] - 1;
        else bhi[a] = S[a] + 1;
      }
      bbox_add_box(D, g, blo, bhi);
      if (D.gcnt) dep = deposit_cell(D, D.gtab + (size_t)g * GT_STRIDE, S[0], S[1], S[2]);
      if (D.melting) rg = g;
      nsp += 1;
    }
    for (int dd = 0; dd < 6; ++dd) {
      uint32_t ci = NIL;
      if ((mask >> dd) & 1u) {
        const P3 xc = place(D, frame_pos(F, dd, sc2)).p;
        const C3 c = cell_of(D, xc);
        ci = cell_index(D, c.x, c.y, c.z);
        const int ta = dd >> 1, ts = (dd & 1) ? -1 : 1;
        const int tx = S[0] + (ta == 0 ? ts : 0), ty = S[1] + (ta == 1 ? ts : 0),
                  tz = S[2] + (ta == 2 ? ts : 0);
        cached_or(D, wc, g, tx, ty, tz, M_CLAIMED);
        nch += 1;
      }
      const Run rc = wave_run(ci);
      if (ci != NIL && rc.off == 0) atomicAdd(&D.ccnt[ci], (uint32_t)rc.len);
      const uint32_t bk = ci == NIL ? NIL : ci / (uint32_t)BRICK_CELLS;
      const Run rb = wave_run(bk);
      if (bk != NIL && rb.off == 0) atomicAdd(&D.bcnt[bk], (uint32_t)rb.len);
    }
    if (D.gcnt) {
      const Run run = wave_run(dep);
      if (dep != NIL && run.off == 0) atomicAdd(&D.gcnt[dep], (uint32_t)run.len);
    }
    if (D.melting) {
      const Run run = wave_run(rg);
      if (rg != NIL && run.off == 0) atomicAdd(&D.greach[rg], (uint32_t)run.len);
    }
  }
  if (nsp) atomicAdd(&s_sp, nsp);
  if (nch) atomicAdd(&s_ch, nch);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_sp) atomicAdd(&D.cnt->spawners, (unsigned long long)s_sp);
    if (s_ch) atomicAdd(&D.cnt->children, (unsigned long long)s_ch);
  }
}

// ----------------------------------------------------------- brick scan ---
// Mode 0 (active particles of the step): writes start, count and the epoch
// of each occupied brick.  Mode 1 (stopped-store re-sort): writes start and
// count of every brick.  Both list the occupied bricks and reset the counts.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = TPB * SCAN_ITEMS;
static_assert(SCAN_TILE == (int)SCAN_TILE_HOST, "brick-scan tile of the host launchers");
static_assert(SCAN_ITEMS == 8, "two 16-byte loads per thread");

// The counts of bricks b0 .. b0 + 7 (zero past the last brick): two 16-byte
// loads when all eight exist (b0 is a multiple of eight and the count array
// 256-byte aligned).
__device__ __forceinline__ void load_counts8(const Dev& D, uint64_t b0, uint32_t c[8]) {
  if (b0 + 8u <= D.n_bricks) {
    const uint4 lo = *reinterpret_cast<const uint4*>(D.bcnt + b0);
    const uint4 hi = *reinterpret_cast<const uint4*>(D.bcnt + b0 + 4);
    c[0] = lo.x;
    c[1] = lo.y;
    c[2] = lo.z;
    c[3] = lo.w;
    c[4] = hi.x;
    c[5] = hi.y;
    c[6] = hi.z;
    c[7] = hi.w;
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = b0 + k < D.n_bricks ? D.bcnt[b0 + k] : 0u;
  }
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_scan_reduce(Bind Bd, int mode) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || (mode == 1 && !resort_due(D))) return;
  __shared__ unsigned long long wsum[TPB / 64];
  const uint64_t b0 = (uint64_t)V.b * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t c[SCAN_ITEMS];
  load_counts8(D, b0, c);
  unsigned long long v = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    v += (unsigned long long)c[k] | ((unsigned long long)(c[k] > 0u) << 32);
  unsigned long long total;
  block_excl_scan64(v, wsum, total);
  if (threadIdx.x == 0) D.scan_tmp[V.b] = total;
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_scan_top(Bind Bd, int mode) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || (mode == 1 && !resort_due(D))) return;
  const uint32_t ntiles = (uint32_t)((D.n_bricks + SCAN_TILE - 1) / SCAN_TILE);
  __shared__ unsigned long long wsum[TPB / 64];
  // Each thread takes a run of consecutive tiles: their sum, one block scan
  // of the sums, then the run's exclusive prefixes.  Runs of up to TOP_RUN
  // tiles are loaded at once into registers (one round trip instead of one
  // per tile); longer runs, for grids of more than TPB x TOP_RUN tiles, loop.
  constexpr uint32_t TOP_RUN = 48;
  const uint32_t per = (ntiles + TPB - 1u) / TPB;
  const uint32_t t0 = threadIdx.x * per;
  unsigned long long carry;
  if (per <= TOP_RUN) {
    unsigned long long v[TOP_RUN];
    unsigned long long sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < TOP_RUN; ++q) {
      v[q] = q < per && t0 + q < ntiles ? D.scan_tmp[t0 + q] : 0ull;
      sum += v[q];
    }
    unsigned long long run = block_excl_scan64(sum, wsum, carry);
#pragma unroll
    for (uint32_t q = 0; q < TOP_RUN; ++q) {
      if (q < per && t0 + q < ntiles) D.scan_tmp[t0 + q] = run;
      run += v[q];
    }
  } else {
    unsigned long long sum = 0;
    for (uint32_t q = 0; q < per; ++q)
      if (t0 + q < ntiles) sum += D.scan_tmp[t0 + q];
    unsigned long long run = block_excl_scan64(sum, wsum, carry);
    for (uint32_t q = 0; q < per; ++q) {
      if (t0 + q >= ntiles) break;
      const unsigned long long x = D.scan_tmp[t0 + q];
      D.scan_tmp[t0 + q] = run;
      run += x;
    }
  }
  if (threadIdx.x == 0) {
    const uint32_t n_out = (uint32_t)(carry & 0xFFFFFFFFull);
    const uint32_t n_occ = (uint32_t)(carry >> 32);
    if (mode == 0) {
      D.cnt->n_out = n_out;
      D.cnt->n_occ = n_occ;
      if (n_out > D.cap_p) atomicOr(&D.cnt->err, ERR_CAPACITY);
    } else {
      D.cnt->n_socc = n_occ;
      D.cnt->n_resorted = n_out;
    }
  }
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_scan_write(Bind Bd, int mode) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || (mode == 1 && !resort_due(D))) return;
  const uint32_t epoch = step_epoch(D);
  __shared__ unsigned long long wsum[TPB / 64];
  const uint64_t b0 = (uint64_t)V.b * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_ITEMS;
  uint32_t c[SCAN_ITEMS];
  load_counts8(D, b0, c);
  unsigned long long v = 0;
  uint32_t any = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v += (unsigned long long)c[k] | ((unsigned long long)(c[k] > 0u) << 32);
    any |= c[k];
  }
  unsigned long long total;
  unsigned long long ex = block_excl_scan64(v, wsum, total) + D.scan_tmp[V.b];
  // Counts back to zero: the eight at once when they all exist.
  const bool whole = b0 + 8u <= D.n_bricks;
  if (whole && any) {
    *reinterpret_cast<uint4*>(D.bcnt + b0) = make_uint4(0u, 0u, 0u, 0u);
    *reinterpret_cast<uint4*>(D.bcnt + b0 + 4) = make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const uint64_t b = b0 + k;
    if (b < D.n_bricks) {
      const uint32_t start = (uint32_t)(ex & 0xFFFFFFFFull);
      const uint32_t occ = (uint32_t)(ex >> 32);
      if (mode == 1) D.bsinfo[b] = make_uint2(start, c[k]);
      if (c[k] > 0u) {
        if (mode == 0) {
          D.binfo[b] = make_uint2(start, c[k]);
          // Step stamp and an empty owner range; the stopped owner word (.w)
          // is kept.
          uint4* m = D.bmeta + b;
          *reinterpret_cast<uint2*>(m) = make_uint2(epoch, NIL);
          reinterpret_cast<uint32_t*>(m)[2] = 0u;
        }
        D.occ[occ] = (uint32_t)b;
        if (!whole) D.bcnt[b] = 0u;
      }
      ex += (unsigned long long)c[k] | ((unsigned long long)(c[k] > 0u) << 32);
    }
  }
}

// One wave per occupied brick, one lane per cell: cell starts from the
// brick start and an exclusive scan of the 64 cell counts.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_cellscan(Bind Bd, int mode) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || (mode == 1 && !resort_due(D))) return;
  const uint32_t nocc = mode == 0 ? D.cnt->n_occ : D.cnt->n_socc;
  const uint32_t waves = V.G * (TPB / 64);
  const uint32_t lane = (uint32_t)lane_id();
  // Software pipeline: the next brick's start and counts are loaded during
  // this one, and its index one brick earlier.
  uint32_t k = V.b * (TPB / 64) + (threadIdx.x >> 6);
  uint32_t b1 = k < nocc ? D.occ[k] : 0u;
  uint32_t b2 = k + waves < nocc ? D.occ[k + waves] : 0u;
  uint32_t start1 = 0u, cnt1 = 0u;
  if (k < nocc) {
    start1 = mode == 0 ? D.binfo[b1].x : D.bsinfo[b1].x;
    cnt1 = D.ccnt[b1 * (uint32_t)BRICK_CELLS + lane];
  }
  for (; k < nocc; k += waves) {
    const uint32_t b = b1, start = start1, cnt = cnt1;
    if (k + waves < nocc) {
      b1 = b2;
      start1 = mode == 0 ? D.binfo[b1].x : D.bsinfo[b1].x;
      cnt1 = D.ccnt[b1 * (uint32_t)BRICK_CELLS + lane];
    }
    if (k + 2u * waves < nocc) b2 = D.occ[k + 2u * waves];
    const uint32_t ci = b * (uint32_t)BRICK_CELLS + lane;
    uint32_t tot;
    const uint32_t ex = wave_excl_scan(cnt, tot);
    if (mode == 0) D.cstart[ci] = start + ex;
    else D.sstart[ci] = start + ex;
  }
}

// ------------------------------------------------------------- scatter ----
// Grain range of a brick (one update per run of equal (brick, grain) lanes).
__device__ __forceinline__ void note_grain(const Dev& D, uint32_t b, uint32_t g) {
  atomicMin(&D.bmeta[b].y, g);
  atomicMax(&D.bmeta[b].z, g);
}
// The same for children, which arrive in no order: the range is read first
// (by the caller, clo and chi), an atomic only when it grows (most children
// join a grain already noted in their brick).  The range only grows, so a read served by the cache (the
// range as it was at the kernel's start, or wider) can only cost an atomic
// that changes nothing.
__device__ __forceinline__ void note_grain_seen(uint32_t* range, uint32_t clo, uint32_t chi,
                                                uint32_t g) {
  if (g < clo) atomicMin(range, g);
  if (g > chi) atomicMax(range + 1, g);
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_scatter(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  const uint32_t n = D.cnt->n_active;
  const Chunk ch = chunk_of(V, n, TPB);
  for (uint32_t base = ch.begin; base < ch.end; base += TPB) {
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < ch.end;
    const uint4 r = valid ? D.A[i] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t fl = valid ? rec_fl(r) : 0u;
    uint32_t ckey = NIL;
    uint32_t g = NIL;
    P3 p = {0.0f, 0.0f, 0.0f};
    if (fl & FL_KEEP) {
      const Placed pl = place(D, rec_pos(D, r));
      g = owner_id(rec_grain(r), pl.code);
      p = pl.p;
      const C3 c = cell_of(D, p);
      ckey = cell_index(D, c.x, c.y, c.z);
    }
    // Ranks within the cell: one decrement per run of equal cells; the cell
    // counts return to zero once every particle has been placed.
    const Run run = wave_run(ckey);
    uint32_t rbase = 0;
    if (ckey != NIL && run.off == 0) rbase = atomicSub(&D.ccnt[ckey], (uint32_t)run.len);
    rbase = __shfl(rbase, run.head);
    // Grain range per brick: one update per run of equal (brick, grain).
    const uint32_t bkey = ckey == NIL ? NIL : ckey / (uint32_t)BRICK_CELLS;
    const uint32_t pb = __shfl_up(bkey, 1u), pg = __shfl_up(g, 1u);
    const bool head = lane_id() == 0 || pb != bkey || pg != g;
    if (ckey != NIL) {
      const uint32_t rank = rbase - (uint32_t)run.len + (uint32_t)run.off;
      const uint32_t dst = D.cstart[ckey] + rank;
      if (dst < D.cap_p) {
        D.B[dst] = with_fl(r, ST_ACTIVE);
        D.P[dst] = pos4(p, g);
        if (D.tagA) D.tagB[dst] = D.tagA[i];
      }
      if (head) note_grain(D, bkey, g);
    }
  }
}

// Children of the spawners (from the per-block spawner lists) to their cell
// slots; clears the spawners' marks of the current step.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_scatter_children(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  __shared__ uint32_t s_off[STREAM_GRID + 1];
  const SpawnView v = spawn_view(D, s_off);
  const Chunk it = chunk_of(V, v.total, 1u);
  for (uint32_t k = it.begin + threadIdx.x; k < it.end; k += TPB) {
    const uint32_t kp = spawn_pos(v, s_off, k);
    const uint4 r = D.A[D.spawn[kp]];
    const uint32_t fl = rec_fl(r);
    const uint32_t gs = rec_grain(r);
    const int d = rec_dir(r);
    int S[3] = {rec_sx(r), rec_sy(r), rec_sz(r)};
    S[d >> 1] += (d & 1) ? -1 : 1;
    const uint32_t slot = D.spslot[kp];
    const uint32_t mask = (fl >> 8) & 63u;
    // The grain row for the children's positions, loaded before the atomics.
    SiteFrame F{};
    if (mask) F = site_frame(load_grow(D.gtab + (size_t)gs * GT_STRIDE), S[0], S[1], S[2]);
    if (slot != NIL) {
      const uint32_t b = site_bit(S[0], S[1], S[2]);
      atomicAnd(D.cbits + (size_t)slot * 24 + CB_NOW + (b >> 6), ~(1ull << (b & 63)));
    }
    if (!mask) continue;
    const float sc = rec_s(r) - D.lambda0;
    for (int dd = 0; dd < 6; ++dd) {
      if (!(mask & (1u << dd))) continue;
      const float4 xc = placed4(D, frame_pos(F, dd, sc), gs);
      const C3 c = cell_of(D, p3_of(xc));
      const uint32_t ci = cell_index(D, c.x, c.y, c.z);
      // The cell start and the brick's grain range are read before the rank
      // atomic: a wave's memory operations retire in order, so a load issued
      // after it would wait for its round trip.
      uint32_t* range = &D.bmeta[ci / (uint32_t)BRICK_CELLS].y;
      const uint32_t cs = D.cstart[ci], rlo = range[0], rhi = range[1];
      const uint32_t rank = atomicSub(&D.ccnt[ci], 1u) - 1u;
      const uint32_t dst = cs + rank;
      if (dst < D.cap_p) {
        D.B[dst] = make_rec(sc, gs, dd, S[0], S[1], S[2], ST_ACTIVE);
        D.P[dst] = xc;
        if (D.tagA) D.tagB[dst] = NIL;
      }
      note_grain_seen(range, rlo, rhi, grain_of(xc));
    }
  }
}

// One wave per occupied brick.  The brick is "dirty" when it holds
// particles of several grains or one of its 27 neighbourhood bricks (itself
// included) holds a particle of another grain, active this step or stopped.
// A particle's contact stencil lies inside the 3x3x3 cells around its cell,
// so it can meet another grain only if those cells reach a flagged brick:
// every cell of a brick flagged itself, and otherwise the cells on the faces,
// edges and corners that border a flagged neighbour.  Dirty bricks get the
// owner words of their cells (read by the containment of their neighbours);
// the particles of the cells that need the test go to one contiguous stretch
// of the global list `dpart` per block.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_dirty(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t epoch = step_epoch(D);
  if (dead(D)) return;
  __shared__ uint32_t s_n, s_np, s_base;
  if (threadIdx.x == 0) {
    s_n = 0;
    s_np = 0;
  }
  __syncthreads();
  const uint32_t nocc = D.cnt->n_occ;
  const Chunk ch = chunk_of(V, nocc, TPB / 64);
  const int lane = lane_id();
  const int nbx = D.nb[0], nby = D.nb[1], nbz = D.nb[2];
  // Neighbour bricks the 3x3x3 cells around this lane's cell reach: bit
  // (ox + 1) + 3 (oy + 1) + 9 (oz + 1).
  const int lx = lane & 3, ly = (lane >> 2) & 3, lz = lane >> 4;
  uint32_t reach = 0;
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int ox = t % 3 - 1, oy = (t / 3) % 3 - 1, oz = t / 9 - 1;
    const bool rx = ox == 0 || (ox < 0 ? lx == 0 : lx == 3);
    const bool ry = oy == 0 || (oy < 0 ? ly == 0 : ly == 3);
    const bool rz = oz == 0 || (oz < 0 ? lz == 0 : lz == 3);
    if (rx && ry && rz) reach |= 1u << t;
  }
  // Summary of one neighbour brick per lane (lanes < 27; lane 13 is the
  // brick itself): {step stamp, owner range of the step's active particles,
  // stopped owner word}, one 16-byte load.
  auto fetch = [&](uint32_t b, uint4& n) {
    n = make_uint4(0u, 0u, 0u, NIL);
    if (lane < 27) {
      const int bx = (int)(b % (uint32_t)nbx) + lane % 3 - 1;
      const int by = (int)((b / (uint32_t)nbx) % (uint32_t)nby) + (lane / 3) % 3 - 1;
      const int bz = (int)(b / ((uint32_t)nbx * (uint32_t)nby)) + lane / 9 - 1;
      if (bx >= 0 && by >= 0 && bz >= 0 && bx < nbx && by < nby && bz < nbz) {
        const uint32_t nb = ((uint32_t)bz * (uint32_t)nby + (uint32_t)by) * (uint32_t)nbx + (uint32_t)bx;
        n = D.bmeta[nb];
      }
    }
  };
  // Software pipeline: the words of the next brick of the wave are loaded
  // during this one, and its index one brick earlier.
  const uint32_t W = TPB / 64;
  const uint32_t k0 = ch.begin + (threadIdx.x >> 6);
  uint32_t b1 = k0 < ch.end ? D.occ[k0] : 0u;
  uint32_t b2 = k0 + W < ch.end ? D.occ[k0 + W] : 0u;
  uint2 own1 = make_uint2(0u, 0u);
  uint4 n1 = make_uint4(0u, 0u, 0u, NIL);
  if (k0 < ch.end) {
    own1 = D.binfo[b1];
    fetch(b1, n1);
  }
  // The stores of a brick are issued in the next iteration, once its loads
  // are on their way: a wave's memory operations retire in order, and stores
  // at the end of an iteration would be waited for before the next one.
  uint32_t pb = NIL;         // brick with stores pending (the same in every lane)
  uint32_t pbown = 0u;       // its owner word
  bool pcells = false;       // its cell owner words are pending (a dirty brick)
  uint32_t powner = 0u;      // this lane's cell owner word
  bool plist = false;        // its list entry is pending (lane 0)
  uint32_t pslot = 0u, poff = 0u;
  unsigned long long pmask = 0ull;
  auto flush = [&]() {
    if (pb == NIL) return;
    if (lane == 0) D.bown[pb] = make_uint2(epoch, pbown);
    if (pcells) D.cown[pb * (uint32_t)BRICK_CELLS + (uint32_t)lane].x = powner;
    if (plist) {
      D.dlist[ch.begin + pslot] = pb;
      D.dmask[ch.begin + pslot] = pmask;
      D.doff[ch.begin + pslot] = poff;
    }
    pb = NIL;
  };
  for (uint32_t k = k0; k < ch.end; k += W) {
    const uint32_t b = b1;
    const uint2 own = own1;
    const uint4 nn = n1;
    if (k + W < ch.end) {
      b1 = b2;
      own1 = D.binfo[b1];
      fetch(b1, n1);
    }
    if (k + 2u * W < ch.end) b2 = D.occ[k + 2u * W];
    // The brick's own owner range (lane 13).
    const uint32_t g = (uint32_t)__shfl((int)nn.y, 13);
    const uint32_t gmax = (uint32_t)__shfl((int)nn.z, 13);
    flush();
    const bool foreign = (nn.x == epoch && !(nn.y == g && nn.z == g)) ||
                         (nn.w != NIL && nn.w != g);
    // Flagged bricks; the brick itself (bit 13) when it holds several grains
    // or lies on a periodic face (its cells' stencils wrap, and owner words
    // do not tell the periods apart).
    bool face = false;
    if (D.periodic) {
      const int cx = (int)(b % (uint32_t)nbx), cy = (int)((b / (uint32_t)nbx) % (uint32_t)nby),
                cz = (int)(b / ((uint32_t)nbx * (uint32_t)nby));
      face = ((D.periodic & 1) && (cx == 0 || cx == nbx - 1)) ||
             ((D.periodic & 2) && (cy == 0 || cy == nby - 1)) ||
             ((D.periodic & 4) && (cz == 0 || cz == nbz - 1));
    }
    const uint32_t flags =
        (uint32_t)__ballot(foreign) | (g != gmax || face ? (1u << 13) : 0u);
    const bool dirty = flags != 0u;
    pb = b;
    pbown = dirty ? BOWN_CELLS : g;
    pcells = false;
    plist = false;
    if (!dirty) continue;
    // Owner grain of the active particles of each of the brick's 64 cells
    // (one lane per cell): the brick's one grain, unless it holds several.
    const uint32_t ci = b * (uint32_t)BRICK_CELLS + (uint32_t)lane;
    const uint32_t st = D.cstart[ci];
    const uint32_t en = lane + 1 < BRICK_CELLS ? D.cstart[ci + 1] : own.x + own.y;
    // Four independent loads per round (the tail round repeats the last
    // particle, which leaves the owner unchanged).
    uint32_t owner = g == gmax && en > st ? g : NIL;
    for (uint32_t j = st; g != gmax && j < en; j += 4u) {
      const uint32_t l = en - 1u;
      const uint32_t g0 = grain_of(D.P[j]), g1 = grain_of(D.P[min(j + 1u, l)]);
      const uint32_t g2 = grain_of(D.P[min(j + 2u, l)]), g3 = grain_of(D.P[min(j + 3u, l)]);
      owner = owner_merge(owner_merge(owner_merge(owner_merge(owner, g0), g1), g2), g3);
    }
    pcells = true;
    powner = owner;
    const bool need = (flags & (1u << 13)) != 0u || (flags & reach) != 0u;
    const uint32_t cnt = need ? en - st : 0u;
    const unsigned long long mask = __ballot(cnt > 0u);
    if (!mask) continue;
    uint32_t tot;
    (void)wave_excl_scan(cnt, tot);
    if (lane == 0) {
      plist = true;
      pslot = atomicAdd(&s_n, 1u);
      pmask = mask;
      poff = atomicAdd(&s_np, tot);
    }
  }
  flush();
  __syncthreads();
  if (threadIdx.x == 0) s_base = s_np ? atomicAdd(&D.cnt->n_dpart, s_np) : 0u;
  __syncthreads();
  const uint32_t nd = s_n, base = s_base;
  // The next dirty brick's list entry is loaded during this one.
  uint32_t k = threadIdx.x >> 6;
  uint32_t nb = 0, noff = 0;
  unsigned long long nmask = 0;
  if (k < nd) {
    nb = D.dlist[ch.begin + k];
    nmask = D.dmask[ch.begin + k];
    noff = D.doff[ch.begin + k];
  }
  for (; k < nd; k += TPB / 64) {
    const uint32_t b = nb, off = noff;
    const unsigned long long mask = nmask;
    if (k + TPB / 64 < nd) {
      nb = D.dlist[ch.begin + k + TPB / 64];
      nmask = D.dmask[ch.begin + k + TPB / 64];
      noff = D.doff[ch.begin + k + TPB / 64];
    }
    const uint32_t ci = b * (uint32_t)BRICK_CELLS + (uint32_t)lane;
    uint32_t st = 0, cnt = 0;
    if ((mask >> lane) & 1ull) {
      const uint2 inf = D.binfo[b];
      st = D.cstart[ci];
      const uint32_t en = lane + 1 < BRICK_CELLS ? D.cstart[ci + 1] : inf.x + inf.y;
      cnt = en - st;
    }
    uint32_t tot;
    const uint32_t ex = wave_excl_scan(cnt, tot);
    for (uint32_t j = 0; j < cnt; ++j) D.dpart[base + off + ex + j] = st + j;
  }
}

// ---------------------------------------------------------- containment ---
// Contact of a particle at p with owner word g and a candidate q (position,
// owner word).  Without periodic axes: another grain within rc.  With them:
// the nearest images within rc, and another grain or the same grain through
// a non-zero period shift (the candidate's period index minus the
// particle's, plus the shift to the nearest image).  g = NIL: any particle.
__device__ __forceinline__ bool meets_periodic(const Dev& D, float4 q, P3 p, uint32_t g,
                                               float rc2) {
  const uint32_t h = grain_of(q);
  float dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
  int shift = 0;
  if (D.periodic & 1) {
    const float k = rintf(dx * D.invL[0]);
    dx = fmaf(-k, D.L[0], dx);
    shift |= (int)k + owner_image(g, 0) - owner_image(h, 0);
  }
  if (D.periodic & 2) {
    const float k = rintf(dy * D.invL[1]);
    dy = fmaf(-k, D.L[1], dy);
    shift |= (int)k + owner_image(g, 1) - owner_image(h, 1);
  }
  if (D.periodic & 4) {
    const float k = rintf(dz * D.invL[2]);
    dz = fmaf(-k, D.L[2], dz);
    shift |= (int)k + owner_image(g, 2) - owner_image(h, 2);
  }
  if (g != NIL && ((g ^ h) & GRAIN_MASK) == 0u && shift == 0) return false;
  return (dx * dx + dy * dy) + dz * dz < rc2;
}
template <bool PER>
__device__ __forceinline__ bool meets(const Dev& D, float4 q, P3 p, uint32_t g, float rc2) {
  if constexpr (PER) return meets_periodic(D, q, p, g, rc2);
  return grain_of(q) != g && dist2(p, p3_of(q)) < rc2;
}
__device__ __forceinline__ bool meets_any(const Dev& D, float4 q, P3 p, uint32_t g, float rc2) {
  return D.periodic ? meets_periodic(D, q, p, g, rc2) : meets<false>(D, q, p, g, rc2);
}

// True if a particle of a grain other than g (g = NIL: of any grain) lies
// within rc of p, among this step's active particles and the stopped ones.
// `tests` counts the candidate particles examined (diagnostics).
__device__ bool foreign_within(const Dev& D, uint32_t epoch, P3 p, uint32_t g, uint32_t& tests) {
  int x0, x1, y0, y1, z0, z1;
  stencil_axis(D, p.x, 0, x0, x1);
  stencil_axis(D, p.y, 1, y0, y1);
  stencil_axis(D, p.z, 2, z0, z1);
  for (int zs = z0; zs <= z1; ++zs)
    for (int ys = y0; ys <= y1; ++ys)
      for (int xs = x0; xs <= x1; ++xs) {
        const int x = wrap_cell(xs, D.n[0]), y = wrap_cell(ys, D.n[1]), z = wrap_cell(zs, D.n[2]);
        const bool cross = x != xs || y != ys || z != zs;
        const uint32_t b = brick_index(D, x, y, z);
        const uint32_t loc = local_index(x, y, z);
        const uint32_t ci = b * (uint32_t)BRICK_CELLS + loc;
        // Brick summaries: a source whose brick holds grain g only (or
        // nothing) cannot hold a foreign particle.
        const uint4 meta = D.bmeta[b];
        if (meta.x == epoch) {
          if (cross || !(meta.y == g && meta.z == g)) {
            const uint2 inf = D.binfo[b];
            const uint32_t st = D.cstart[ci];
            const uint32_t en =
                (loc + 1u < (uint32_t)BRICK_CELLS) ? D.cstart[ci + 1] : inf.x + inf.y;
            for (uint32_t j = st; j < en; ++j) {
              const float4 q = D.P[j];
              ++tests;
              if (meets_any(D, q, p, g, D.rc2)) return true;
            }
          }
        }
        if (meta.w != NIL && (cross || meta.w != g)) {
          const uint2 bs = D.bsinfo[b];
          if (bs.y > 0u) {
            const uint32_t st = D.sstart[ci];
            const uint32_t en =
                (loc + 1u < (uint32_t)BRICK_CELLS) ? D.sstart[ci + 1] : bs.x + bs.y;
            for (uint32_t j = st; j < en; ++j) {
              const float4 q = D.PS[j];
              ++tests;
              if (meets_any(D, q, p, g, D.rc2)) return true;
            }
          }
          for (uint32_t j = D.shead[ci]; j != NIL; j = D.snext[j]) {
            const float4 q = D.PS[j];
            ++tests;
            if (meets_any(D, q, p, g, D.rc2)) return true;
          }
        }
      }
  return false;
}

// Owner words of one cell for a particle of grain g: whether the cell holds
// active (this step) or stopped particles of another grain.  Two independent
// 8-byte loads: the brick word {step, grain of a single-grain brick or
// BOWN_CELLS} and the cell word {active owner, stopped owner}.  A brick not
// occupied this step holds no active particle.
struct CellOwners {
  uint32_t ci, b;
  bool act, stp;
};

// With periodic axes a stencil cell past a face wraps, and every particle
// there is a candidate: the owner word cannot tell a particle's own period
// from the next one.
// The brick word of the previous cell is reused when the cell lies in the
// same brick (the cells of a stencil mostly do): brick cb, its word cbw.
template <bool PER>
__device__ __forceinline__ CellOwners cell_owners(const Dev& D, uint32_t epoch, int x, int y,
                                                  int z, uint32_t g, uint32_t& cb, uint2& cbw) {
  bool cross = false;
  if constexpr (PER) {
    const int xw = wrap_cell(x, D.n[0]), yw = wrap_cell(y, D.n[1]), zw = wrap_cell(z, D.n[2]);
    cross = xw != x || yw != y || zw != z;
    x = xw;
    y = yw;
    z = zw;
  }
  CellOwners o;
  o.b = brick_index(D, x, y, z);
  o.ci = o.b * (uint32_t)BRICK_CELLS + local_index(x, y, z);
  if (o.b != cb) {
    cb = o.b;
    cbw = D.bown[o.b];
  }
  const uint2 bw = cbw;
  const uint2 cw = D.cown[o.ci];
  const uint32_t aown = bw.x != epoch ? NIL : (bw.y == BOWN_CELLS ? cw.x : bw.y);
  o.act = aown != NIL && (cross || aown != g);
  o.stp = cw.y != NIL && (cross || cw.y != g);
  return o;
}

// Candidates Q[st, en) in groups of four independent loads (the tail group
// repeats its last candidate, which does not change the outcome).
template <bool PER>
__device__ __forceinline__ bool scan_range(const Dev& D, const float4* __restrict__ Q, uint32_t st,
                                           uint32_t en, P3 p, uint32_t g, float rc2,
                                           uint32_t& tests) {
  for (uint32_t j = st; j < en; j += 4u) {
    const uint32_t l = en - 1u;
    const float4 q0 = Q[j];
    const float4 q1 = Q[min(j + 1u, l)];
    const float4 q2 = Q[min(j + 2u, l)];
    const float4 q3 = Q[min(j + 3u, l)];
    tests += min(en - j, 4u);
    const int m = (int)meets<PER>(D, q0, p, g, rc2) | (int)meets<PER>(D, q1, p, g, rc2) |
                  (int)meets<PER>(D, q2, p, g, rc2) | (int)meets<PER>(D, q3, p, g, rc2);
    if (m) return true;
  }
  return false;
}

// Candidate ranges of one cell: active particles [ast, aen), cell-sorted
// stopped particles [sst, sen), recent stops from list head hd.
struct CellRanges {
  uint32_t ast, aen, sst, sen, hd;
};

// The brick's end of the active store is read only for its last cell; its
// stopped-store word is reused from the previous cell of the same brick
// (brick sb, word sbw).
__device__ __forceinline__ CellRanges cell_ranges(const Dev& D, const CellOwners& o, uint32_t& sb,
                                                  uint2& sbw) {
  CellRanges r = {0u, 0u, 0u, 0u, NIL};
  const bool last = (o.ci & (uint32_t)(BRICK_CELLS - 1)) == (uint32_t)(BRICK_CELLS - 1);
  if (o.act) {
    r.ast = D.cstart[o.ci];
    if (last) {
      const uint2 inf = D.binfo[o.b];
      r.aen = inf.x + inf.y;
    } else {
      r.aen = D.cstart[o.ci + 1];
    }
  }
  if (o.stp) {
    if (o.b != sb) {
      sb = o.b;
      sbw = D.bsinfo[o.b];
    }
    const uint2 bs = sbw;
    const uint32_t t0 = D.sstart[o.ci];
    const uint32_t t1 = last ? 0u : D.sstart[o.ci + 1];
    const uint32_t hd = D.shead[o.ci];
    if (bs.y > 0u) {
      r.sst = t0;
      r.sen = last ? bs.x + bs.y : t1;
    }
    r.hd = hd;
  }
  return r;
}

template <bool PER>
__device__ __forceinline__ bool walk_recent(const Dev& D, uint32_t j, P3 p, uint32_t g,
                                            uint32_t& tests) {
  for (; j != NIL; j = D.snext[j]) {
    ++tests;
    if (meets<PER>(D, D.PS[j], p, g, D.rc2)) return true;
  }
  return false;
}

// ----------------------------------------------- wave-shared candidates ---
// The candidates of a particle are very uneven (from none to long cell lists),
// and a wave waits for its slowest lane.  The containment therefore lists,
// for the wave's 64 particles, every candidate source of every stencil cell
// that holds another grain (a range of the cell-sorted active store, a range
// of the cell-sorted stopped store, the head of a recent-stop list) in shared
// memory, and the lanes take the sources in turn, whichever particle they
// belong to.  Entry: {first index or list head, length, kind << 6 | lane of
// the particle}.
constexpr int CE_MAX = 384;  // entries per wave and round
constexpr uint32_t CE_ACTIVE = 0u, CE_STOPPED = 1u, CE_RECENT = 2u;

// Cell k of the stencil: S8 (2 x 2 x 2 cells, k < 8) or 3 x 3 x 3 (k < 27).
// False for a cell outside the clamped stencil (or the repeat of a clamped
// axis in the 2 x 2 x 2 case).
struct Stencil {
  int x0, x1, y0, y1, z0, z1;
};
template <bool S8>
__device__ __forceinline__ bool stencil_cell(const Stencil& s, int k, int& x, int& y, int& z) {
  if (S8) {
    x = (k & 1) ? s.x1 : s.x0;
    y = (k & 2) ? s.y1 : s.y0;
    z = (k & 4) ? s.z1 : s.z0;
    return !(((k & 1) && s.x1 == s.x0) || ((k & 2) && s.y1 == s.y0) || ((k & 4) && s.z1 == s.z0));
  }
  x = s.x0 + k % 3;
  y = s.y0 + (k / 3) % 3;
  z = s.z0 + k / 9;
  return x <= s.x1 && y <= s.y1 && z <= s.z1;
}

// For the 2 x 2 x 2 stencil: the particle's own cell and, per axis, its
// squared distance (in cells) to the neighbouring layer of the stencil.  A
// stencil cell whose box lies farther than rc from the particle holds no
// contact; the test keeps a margin of 0.01 cells (20 nm at 2 um cells),
// far above the FP32 rounding of cell coordinates and distances, so a
// skipped cell can never hold a particle that the distance test accepts.
struct Near {
  int c[3];
  float u[3];  // cell coordinates of the particle
  float d2[3];
  float lim2;
};
__device__ __forceinline__ Near near_of(const Dev& D, P3 p) {
  Near n;
  const float x[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float u = (x[a] - D.lo[a]) * D.inv_h;
    const float fl = floorf(u);
    n.u[a] = u;
    n.c[a] = (int)fminf(fmaxf(fl, 0.0f), (float)(D.n[a] - 1));
    const float f = u - fl;
    const float d = f >= 0.5f ? 1.0f - f : f;
    n.d2[a] = d * d;
  }
  const float lim = sqrtf(D.rc2) * D.inv_h + 0.01f;
  n.lim2 = lim * lim;
  return n;
}
// The stopped particles of stencil cell (x, y, z), within the slabs of
// mask m, all lie farther than rc from the particle (same margin).
__device__ __forceinline__ bool slabs_far(const Near& n, uint32_t m, int x, int y, int z) {
  const int cc[3] = {x, y, z};
  float d2 = 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t s = (m >> (8 * a)) & 0xFFu;
    if (!s) return false;
    const float lo = (float)cc[a] + 0.125f * (float)(__ffs((int)s) - 1);
    const float hi = (float)cc[a] + 0.125f * (float)(32 - __clz((int)s));
    const float d = fmaxf(fmaxf(lo - n.u[a], n.u[a] - hi), 0.0f);
    d2 += d * d;
  }
  return d2 > n.lim2;
}
__device__ __forceinline__ bool near_skips(const Near& n, int x, int y, int z) {
  const float d2 = (x != n.c[0] ? n.d2[0] : 0.0f) + (y != n.c[1] ? n.d2[1] : 0.0f) +
                   (z != n.c[2] ? n.d2[2] : 0.0f);
  return d2 > n.lim2;
}

// Foreign-owner bits of the stencil cells (bit k: cell k holds active,
// resp. stopped particles of another grain).  Owner words are loaded one
// z-layer of the stencil at a time, all cells of a layer together.  With
// the 2 x 2 x 2 stencil, cells out of reach (near_skips) are left out, and
// so are stopped particles whose slabs in their cell lie out of reach
// (slabs_far).  Both take the stencil cells unwrapped: on a periodic axis
// a cell past a face is the image of the cell it wraps to, at the distance
// of that image, and with r_c <= h/2 only the images through the stencil's
// own side can come within r_c.
template <bool S8, bool PER>
__device__ __forceinline__ void stencil_owners(const Dev& D, uint32_t epoch, const Stencil& st,
                                               const Near& nr, uint32_t g, uint32_t& act,
                                               uint32_t& stp) {
  constexpr int NL = S8 ? 2 : 3, PL = S8 ? 4 : 9;
  act = 0u;
  stp = 0u;
  uint32_t cb = NIL;
  uint2 cbw = make_uint2(0u, 0u);
  for (int l = 0; l < NL; ++l) {
#pragma unroll
    for (int u = 0; u < PL; ++u) {
      const int k = l * PL + u;
      int x, y, z;
      if (!stencil_cell<S8>(st, k, x, y, z)) continue;
      if (S8 && near_skips(nr, x, y, z)) continue;
      const CellOwners o = cell_owners<PER>(D, epoch, x, y, z, g, cb, cbw);
      bool ostp = o.stp;
      if (S8) {
        // The slab mask, loaded with the owner words: stopped particles out
        // of reach are no sources.
        const uint32_t m = D.smask[o.ci];
        ostp = ostp && !slabs_far(nr, m, x, y, z);
      }
      act |= (uint32_t)o.act << k;
      stp |= (uint32_t)ostp << k;
    }
  }
}

// Writes the entries of the cells with bits in act / stp to e[0 ..).
template <bool S8, bool PER>
__device__ __forceinline__ void stencil_entries(const Dev& D, const Stencil& st, uint32_t act,
                                                uint32_t stp, uint32_t lane, uint3* e) {
  uint32_t n = 0;
  uint32_t sb = NIL;
  uint2 sbw = make_uint2(0u, 0u);
  auto cell = [&](int k) {
    if (!(((act | stp) >> k) & 1u)) return;
    int x, y, z;
    (void)stencil_cell<S8>(st, k, x, y, z);
    if constexpr (PER) {
      x = wrap_cell(x, D.n[0]);
      y = wrap_cell(y, D.n[1]);
      z = wrap_cell(z, D.n[2]);
    }
    CellOwners o;
    o.b = brick_index(D, x, y, z);
    o.ci = o.b * (uint32_t)BRICK_CELLS + local_index(x, y, z);
    o.act = (act >> k) & 1u;
    o.stp = (stp >> k) & 1u;
    const CellRanges r = cell_ranges(D, o, sb, sbw);
    if (o.act) e[n++] = make_uint3(r.ast, r.aen - r.ast, (CE_ACTIVE << 6) | lane);
    if (o.stp) {
      e[n++] = make_uint3(r.sst, r.sen - r.sst, (CE_STOPPED << 6) | lane);
      e[n++] = make_uint3(r.hd, 0u, (CE_RECENT << 6) | lane);
    }
  };
  if constexpr (S8) {
#pragma unroll 4
    for (int k = 0; k < 8; ++k) cell(k);
  } else {
    for (int k = 0; k < 27; ++k) cell(k);
  }
}


constexpr uint32_t HIT_BUF = 64;  // stops held per wave before they are written out
struct ContainShared {
  uint32_t n, tests;
  float4 pos[TPB];
  uint32_t hit[TPB];
  uint3 ent[TPB / 64][CE_MAX];
  uint2 hbuf[TPB / 64][HIT_BUF];  // {position in the block's stop list, particle}
};

// Containment (particles of two grains that meet stop, Sec. 2.1.2; the
// neighbour search, Sec. 2.3) of the particles listed in dpart (those of the
// cells of dirty bricks that can reach another grain), 64 per wave: owner
// words of the stencil cells per particle, then the wave's candidate sources
// shared out among its lanes, in rounds of at most CE_MAX entries (a lane's
// sources stay in one round).  Hits go to the block's region of the stop
// list.
template <bool S8, bool PER>
__device__ __forceinline__ void contain_body(const Dev& D, const VGrid& V, uint32_t epoch,
                                             ContainShared& S) {
  if (threadIdx.x == 0) {
    S.n = 0;
    S.tests = 0;
  }
  __syncthreads();
  const uint32_t lb = logical_block(V);
  const uint32_t nd = D.cnt->n_dpart;
  const Chunk ch = chunk_of(V, nd, TPB);
  const uint32_t lane = (uint32_t)lane_id();
  const uint32_t w = threadIdx.x >> 6;
  uint3* ent = S.ent[w];
  uint2* hbuf = S.hbuf[w];
  uint32_t nbuf = 0;  // stops held in hbuf (the same in every lane)
  const float rc2 = D.rc2;
  uint32_t tests = 0;
  // The particle of the next group is fetched during this one (its list
  // entry two groups ahead), off the critical path.
  uint32_t i1 = 0, i2 = 0;
  float4 q1 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (ch.begin + threadIdx.x < ch.end) {
    i1 = D.dpart[ch.begin + threadIdx.x];
    q1 = D.P[i1];
  }
  if (ch.begin + TPB + threadIdx.x < ch.end) i2 = D.dpart[ch.begin + TPB + threadIdx.x];
  for (uint32_t k0 = ch.begin; k0 < ch.end; k0 += TPB) {
    const uint32_t k = k0 + threadIdx.x;
    const uint32_t i = i1;
    const float4 q = q1;
    if (k + TPB < ch.end) {
      i1 = i2;
      q1 = D.P[i1];
    }
    if (k + 2u * TPB < ch.end) i2 = D.dpart[k + 2u * TPB];
    uint32_t act = 0u, stp = 0u;
    Stencil st = {0, 0, 0, 0, 0, 0};
    if (k < ch.end) {
      S.pos[threadIdx.x] = q;
      const P3 p = p3_of(q);
      stencil_axis(D, p.x, 0, st.x0, st.x1);
      stencil_axis(D, p.y, 1, st.y0, st.y1);
      stencil_axis(D, p.z, 2, st.z0, st.z1);
      Near nr{};
      if (S8) nr = near_of(D, p);
      stencil_owners<S8, PER>(D, epoch, st, nr, grain_of(q), act, stp);
    }
    S.hit[threadIdx.x] = 0u;
    // Rounds: the lanes whose sources fit after those of the lanes before
    // them (at most 3 per stencil cell, so every round takes one lane at
    // least).  Entries, positions and hit flags are the wave's own, so the
    // rounds order LDS within the wave only and the block's waves run
    // independently.
    uint32_t ne = (uint32_t)__popc(act) + 2u * (uint32_t)__popc(stp);
    for (;;) {
      uint32_t tot;
      const uint32_t e0 = wave_excl_scan(ne, tot);
      const bool take = ne > 0u && e0 + ne <= (uint32_t)CE_MAX;
      uint32_t used;
      (void)wave_excl_scan(take ? ne : 0u, used);
      if (take) {
        stencil_entries<S8, PER>(D, st, act, stp, lane, ent + e0);
        ne = 0u;
      }
      wave_lds_sync();
      for (uint32_t t = lane; t < used; t += 64u) {
        const uint3 en = ent[t];
        const uint32_t L = w * 64u + (en.z & 63u);
        if (S.hit[L]) continue;
        const float4 pq = S.pos[L];
        const uint32_t kind = en.z >> 6;
        bool h;
        if (kind == CE_RECENT)
          h = walk_recent<PER>(D, en.x, p3_of(pq), grain_of(pq), tests);
        else
          h = scan_range<PER>(D, kind == CE_ACTIVE ? D.P : D.PS, en.x, en.x + en.y, p3_of(pq),
                              grain_of(pq), rc2, tests);
        if (h) S.hit[L] = 1u;
      }
      wave_lds_sync();
      if (!__any(ne > 0u)) break;
    }
    // Stops are held in LDS and written out a few groups at a time: a wave's
    // memory operations retire in order, so a store here would hold back the
    // first loads of the next group.
    const bool hit = k < ch.end && S.hit[threadIdx.x] != 0u;
    const unsigned long long m = __ballot(hit);
    if (m) {
      const uint32_t c = (uint32_t)__popcll(m);
      if (nbuf + c > HIT_BUF) {
        wave_lds_sync();
        for (uint32_t t = lane; t < nbuf; t += 64u) D.newstop[ch.begin + hbuf[t].x] = hbuf[t].y;
        wave_lds_sync();
        nbuf = 0;
      }
      const int leader = __ffsll((long long)m) - 1;
      uint32_t wb = 0;
      if ((int)lane == leader) wb = atomicAdd(&S.n, c);
      wb = __shfl(wb, leader);
      const uint32_t r = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (hit) hbuf[nbuf + r] = make_uint2(wb + r, i);
      nbuf += c;
    }
  }
  wave_lds_sync();
  for (uint32_t t = lane; t < nbuf; t += 64u) D.newstop[ch.begin + hbuf[t].x] = hbuf[t].y;
  // Pair tests: one shared-memory add per wave, one global add per block.
  uint32_t wtests;
  (void)wave_excl_scan(tests, wtests);
  if (lane == 0u && wtests) atomicAdd(&S.tests, wtests);
  __syncthreads();
  if (threadIdx.x == 0) {
    D.newstop_cnt[lb] = S.n;
    if (S.tests) atomicAdd(&D.cnt->pair_tests, (unsigned long long)S.tests);
    if (lb == 0) atomicAdd(&D.cnt->dirty_tests, (unsigned long long)nd);
  }
}

// PM: 0 without periodic axes, 1 with them, 2 as each context has them (a
// batched launch); separate instantiations keep the plain case free of the
// periodic code.
template <class Bind, int PM>
__global__ __launch_bounds__(TPB, 6) void k_contain(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t epoch = step_epoch(D);
  if (dead(D)) return;
  __shared__ ContainShared S;
  const bool per = PM == 1 || (PM == 2 && D.periodic != 0);
  if constexpr (PM != 1) {
    if (!per) {
      if (D.stencil8) contain_body<true, false>(D, V, epoch, S);
      else contain_body<false, false>(D, V, epoch, S);
      return;
    }
  }
  if constexpr (PM != 0) {
    if (D.stencil8) contain_body<true, true>(D, V, epoch, S);
    else contain_body<false, true>(D, V, epoch, S);
  }
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_stoplink(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  __shared__ uint32_t s_base;
  const uint32_t n = D.cnt->n_dpart, G = D.sched[TK_CONTAIN];
  const Chunk rr = regions_of(V, G);
  for (uint32_t rg = rr.begin; rg < rr.end; ++rg) {
    const uint32_t cnt = D.newstop_cnt[rg];
    if (cnt == 0u) continue;
    const uint32_t beg = chunk_at(n, TPB, G, rg).begin;
    __syncthreads();
    if (threadIdx.x == 0) {
      s_base = atomicAdd(&D.cnt->n_stopped, cnt);
      atomicAdd(&D.cnt->n_newstop, cnt);
    }
    __syncthreads();
    const uint32_t base = s_base;
    for (uint32_t k = threadIdx.x; k < cnt; k += TPB) {
      const uint32_t i = D.newstop[beg + k];
      const uint4 r = with_fl(D.B[i], ST_STOPPED);
      D.B[i] = r;
      stopped_put(D, base + k, r, D.P[i]);
      if (D.tagA) {
        const uint32_t tag = D.tagB[i];
        if (tag != NIL) {
          D.adj_nact[tag] = (int32_t)(D.cnt->step - D.adj_step0) + 1;
          D.adj_sfin[tag] = rec_s(r);
        }
      }
    }
  }
}

// ----------------------------------------------------------- nucleation ---
// Image k (0..26) of y: y shifted by one period or none along each periodic
// axis; false for a shift along an axis that is not periodic.
__device__ __forceinline__ bool image_of(const Dev& D, P3 y, int k, P3& out) {
  const int sx = k % 3 - 1, sy = (k / 3) % 3 - 1, sz = k / 9 - 1;
  if ((sx && !(D.periodic & 1)) || (sy && !(D.periodic & 2)) || (sz && !(D.periodic & 4)))
    return false;
  out = P3{fmaf((float)sx, D.L[0], y.x), fmaf((float)sy, D.L[1], y.y), fmaf((float)sz, D.L[2], y.z)};
  return true;
}

// Site position y (or, with periodic axes, one of its images) lies on a
// claimed or reached lattice site of grain g.
__device__ __forceinline__ bool covers_at(const Dev& D, uint32_t g, P3 y, float inv_l) {
  int l[3];
  lattice_round(D.gtab + (size_t)g * GT_STRIDE, inv_l, y, l);
  const int32_t* bb = D.gbox + (size_t)g * 6;
  if (l[0] < bb[0] || l[1] < bb[1] || l[2] < bb[2] || l[0] > bb[3] || l[1] > bb[4] || l[2] > bb[5])
    return false;
  return claim_test(D, g, l[0], l[1], l[2], M_CLAIMED | M_REACHED);
}
__device__ __forceinline__ bool covers(const Dev& D, uint32_t g, P3 y, float inv_l) {
  if (!D.periodic) return covers_at(D, g, y, inv_l);
  for (int k = 0; k < 27; ++k) {
    P3 yi;
    if (image_of(D, y, k, yi) && covers_at(D, g, yi, inv_l)) return true;
  }
  return false;
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_nuc_test(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t epoch = step_epoch(D);
  const float lin_c = lin_const(D);
  if (dead(D)) return;
  const uint32_t ng = D.cnt->n_grains;
  const float inv_l = 1.0f / D.lambda0;
  for (uint32_t i = V.b * TPB + threadIdx.x; i < D.n_sites; i += V.G * TPB) {
    if (D.sstate[i] != SITE_DORMANT) continue;
    const float* T = D.stab + (size_t)i * GT_STRIDE;
    const P3 y = {T[0], T[1], T[2]};
    const float dT = field_at(D, y, lin_c) - D.theta;
    if (!isfinite(dT)) {
      atomicOr(&D.cnt->err, ERR_NUMERIC);
      continue;
    }
    if (!(dT >= T[3])) continue;
    // With melting claims shrink, so an engulfed site is tested again every
    // step, first against the grain that covered it at its last test.
    const uint32_t hint = D.melting ? D.sgrain[i] : NIL;
    if (hint < ng && covers(D, hint, y, inv_l)) continue;
    bool claimed = false;
    uint32_t g = 0;
    for (; g < ng; ++g)
      if (g != hint && covers(D, g, y, inv_l)) {
        claimed = true;
        break;
      }
    if (claimed) {
      // Without melting claims never shrink: the site can never fire.
      if (!D.melting) D.sstate[i] = SITE_ENGULFED;
      else D.sgrain[i] = g;
      continue;
    }
    uint32_t tests = 0;
    if (foreign_within(D, epoch, y, NIL, tests)) continue;
    D.cand[i] = 1u;
    atomicAdd(&D.cnt->n_cand, 1u);
  }
}

// One block: candidates in site order; a candidate is blocked by a site fired
// earlier in the same step when it lies within rc of that site or rounds to
// that grain's origin site.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_nuc_fire(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  if (D.cnt->n_cand == 0u) return;
  __shared__ uint32_t list[TPB];
  __shared__ uint32_t wsum[TPB / 64];
  __shared__ uint32_t s_nlist, s_nfired, s_blocked;
  const uint32_t ng0 = D.cnt->n_grains;
  const uint32_t n_out = D.cnt->n_out;
  const float inv_l = 1.0f / D.lambda0;
  if (threadIdx.x == 0) s_nfired = 0;
  __syncthreads();
  for (uint32_t c0 = 0; c0 < D.n_sites; c0 += TPB) {
    const uint32_t i = c0 + threadIdx.x;
    uint32_t c = 0;
    if (i < D.n_sites) {
      c = D.cand[i];
      if (c) D.cand[i] = 0u;
    }
    uint32_t tot;
    const uint32_t pos = block_excl_scan(c, wsum, tot);
    if (c) list[pos] = i;
    if (threadIdx.x == 0) s_nlist = tot;
    __syncthreads();
    const uint32_t nl = s_nlist;
    for (uint32_t q = 0; q < nl; ++q) {
      const uint32_t si = list[q];
      const float* T = D.stab + (size_t)si * GT_STRIDE;
      const P3 y = {T[0], T[1], T[2]};
      if (threadIdx.x == 0) s_blocked = 0;
      __syncthreads();
      const uint32_t nf = s_nfired;
      for (uint32_t g = ng0 + threadIdx.x; g < ng0 + nf; g += TPB) {
        const float* G = D.gtab + (size_t)g * GT_STRIDE;
        const P3 cg = {G[0], G[1], G[2]};
        bool blocked = false;
        for (int k = 0; k < (D.periodic ? 27 : 1); ++k) {
          P3 yi = y;
          if (D.periodic && !image_of(D, y, k, yi)) continue;
          int l[3];
          lattice_round(G, inv_l, yi, l);
          blocked |= dist2(yi, cg) < D.rc2 || (l[0] == 0 && l[1] == 0 && l[2] == 0);
        }
        if (blocked) atomicOr(&s_blocked, 1u);
      }
      __syncthreads();
      if (threadIdx.x == 0 && s_blocked == 0u) {
        const uint32_t g = ng0 + nf;
        if (g >= D.cap_grains || (uint64_t)n_out + 6ull * (nf + 1) > (uint64_t)D.cap_p) {
          atomicOr(&D.cnt->err, ERR_CAPACITY);
        } else {
          float* Gd = D.gtab + (size_t)g * GT_STRIDE;
          for (int k = 0; k < GT_STRIDE; ++k) Gd[k] = T[k];
          Gd[3] = 0.0f;
          int32_t* bb = D.gbox + (size_t)g * 6;
          for (int k = 0; k < 6; ++k) bb[k] = 0;
          claim_or(D, g, 0, 0, 0, M_CLAIMED | M_REACHED);
          if (D.gcnt) deposit_site(D, T, 0, 0, 0);
          D.greach[g] = 1u;
          D.gdead[g] = 0u;
          D.gsite[g] = (int32_t)si;
          for (int d = 0; d < 6; ++d) {
            D.B[n_out + 6 * nf + d] = make_rec(0.0f, g, d, 0, 0, 0, ST_ACTIVE);
            if (D.tagA) D.tagB[n_out + 6 * nf + d] = NIL;
          }
          D.sstate[si] = SITE_FIRED;
          s_nfired = nf + 1;
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    D.cnt->n_fired = s_nfired;
    D.cnt->n_grains = ng0 + s_nfired;
    D.cnt->nucleated += s_nfired;
  }
}

template <class Bind>
__global__ void k_finish(Bind Bd, double dt) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  Counters* c = D.cnt;
  if (c->err & (ERR_CAPACITY | HOLD)) return;
  // The step's sorted output becomes the next step's input; the step ends.
  c->par ^= 1u;
  c->t = c->t + dt;
  c->step += 1ull;
  c->epoch += 1u;
  if (c->epoch == 0u) c->err |= ERR_CAPACITY;  // brick step stamps exhausted (2^32 steps)
  c->n_active = c->n_out + 6u * c->n_fired;
  c->n_live = c->n_out - c->n_newstop + 6u * c->n_fired;
  c->contained += c->n_newstop;
  c->n_newstop = 0;
  c->n_dpart = 0;
  c->n_cand = 0;
  c->n_fired = 0;
}

template <class Bind>
__global__ void k_reset_stats(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  Counters* c = D.cnt;
  c->advanced = 0;
  c->exited = 0;
  c->spawners = 0;
  c->children = 0;
  c->contained = 0;
  c->nucleated = 0;
  c->max_step = 0;
  c->pair_tests = 0;
  c->dirty_tests = 0;
  c->melted = 0;
  c->removed = 0;
  c->reactivated = 0;
  c->grains_melted = 0;
}

// ------------------------------------------------ stopped-store re-sort ---
// Counting sort of S[0, n_stopped) by cell into S2: counts, brick scan
// (mode 1), cell scan (mode 1), scatter.  Clears the recent-particle lists.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_srb_count(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || !resort_due(D)) return;
  const uint32_t n = min(D.cnt->n_stopped, D.cap_s);
  const uint32_t ns = D.cnt->n_sorted;
  const Chunk ch = chunk_of(V, n, TPB);
  for (uint32_t base = ch.begin; base < ch.end; base += TPB) {
    const uint32_t j = base + threadIdx.x;
    uint32_t ckey = NIL;
    if (j < ch.end) {
      // A record removed by melting (NaN position) is dropped; the list head
      // of its cell is cleared all the same.
      const float4 q = D.PS[j];
      const bool gone = isnan(q.x);
      const C3 c = cell_of(D, gone ? place(D, rec_pos(D, D.S[j])).p : p3_of(q));
      ckey = cell_index(D, c.x, c.y, c.z);
      if (j >= ns) D.shead[ckey] = NIL;
      if (gone) ckey = NIL;
    }
    const Run rc = wave_run(ckey);
    if (ckey != NIL && rc.off == 0) atomicAdd(&D.ccnt[ckey], (uint32_t)rc.len);
    const uint32_t bkey = ckey == NIL ? NIL : ckey / (uint32_t)BRICK_CELLS;
    const Run rb = wave_run(bkey);
    if (bkey != NIL && rb.off == 0) atomicAdd(&D.bcnt[bkey], (uint32_t)rb.len);
  }
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_srb_scatter(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || !resort_due(D)) return;
  const uint32_t n = min(D.cnt->n_stopped, D.cap_s);
  const Chunk ch = chunk_of(V, n, TPB);
  // The record comes with the position and the cell start before the rank
  // atomic: a wave's memory operations retire in order, so a load issued
  // after the atomic would wait for its round trip.
  for (uint32_t base = ch.begin; base < ch.end; base += TPB) {
    const uint32_t j = base + threadIdx.x;
    uint32_t ckey = NIL;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    if (j < ch.end) {
      q = D.PS[j];
      r = D.S[j];
      if (!isnan(q.x)) {
        const C3 c = cell_of(D, p3_of(q));
        ckey = cell_index(D, c.x, c.y, c.z);
      }
    }
    const uint32_t cs = ckey != NIL ? D.sstart[ckey] : 0u;
    const Run run = wave_run(ckey);
    uint32_t rbase = 0;
    if (ckey != NIL && run.off == 0) rbase = atomicSub(&D.ccnt[ckey], (uint32_t)run.len);
    rbase = __shfl(rbase, run.head);
    if (ckey != NIL) {
      const uint32_t dst = cs + rbase - (uint32_t)run.len + (uint32_t)run.off;
      if (dst < D.cap_s) {
        D.S2[dst] = r;
        D.PS2[dst] = q;
      }
    }
  }
}

template <class Bind>
__global__ void k_srb_finish(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if ((D.cnt->err & (ERR_CAPACITY | HOLD)) || !resort_due(D)) return;
  // The re-sorted copy (the records not removed by melting) becomes the
  // stopped store.
  D.cnt->n_sorted = D.cnt->n_resorted;
  D.cnt->n_stopped = D.cnt->n_resorted;
  D.cnt->spar ^= 1u;
}

// ------------------------------------------------------------- resample ---

// Rosenthal moving point source on a linear background, evaluated in FP64
// at every node and stored as FP32 undercooling.
// Grid-stride walk over the points of an n0 x n1 x n2 grid: the indices
// (i, j, k) of the point v are carried from one step to the next (the stride
// split the same way once), so that no step divides.
struct GridWalk {
  uint64_t n0, n1, s0, s1, s2, v, stride, i, j, k;
  __device__ GridWalk(uint64_t n0_, uint64_t n1_, uint64_t v0, uint64_t stride_)
      : n0(n0_), n1(n1_), v(v0), stride(stride_) {
    s0 = stride % n0;
    s1 = (stride / n0) % n1;
    s2 = stride / (n0 * n1);
    i = v % n0;
    j = (v / n0) % n1;
    k = v / (n0 * n1);
  }
  __device__ uint64_t next() {
    i += s0;
    const uint64_t ci = i >= n0 ? 1u : 0u;
    i -= ci * n0;
    j += s1 + ci;
    const uint64_t cj = j >= n1 ? 1u : 0u;
    j -= cj * n1;
    k += s2 + cj;
    v += stride;
    return v;
  }
};

template <class Bind>
__global__ __launch_bounds__(TPB) void k_resample(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const Rosenthal& a = D.ros;
  const double t = D.cnt->t;
  const uint64_t total = (uint64_t)D.fn[0] * D.fn[1] * D.fn[2];
  const double L = a.x_end - a.x_start;
  const double phase = fmod(a.U * t, 2.0 * L);
  double xs, sg;
  if (phase < L) {
    xs = a.x_start + phase;
    sg = 1.0;
  } else {
    xs = a.x_start + 2.0 * L - phase;
    sg = -1.0;
  }
  const double base_t = a.dT0 + a.rate * t;
  const double k2 = -a.U / (2.0 * a.alpha);
  const double qn = a.q / (2.0 * M_PI);
  GridWalk gw((uint64_t)D.fn[0], (uint64_t)D.fn[1], (uint64_t)V.b * TPB + threadIdx.x,
              (uint64_t)V.G * TPB);
  for (uint64_t v = gw.v; v < total; v = gw.next()) {
    const double X = a.o[0] + (double)gw.i * a.sp[0];
    const double Y = a.o[1] + (double)gw.j * a.sp[1];
    const double Z = a.o[2] + (double)gw.k * a.sp[2];
    const double xi = sg * (X - xs), dy = Y - a.ys, dz = Z - a.zs;
    double r = sqrt(xi * xi + dy * dy + dz * dz);
    if (r < a.r_min) r = a.r_min;
    const double rise = qn / r * exp(k2 * (xi + r));
    double dT = base_t + a.grad[0] * X + a.grad[1] * Y + a.grad[2] * Z - rise;
    if (dT < a.dT_min) dT = a.dT_min;
    D.fgrid[v] = (float)dT;
  }
}

// -------------------------------------------------------------- melting ---
// Melting by walk-back (Sec. 2.1.3), at the start of a step when enabled,
// with the field of the step (the undercooling dT = field - theta):
//   1. a reached site S of a grain with dT(x_S) < 0 melts: it is no longer
//      claimed or reached (k_melt_sites; the melted sites are marked in the
//      slot's this-step words, which are clear at the start of a step);
//   2. a particle whose departure site melted is removed, an active one's
//      target released (k_advance for active particles, k_melt_stopped for
//      stopped ones); departure sites are reached sites, so the test is
//      dT(x_D) < 0 with the same arithmetic as in 1;
//   3. walk-back: each melted site T whose first direction d (0..5) with
//      S = T - e_d a reached site of the grain gives an active particle at S
//      moving towards T (travel 0), and T is claimed as its target
//      (k_walkback);
//   4. a grain left without reached sites has melted entirely; its
//      nucleation site is dormant again (k_melt_grains).
// Work is confined by lower bounds of the field over boxes: a box whose
// bound is not negative holds no melting site.

// Least node value of each cell of a node grid.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_field_cellmin(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || !(D.fkind == F_GRID || D.fkind == F_ROSENTHAL)) return;
  const uint32_t cx = (uint32_t)D.fn[0] - 1u, cy = (uint32_t)D.fn[1] - 1u, cz = (uint32_t)D.fn[2] - 1u;
  const uint64_t total = (uint64_t)cx * cy * cz;
  const size_t sy = (size_t)D.fn[0], sz = (size_t)D.fn[0] * (size_t)D.fn[1];
  GridWalk gw(cx, cy, (uint64_t)V.b * TPB + threadIdx.x, (uint64_t)V.G * TPB);
  for (uint64_t v = gw.v; v < total; v = gw.next()) {
    const size_t b = gw.k * sz + gw.j * sy + gw.i;
    const float* g = D.fgrid;
    float m = fminf(fminf(g[b], g[b + 1]), fminf(g[b + sy], g[b + sy + 1]));
    m = fminf(m, fminf(fminf(g[b + sz], g[b + sz + 1]), fminf(g[b + sz + sy], g[b + sz + sy + 1])));
    D.fcmin[v] = m;
  }
}

// Least of the cell minima over each block of 4 x 4 x 4 cells (clipped at
// the grid's end).
template <class Bind>
__global__ __launch_bounds__(TPB) void k_field_coarsemin(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D) || !(D.fkind == F_GRID || D.fkind == F_ROSENTHAL)) return;
  const uint32_t cx = (uint32_t)D.fn[0] - 1u, cy = (uint32_t)D.fn[1] - 1u, cz = (uint32_t)D.fn[2] - 1u;
  const uint32_t kx = (cx + 3u) >> 2, ky = (cy + 3u) >> 2, kz = (cz + 3u) >> 2;
  const uint64_t total = (uint64_t)kx * ky * kz;
  for (uint64_t v = (uint64_t)V.b * TPB + threadIdx.x; v < total; v += (uint64_t)V.G * TPB) {
    const uint32_t i = (uint32_t)(v % kx), j = (uint32_t)((v / kx) % ky),
                   k = (uint32_t)(v / ((uint64_t)kx * ky));
    float m = INFINITY;
    for (uint32_t c = 4u * k; c < min(4u * k + 4u, cz); ++c)
      for (uint32_t b = 4u * j; b < min(4u * j + 4u, cy); ++b)
        for (uint32_t a = 4u * i; a < min(4u * i + 4u, cx); ++a)
          m = fminf(m, D.fcmin[((size_t)c * cy + b) * cx + a]);
    D.fcoarse[v] = m;
  }
}

// Box of world positions holding every site of a brick (sites 0..7 of each
// axis lie at most 4 lattice steps from site 3) or of one z layer of it
// (half_z = 0), padded by half a lattice step against the rounding of the
// site positions.
__device__ __forceinline__ void brick_box(const float* __restrict__ G, int bx, int by, int bz,
                                          int w, float half_z, P3& lo, P3& hi) {
  const P3 c = lattice_pos(G, bx * 8 + 3, by * 8 + 3, bz * 8 + w, 0, 0.0f);
  const float ex = 4.5f * (fabsf(G[13]) + fabsf(G[14])) + half_z * fabsf(G[15]);
  const float ey = 4.5f * (fabsf(G[16]) + fabsf(G[17])) + half_z * fabsf(G[18]);
  const float ez = 4.5f * (fabsf(G[19]) + fabsf(G[20])) + half_z * fabsf(G[21]);
  lo = P3{c.x - ex, c.y - ey, c.z - ez};
  hi = P3{c.x + ex, c.y + ey, c.z + ez};
}

// Occupied claim slots, from the list of their keys, in groups of 64 per
// wave: each lane bounds the field over the brick of its key; the bricks
// whose bound is negative are then taken one at a time by the whole wave, a
// z layer of 64 sites per pass, one site per lane (the bit of a site in its
// layer word is its lane).  The reached sites below zero undercooling melt;
// a slot with melted sites goes to the walk-back list.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_melt_sites(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  const float lin_c = lin_const(D);
  const int lane = lane_id();
  __shared__ uint32_t s_melted;
  if (threadIdx.x == 0) s_melted = 0;
  __syncthreads();
  uint32_t melted = 0;
  const uint64_t used = min((uint64_t)D.cnt->claim_used, D.cmask + 1);
  const uint64_t waves = (uint64_t)V.G * (TPB / 64);
  for (uint64_t base = ((uint64_t)V.b * (TPB / 64) + (threadIdx.x >> 6)) * 64; base < used;
       base += waves * 64) {
    bool cand = false;
    unsigned long long key = CLAIM_EMPTY;
    if (base + lane < used) {
      key = D.clist[base + lane];
      const float* G = D.gtab + (size_t)(key >> 36) * GT_STRIDE;
      P3 lo, hi;
      brick_box(G, (int)((key >> 24) & 0xFFFull) - 2048, (int)((key >> 12) & 0xFFFull) - 2048,
                (int)(key & 0xFFFull) - 2048, 3, 4.5f, lo, hi);
      cand = may_melt(D, lo, hi, lin_c);
    }
    unsigned long long todo = __ballot(cand);
    while (todo) {
      const int src = __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const unsigned long long key_c =
          ((unsigned long long)__shfl((uint32_t)(key >> 32), src) << 32) |
          (unsigned long long)__shfl((uint32_t)key, src);
      const int64_t found = claim_find(D, key_c);
      if (found < 0) continue;  // listed keys are in the hash: never taken
      const uint64_t slot = (uint64_t)found;
      const uint32_t g = (uint32_t)(key_c >> 36);
      const int bx = (int)((key_c >> 24) & 0xFFFull) - 2048;
      const int by = (int)((key_c >> 12) & 0xFFFull) - 2048;
      const int bz = (int)(key_c & 0xFFFull) - 2048;
      const float* G = D.gtab + (size_t)g * GT_STRIDE;
      unsigned long long* q = D.cbits + slot * 24;
      uint32_t n = 0;
      for (int w = 0; w < 8; ++w) {
        const unsigned long long rm = q[CB_REACHED + w];
        if (!rm) continue;
        P3 lo, hi;
        brick_box(G, bx, by, bz, w, 0.0f, lo, hi);
        if (!may_melt(D, lo, hi, lin_c)) continue;
        const int sx = bx * 8 + (lane & 7), sy = by * 8 + (lane >> 3), sz = bz * 8 + w;
        bool melt = false;
        if ((rm >> lane) & 1ull)
          melt = field_at(D, lattice_pos(G, sx, sy, sz, 0, 0.0f), lin_c) - D.theta < 0.0f;
        const unsigned long long mask = __ballot(melt);
        if (!mask) continue;
        if (lane == 0) {
          atomicAnd(q + CB_CLAIMED + w, ~mask);
          atomicAnd(q + CB_REACHED + w, ~mask);
          atomicOr(q + CB_NOW + w, mask);
        }
        n += (uint32_t)__popcll(mask);
        if (melt && D.gcnt) {
          const uint32_t cell = deposit_cell(D, G, sx, sy, sz);
          if (cell != NIL) atomicSub(&D.gcnt[cell], 1u);
        }
      }
      if (n && lane == 0) {
        atomicSub(&D.greach[g], n);
        melted += n;
        D.mslots[atomicAdd(&D.cnt->n_melt_slots, 1u)] = (uint32_t)slot;
      }
    }
  }
  if (melted) atomicAdd(&s_melted, melted);
  __syncthreads();
  if (threadIdx.x == 0 && s_melted) atomicAdd(&D.cnt->melted, (unsigned long long)s_melted);
}

// Reached bit of site (sx, sy, sz) of grain g: from the given slot's words
// when the site is in that slot's brick, else through the hash.
__device__ __forceinline__ bool reached_at(const Dev& D, uint32_t g, uint64_t own_key,
                                           const unsigned long long* own, int sx, int sy, int sz) {
  const uint64_t key = claim_key(g, sx, sy, sz);
  const unsigned long long* q = own;
  if (key != own_key) {
    const int64_t slot = claim_find(D, key);
    if (slot < 0) return false;
    q = D.cbits + (size_t)slot * 24;
  }
  const uint32_t b = site_bit(sx, sy, sz);
  return (load_relaxed(q + CB_REACHED + (b >> 6)) >> (b & 63)) & 1ull;
}

// One wave per listed slot, a z layer of 64 sites per pass, one site per
// lane: each site melted in this step is re-approached from its first
// reached neighbour; the slot's marks are cleared.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_walkback(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  const int lane = lane_id();
  __shared__ uint32_t s_new;
  if (threadIdx.x == 0) s_new = 0;
  __syncthreads();
  uint32_t made = 0;
  const uint32_t n = D.cnt->n_melt_slots;
  const uint32_t waves = V.G * (TPB / 64);
  for (uint32_t k = V.b * (TPB / 64) + (threadIdx.x >> 6); k < n; k += waves) {
    const uint64_t slot = D.mslots[k];
    const unsigned long long key = D.ckeys[slot];
    unsigned long long* q = D.cbits + slot * 24;
    const uint32_t g = (uint32_t)(key >> 36);
    const int bx = (int)((key >> 24) & 0xFFFull) - 2048;
    const int by = (int)((key >> 12) & 0xFFFull) - 2048;
    const int bz = (int)(key & 0xFFFull) - 2048;
    for (int w = 0; w < 8; ++w) {
      const unsigned long long mm = load_relaxed(q + CB_NOW + w);
      if (!mm) continue;
      bool claim = false;
      if ((mm >> lane) & 1ull) {
        const int T[3] = {bx * 8 + (lane & 7), by * 8 + (lane >> 3), bz * 8 + w};
        for (int d = 0; d < 6; ++d) {
          const int a = d >> 1, sg = (d & 1) ? -1 : 1;
          const int sx = T[0] - (a == 0 ? sg : 0), sy = T[1] - (a == 1 ? sg : 0),
                    sz = T[2] - (a == 2 ? sg : 0);
          if (!reached_at(D, g, key, q, sx, sy, sz)) continue;
          const uint32_t j = atomicAdd(&D.cnt->n_active, 1u);
          if (j >= D.cap_p) {
            // No room: the count is taken back (it bounds every reader of A).
            atomicSub(&D.cnt->n_active, 1u);
            atomicOr(&D.cnt->err, ERR_CAPACITY);
          } else {
            D.A[j] = make_rec(0.0f, g, d, sx, sy, sz, ST_ACTIVE);
            if (D.tagA) D.tagA[j] = NIL;
            atomicAdd(&D.cnt->n_live, 1u);
            claim = true;
            made += 1;
          }
          break;
        }
      }
      const unsigned long long cm = __ballot(claim);
      if (lane == 0) {
        if (cm) atomicOr(q + CB_CLAIMED + w, cm);
        atomicAnd(q + CB_NOW + w, ~mm);
      }
    }
  }
  if (made) atomicAdd(&s_new, made);
  __syncthreads();
  if (threadIdx.x == 0 && s_new) atomicAdd(&D.cnt->reactivated, (unsigned long long)s_new);
}

// Grains left without reached sites have melted entirely: their nucleation
// sites are dormant again.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_melt_grains(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  const uint32_t ng = D.cnt->n_grains;
  for (uint32_t g = V.b * TPB + threadIdx.x; g < ng; g += V.G * TPB) {
    if (D.gdead[g] || D.greach[g] != 0u) continue;
    D.gdead[g] = 1u;
    atomicAdd(&D.cnt->grains_melted, 1ull);
    const int32_t si = D.gsite[g];
    if (si >= 0) D.sstate[si] = SITE_DORMANT;
  }
  if (V.b == 0 && threadIdx.x == 0) D.cnt->n_melt_slots = 0;
}

// Stopped particles whose departure site melted are removed: the record is
// retired and its position made NaN, so that no test meets it; the re-sort
// drops it.  The cell-sorted prefix of the store is taken brick by brick:
// lanes bound the field over their bricks (padded by the reach of a stopped
// particle from its departure site, under 2 lambda0; bricks on the faces of
// the grid, which also hold the particles beyond it, reach out without
// limit), and the records of the bricks whose bound is negative are tested
// by the whole wave; the unsorted tail is tested record by record.
__device__ __forceinline__ uint32_t melt_stopped_rec(const Dev& D, uint32_t j, float lin_c) {
  const uint4 r = D.S[j];
  if ((rec_fl(r) & 3u) == ST_RETIRED) return 0u;
  const float* G = D.gtab + (size_t)rec_grain(r) * GT_STRIDE;
  if (!departure_melted(D, G, rec_sx(r), rec_sy(r), rec_sz(r), lin_c)) return 0u;
  D.S[j] = with_fl(r, ST_RETIRED);
  const float nan = __uint_as_float(0x7FC00000u);
  D.PS[j] = make_float4(nan, nan, nan, __uint_as_float(rec_grain(r)));
  return 1u;
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_melt_stopped(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (dead(D)) return;
  const float lin_c = lin_const(D);
  const int lane = lane_id();
  __shared__ uint32_t s_rm;
  if (threadIdx.x == 0) s_rm = 0;
  __syncthreads();
  uint32_t rm = 0;
  const uint32_t n = min(D.cnt->n_stopped, D.cap_s);
  const uint32_t ns = min(D.cnt->n_sorted, n);
  const uint32_t nb = D.n_bricks;
  const float h = 1.0f / D.inv_h;
  const float pad = 2.01f * D.lambda0 + 0.01f * h;
  constexpr float FAR = 1e30f;
  const uint64_t waves = (uint64_t)V.G * (TPB / 64);
  for (uint64_t base = ((uint64_t)V.b * (TPB / 64) + (threadIdx.x >> 6)) * 64; base < nb;
       base += waves * 64) {
    bool cand = false;
    uint2 bs = make_uint2(0u, 0u);
    if (base + lane < nb) {
      const uint32_t b = (uint32_t)(base + lane);
      bs = D.bsinfo[b];
      if (bs.y && bs.x < ns) {
        const int i[3] = {(int)(b % (uint32_t)D.nb[0]),
                          (int)((b / (uint32_t)D.nb[0]) % (uint32_t)D.nb[1]),
                          (int)(b / ((uint32_t)D.nb[0] * (uint32_t)D.nb[1]))};
        float l[3], u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          // Cells clamp positions beyond the grid into its outer cells.
          l[a] = i[a] == 0 ? -FAR : D.lo[a] + (float)(4 * i[a]) * h - pad;
          u[a] = 4 * i[a] + 4 >= D.n[a] ? FAR : D.lo[a] + (float)(4 * i[a] + 4) * h + pad;
        }
        cand = may_melt(D, P3{l[0], l[1], l[2]}, P3{u[0], u[1], u[2]}, lin_c);
      }
    }
    unsigned long long todo = __ballot(cand);
    while (todo) {
      const int src = __ffsll((long long)todo) - 1;
      todo &= todo - 1ull;
      const uint32_t start = __shfl(bs.x, src);
      const uint32_t end = min(start + __shfl(bs.y, src), ns);
      for (uint32_t j = start + (uint32_t)lane; j < end; j += 64u) rm += melt_stopped_rec(D, j, lin_c);
    }
  }
  for (uint32_t j = ns + V.b * TPB + threadIdx.x; j < n; j += V.G * TPB) rm += melt_stopped_rec(D, j, lin_c);
  if (rm) atomicAdd(&s_rm, rm);
  __syncthreads();
  if (threadIdx.x == 0 && s_rm) atomicAdd(&D.cnt->removed, (unsigned long long)s_rm);
}

// Reached sites of every grain from the claim hash; grains with none are
// marked melted, and with melting on every engulfed site is tested again.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_count_reached(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint64_t slots = D.cmask + 1;
  for (uint64_t v = (uint64_t)V.b * TPB + threadIdx.x; v < slots; v += (uint64_t)V.G * TPB) {
    const unsigned long long key = D.ckeys[v];
    if (key == CLAIM_EMPTY) continue;
    uint32_t n = 0;
    for (int w = 0; w < 8; ++w) n += (uint32_t)__popcll(D.cbits[v * 24 + CB_REACHED + w]);
    if (n) atomicAdd(&D.greach[(uint32_t)(key >> 36)], n);
  }
}
template <class Bind>
__global__ __launch_bounds__(TPB) void k_count_finish(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t ng = D.cnt->n_grains;
  for (uint32_t g = V.b * TPB + threadIdx.x; g < ng; g += V.G * TPB) D.gdead[g] = D.greach[g] == 0u;
  if (D.melting)
    for (uint32_t i = V.b * TPB + threadIdx.x; i < D.n_sites; i += V.G * TPB)
      if (D.sstate[i] == SITE_ENGULFED) D.sstate[i] = SITE_DORMANT;
}

// --------------------------------------------------------- init / load ----
// Empty brick summaries (no step stamp, no owner); the step stamps start
// at 1 (0 marks bricks never occupied).
template <class Bind>
__global__ __launch_bounds__(TPB) void k_fill_bmeta(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  if (V.b == 0 && threadIdx.x == 0) D.cnt->epoch = 1u;
  for (uint64_t b = (uint64_t)V.b * TPB + threadIdx.x; b < D.n_bricks;
       b += (uint64_t)V.G * TPB)
    D.bmeta[b] = make_uint4(0u, NIL, 0u, NIL);
}

// New records A[first, first+count): those marked stopped, and (with box
// exit, when exit_rule is set: new envelopes) those outside the box, move to
// the stopped store.  A loaded state keeps the states it was given.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_classify_new(Bind Bd, uint32_t first, uint32_t count,
                                                      int32_t exit_rule) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  for (uint32_t k0 = V.b * TPB; k0 < count; k0 += V.G * TPB) {
    const uint32_t k = k0 + threadIdx.x;
    bool out = false;
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    P3 x = {0.0f, 0.0f, 0.0f};
    const uint32_t i = first + k;
    if (k < count) {
      r = D.A[i];
      x = rec_pos(D, r);
      if ((rec_fl(r) & 3u) == ST_STOPPED) {
        out = true;
      } else if (D.box_exit && exit_rule) {
        out = !in_box(D, x);
      }
      if (out) {
        r = with_fl(r, ST_STOPPED);
        D.A[i] = r;
        atomicSub(&D.cnt->n_live, 1u);
      }
    }
    const uint32_t j = wave_append(out, &D.cnt->n_stopped);
    if (out) stopped_put(D, j, r, placed4(D, x, rec_grain(r)));
  }
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_claim_ball(Bind Bd, uint32_t g, int32_t r) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const int32_t w = 2 * r + 1;
  const uint64_t total = (uint64_t)w * w * w;
  for (uint64_t v = (uint64_t)V.b * TPB + threadIdx.x; v < total;
       v += (uint64_t)V.G * TPB) {
    const int x = (int)(v % w) - r;
    const int y = (int)((v / w) % w) - r;
    const int z = (int)(v / ((uint64_t)w * w)) - r;
    if (abs(x) + abs(y) + abs(z) <= r) {
      claim_or(D, g, x, y, z, M_CLAIMED | M_REACHED);
      atomicAdd(&D.greach[g], 1u);
      if (D.gcnt) deposit_site(D, D.gtab + (size_t)g * GT_STRIDE, x, y, z);
    }
  }
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_claim_list(Bind Bd, const int32_t* grain, const int32_t* site,
                                                    const uint8_t* flags, uint32_t n) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  for (uint32_t k = V.b * TPB + threadIdx.x; k < n; k += V.G * TPB) {
    const uint32_t g = (uint32_t)grain[k];
    const int x = site[3 * k], y = site[3 * k + 1], z = site[3 * k + 2];
    uint32_t m = 0;
    if (flags[k] & 1u) m |= M_CLAIMED;
    if (flags[k] & 2u) m |= M_REACHED;
    if (m) {
      claim_or(D, g, x, y, z, m);
      bbox_add(D, g, x, y, z);
    }
  }
}


// --------------------------------------------------------------- export ---
struct PartOut {
  float x, y, z, s;
  int32_t site[3];
  uint32_t grain;
  uint8_t dir, state;
  uint16_t pad;
  int32_t cell[3];
};
static_assert(sizeof(PartOut) == 48, "particle record layout");

__device__ __forceinline__ void put_particle(const Dev& D, uint4 r, uint32_t state, PartOut* o) {
  const P3 p = rec_pos(D, r);
  const C3 c = cell_of(D, place(D, p).p);
  PartOut v;
  v.x = p.x;
  v.y = p.y;
  v.z = p.z;
  v.s = rec_s(r);
  v.site[0] = rec_sx(r);
  v.site[1] = rec_sy(r);
  v.site[2] = rec_sz(r);
  v.grain = rec_grain(r);
  v.dir = (uint8_t)rec_dir(r);
  v.state = (uint8_t)state;
  v.pad = 0;
  v.cell[0] = c.x;
  v.cell[1] = c.y;
  v.cell[2] = c.z;
  *o = v;
}

struct Window {
  float lo[3], hi[3];
  int32_t on;
};

__device__ __forceinline__ bool in_window(const Window& w, P3 p) {
  return !w.on || (p.x >= w.lo[0] && p.x < w.hi[0] && p.y >= w.lo[1] && p.y < w.hi[1] &&
                   p.z >= w.lo[2] && p.z < w.hi[2]);
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_export_particles(Bind Bd, uint32_t* counter, PartOut* out,
                                                          uint32_t cap_out, Window win) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t na = D.cnt->n_active, ns = min(D.cnt->n_stopped, D.cap_s);
  for (uint32_t k0 = V.b * TPB; k0 < na + ns; k0 += V.G * TPB) {
    const uint32_t k = k0 + threadIdx.x;
    bool take = false;
    uint4 r = make_uint4(0u, 0u, 0u, 0u);
    uint32_t st = ST_ACTIVE;
    if (k < na) {
      r = D.A[k];
      take = (rec_fl(r) & 3u) == ST_ACTIVE;
    } else if (k < na + ns) {
      r = D.S[k - na];
      take = (rec_fl(r) & 3u) != ST_RETIRED;  // removed by melting
      st = ST_STOPPED;
    }
    if (take && win.on) take = in_window(win, place(D, rec_pos(D, r)).p);
    const uint32_t j = wave_append(take, counter);
    if (take && j < cap_out) put_particle(D, r, st, out + j);
  }
}

struct ClaimOut {
  uint32_t grain;
  int32_t site[3];
  uint32_t flags;
};
static_assert(sizeof(ClaimOut) == 20, "claim record layout");

template <class Bind>
__global__ __launch_bounds__(TPB) void k_export_claims(Bind Bd, uint32_t* counter, ClaimOut* out,
                                                       uint32_t cap_out, Window win) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint64_t slots = D.cmask + 1;
  for (uint64_t v = (uint64_t)V.b * TPB + threadIdx.x; v < slots * 8;
       v += (uint64_t)V.G * TPB) {
    const uint64_t slot = v >> 3;
    const uint32_t w = (uint32_t)(v & 7u);
    const unsigned long long key = D.ckeys[slot];
    if (key == CLAIM_EMPTY) continue;
    const unsigned long long cm = D.cbits[slot * 24 + CB_CLAIMED + w];
    const unsigned long long rm = D.cbits[slot * 24 + CB_REACHED + w];
    unsigned long long any = cm | rm;
    if (!any) continue;
    const uint32_t g = (uint32_t)(key >> 36);
    const int bx = (int)((key >> 24) & 0xFFFull) - 2048;
    const int by = (int)((key >> 12) & 0xFFFull) - 2048;
    const int bz = (int)(key & 0xFFFull) - 2048;
    if (win.on) {
      const float* G = D.gtab + (size_t)g * GT_STRIDE;
      unsigned long long keep = 0;
      unsigned long long m = any;
      while (m) {
        const int bit = __ffsll((long long)m) - 1;
        m &= m - 1ull;
        const P3 p = lattice_pos(G, bx * 8 + (bit & 7), by * 8 + ((bit >> 3) & 7), bz * 8 + (int)w,
                                 0, 0.0f);
        if (in_window(win, place(D, p).p)) keep |= 1ull << bit;
      }
      any = keep;
      if (!any) continue;
    }
    const uint32_t base = atomicAdd(counter, (uint32_t)__popcll(any));
    uint32_t k = 0;
    while (any) {
      const int bit = __ffsll((long long)any) - 1;
      any &= any - 1ull;
      const uint32_t j = base + k++;
      if (j >= cap_out) continue;
      ClaimOut o;
      o.grain = g;
      o.site[0] = bx * 8 + (bit & 7);
      o.site[1] = by * 8 + ((bit >> 3) & 7);
      o.site[2] = bz * 8 + (int)w;
      o.flags = (uint32_t)((cm >> bit) & 1ull) | ((uint32_t)((rm >> bit) & 1ull) << 1);
      out[j] = o;
    }
  }
}

// Claim bricks for a saved state: each occupied slot with a claimed or
// reached site as {grain, brick xyz, claimed[8], reached[8]} (144 bytes).
struct SlotOut {
  uint32_t grain;
  int32_t brick[3];
  unsigned long long claimed[8], reached[8];
};
static_assert(sizeof(SlotOut) == 144, "claim brick record layout");

template <class Bind>
__global__ __launch_bounds__(TPB) void k_export_slots(Bind Bd, uint32_t* counter, SlotOut* out,
                                                      uint32_t cap_out) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint64_t slots = D.cmask + 1;
  for (uint64_t k0 = (uint64_t)V.b * TPB; k0 < slots; k0 += (uint64_t)V.G * TPB) {
    const uint64_t slot = k0 + threadIdx.x;
    bool take = false;
    unsigned long long key = CLAIM_EMPTY;
    if (slot < slots) {
      key = D.ckeys[slot];
      if (key != CLAIM_EMPTY) {
        unsigned long long any = 0;
        for (int w = 0; w < 16; ++w) any |= D.cbits[slot * 24 + w];
        take = any != 0ull;
      }
    }
    const uint32_t j = wave_append(take, counter);
    if (!take || j >= cap_out) continue;
    SlotOut o;
    o.grain = (uint32_t)(key >> 36);
    o.brick[0] = (int)((key >> 24) & 0xFFFull) - 2048;
    o.brick[1] = (int)((key >> 12) & 0xFFFull) - 2048;
    o.brick[2] = (int)(key & 0xFFFull) - 2048;
    for (int w = 0; w < 8; ++w) {
      o.claimed[w] = D.cbits[slot * 24 + CB_CLAIMED + w];
      o.reached[w] = D.cbits[slot * 24 + CB_REACHED + w];
    }
    out[j] = o;
  }
}

// Claim bricks of a saved state into the claim hash, with the grains'
// bounding boxes grown to the occupied sites of each brick.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_claim_slots(Bind Bd, const SlotOut* in, uint32_t n) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  for (uint32_t k = V.b * TPB + threadIdx.x; k < n; k += V.G * TPB) {
    const SlotOut r = in[k];
    unsigned long long occ = 0;  // sites of the brick's 8 x 8 columns
    int z0 = 8, z1 = -1;
    for (int w = 0; w < 8; ++w) {
      const unsigned long long m = r.claimed[w] | r.reached[w];
      occ |= m;
      if (m) {
        z0 = min(z0, w);
        z1 = w;
      }
    }
    if (!occ) continue;
    const int sx = r.brick[0] * 8, sy = r.brick[1] * 8, sz = r.brick[2] * 8;
    const int64_t slot = claim_get(D, claim_key(r.grain, sx, sy, sz));
    if (slot < 0) continue;
    unsigned long long* w8 = D.cbits + (size_t)slot * 24;
    for (int w = 0; w < 8; ++w) {
      if (r.claimed[w]) atomicOr(w8 + CB_CLAIMED + w, r.claimed[w]);
      if (r.reached[w]) atomicOr(w8 + CB_REACHED + w, r.reached[w]);
    }
    // Occupied rows (y) and columns (x) of the brick.
    uint32_t rows = 0, cols = 0;
    for (int y = 0; y < 8; ++y) {
      const uint32_t b = (uint32_t)((occ >> (8 * y)) & 0xFFull);
      if (b) rows |= 1u << y;
      cols |= b;
    }
    const int lo[3] = {sx + __ffs(cols) - 1, sy + __ffs(rows) - 1, sz + z0};
    const int hi[3] = {sx + 31 - __clz(cols), sy + 31 - __clz(rows), sz + z1};
    bbox_add_box(D, r.grain, lo, hi);
  }
}

// Grain map: voxel centre y takes the grain whose reached site is y's rounded
// lattice position; nearest such site wins, then the lower grain.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_grain_map(Bind Bd, int32_t n0, int32_t n1, int32_t n2,
                                                   float o0, float o1, float o2, float s0, float s1,
                                                   float s2, uint32_t* out) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint64_t total = (uint64_t)n0 * n1 * n2;
  const uint32_t ng = D.cnt->n_grains;
  const float inv_l = 1.0f / D.lambda0;
  for (uint64_t v = (uint64_t)V.b * TPB + threadIdx.x; v < total;
       v += (uint64_t)V.G * TPB) {
    const uint64_t i = v % (uint64_t)n0, j = (v / (uint64_t)n0) % (uint64_t)n1,
                   k = v / ((uint64_t)n0 * n1);
    const P3 y = {o0 + ((float)i + 0.5f) * s0, o1 + ((float)j + 0.5f) * s1,
                  o2 + ((float)k + 0.5f) * s2};
    uint32_t best = 0;
    float bd = INFINITY;
    for (uint32_t g = 0; g < ng; ++g) {
      const float* G = D.gtab + (size_t)g * GT_STRIDE;
      // The voxel centre and, with periodic axes, its images.
      for (int k = 0; k < (D.periodic ? 27 : 1); ++k) {
        P3 yi = y;
        if (D.periodic && !image_of(D, y, k, yi)) continue;
        int l[3];
        lattice_round(G, inv_l, yi, l);
        const int32_t* bb = D.gbox + (size_t)g * 6;
        if (l[0] < bb[0] || l[1] < bb[1] || l[2] < bb[2] || l[0] > bb[3] || l[1] > bb[4] ||
            l[2] > bb[5])
          continue;
        if (!claim_test(D, g, l[0], l[1], l[2], M_REACHED)) continue;
        const P3 ps = lattice_pos(G, l[0], l[1], l[2], 0, 0.0f);
        const float d = dist2(yi, ps);
        if (d < bd) {
          bd = d;
          best = g + 1;
        }
      }
    }
    out[v] = best;
  }
}

// Node undercooling of a temperature-and-solute field (Sec. 3.4: the local
// undercooling is taken with respect to the liquidus of the local solute
// concentration), formed in FP64 and stored in FP32.
__global__ __launch_bounds__(TPB) void k_solute_nodes(const double* __restrict__ T,
                                                      const double* __restrict__ w, double liq_T,
                                                      double liq_m, uint64_t n,
                                                      float* __restrict__ out) {
  for (uint64_t k = (uint64_t)blockIdx.x * TPB + threadIdx.x; k < n;
       k += (uint64_t)gridDim.x * TPB)
    out[k] = (float)((liq_T + liq_m * w[k]) - T[k]);
}

// Deposition counts from the whole claim hash (every reached site), after
// the counts were cleared: one lane per (slot, z-layer) word.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_deposit_all(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint64_t slots = D.cmask + 1;
  for (uint64_t v = (uint64_t)V.b * TPB + threadIdx.x; v < slots * 8;
       v += (uint64_t)V.G * TPB) {
    const uint64_t slot = v >> 3;
    const uint32_t w = (uint32_t)(v & 7u);
    const unsigned long long key = D.ckeys[slot];
    if (key == CLAIM_EMPTY) continue;
    unsigned long long rm = D.cbits[slot * 24 + CB_REACHED + w];
    if (!rm) continue;
    const uint32_t g = (uint32_t)(key >> 36);
    const int bx = (int)((key >> 24) & 0xFFFull) - 2048;
    const int by = (int)((key >> 12) & 0xFFFull) - 2048;
    const int bz = (int)(key & 0xFFFull) - 2048;
    const float* G = D.gtab + (size_t)g * GT_STRIDE;
    while (rm) {
      const int bit = __ffsll((long long)rm) - 1;
      rm &= rm - 1ull;
      deposit_site(D, G, bx * 8 + (bit & 7), by * 8 + ((bit >> 3) & 7), bz * 8 + (int)w);
    }
  }
}

// Mushy-zone fraction of every deposition cell: min(1, count lambda0^3 / V).
__global__ __launch_bounds__(TPB) void k_mushy_fraction(const uint32_t* __restrict__ cnt,
                                                        uint64_t n, double site_over_cell,
                                                        float* __restrict__ out) {
  for (uint64_t k = (uint64_t)blockIdx.x * TPB + threadIdx.x; k < n;
       k += (uint64_t)gridDim.x * TPB)
    out[k] = (float)fmin(1.0, (double)cnt[k] * site_over_cell);
}

// ============================================================== adjoint ===
// Gradients of the final positions of the tracked particles with respect to
// the kinetic coefficients a0, a1 and the undercooling offset theta, with
// the deactivation masks frozen from a recorded forward run (Sec. 2.1.2
// kinetics, Eq. (2)).  Under frozen masks a particle's travel obeys
//   s_{k+1} = s_k + dt v(F(x(s_k), t_k) - theta)   for steps k < nact,
// x(s) = c + R (lambda0 site + s e_d), and nothing else couples particles.
// Reverse mode per particle, with u = R e_d and lambda = dL/ds:
//   lambda_N = <dL/dx_N, u>;  for k = nact-1 .. 0:
//     dL/da_j += lambda_{k+1} dt dT_k^b_j (dT_k > 0),
//     dL/dtheta -= lambda_{k+1} dt v'(dT_k),
//     lambda_k = lambda_{k+1} (1 + dt v'(dT_k) <grad F(x_k), u>).
// lambda is FP32; the parameter gradients are accumulated in FP64 and
// reduced in a fixed order.

// dv/d(dT), Eq. (2) differentiated.
__device__ __forceinline__ float velocity_slope(const Dev& D, float dT) {
  if (!(dT > 0.0f)) return 0.0f;
  if (D.kin_poly) return dT * fmaf(3.0f * D.ka[1], dT, 2.0f * D.ka[0]);
  const float l = log2f(dT);
  return D.ka[0] * D.kb[0] * exp2f((D.kb[0] - 1.0f) * l) +
         D.ka[1] * D.kb[1] * exp2f((D.kb[1] - 1.0f) * l);
}

// Gradient of the undercooling interpolant at p: the derivative of the
// trilinear form, zero along an axis clamped outside the grid.
__device__ __forceinline__ P3 field_grad(const Dev& D, P3 p) {
  if (D.fkind == F_UNIFORM) return P3{0.0f, 0.0f, 0.0f};
  if (D.fkind == F_LINEAR) return P3{D.fgrad[0], D.fgrad[1], D.fgrad[2]};
  p = place(D, p).p;
  float u[3] = {(p.x - D.fo[0]) * D.finv[0], (p.y - D.fo[1]) * D.finv[1],
                (p.z - D.fo[2]) * D.finv[2]};
  int i0[3];
  float f[3];
  bool cl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float fl = floorf(u[a]);
    fl = fmaxf(fl, 0.0f);
    fl = fminf(fl, (float)(D.fn[a] - 2));
    i0[a] = (int)fl;
    const float w = u[a] - fl;
    cl[a] = w < 0.0f || w > 1.0f;
    f[a] = fminf(fmaxf(w, 0.0f), 1.0f);
  }
  const size_t sy = (size_t)D.fn[0], sz = (size_t)D.fn[0] * (size_t)D.fn[1];
  const size_t b = (size_t)i0[2] * sz + (size_t)i0[1] * sy + (size_t)i0[0];
  const float* __restrict__ g = D.fgrid;
  const float c000 = g[b], c100 = g[b + 1], c010 = g[b + sy], c110 = g[b + sy + 1];
  const float c001 = g[b + sz], c101 = g[b + sz + 1], c011 = g[b + sz + sy], c111 = g[b + sz + sy + 1];
  const float c00 = fmaf(f[0], c100 - c000, c000), c10 = fmaf(f[0], c110 - c010, c010);
  const float c01 = fmaf(f[0], c101 - c001, c001), c11 = fmaf(f[0], c111 - c011, c011);
  const float c0 = fmaf(f[1], c10 - c00, c00), c1 = fmaf(f[1], c11 - c01, c01);
  const float d0y0 = fmaf(f[1], (c110 - c010) - (c100 - c000), c100 - c000);
  const float d0y1 = fmaf(f[1], (c111 - c011) - (c101 - c001), c101 - c001);
  const float gx = fmaf(f[2], d0y1 - d0y0, d0y0);
  const float gy = fmaf(f[2], (c11 - c01) - (c10 - c00), c10 - c00);
  const float gz = c1 - c0;
  return P3{cl[0] ? 0.0f : gx * D.finv[0], cl[1] ? 0.0f : gy * D.finv[1],
            cl[2] ? 0.0f : gz * D.finv[2]};
}

// Tracked set: the records of the active store at the start of the
// recorded run, tag i = storage index i.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_adj_init(Bind Bd, uint32_t n, int32_t n_steps) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  for (uint32_t i = V.b * TPB + threadIdx.x; i < n; i += V.G * TPB) {
    const uint4 r = D.A[i];
    D.adj_rec[i] = r;
    D.tagA[i] = i;
    const bool act = (rec_fl(r) & 3u) == ST_ACTIVE;
    D.adj_nact[i] = act ? n_steps : 0;
    D.adj_sfin[i] = rec_s(r);
  }
}

// After the last recorded step: travel of the tracked particles still active.
template <class Bind>
__global__ __launch_bounds__(TPB) void k_adj_final(Bind Bd) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t n = D.cnt->n_active;
  for (uint32_t i = V.b * TPB + threadIdx.x; i < n; i += V.G * TPB) {
    const uint32_t t = D.tagA[i];
    const uint4 r = D.A[i];
    if (t != NIL && (rec_fl(r) & 3u) == ST_ACTIVE) D.adj_sfin[t] = rec_s(r);
  }
}

// Final positions of the tracked particles, [n][3].
template <class Bind>
__global__ __launch_bounds__(TPB) void k_adj_positions(Bind Bd, uint32_t n, float* xN) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  for (uint32_t i = V.b * TPB + threadIdx.x; i < n; i += V.G * TPB) {
    const uint4 r = D.adj_rec[i];
    const float* G = D.gtab + (size_t)rec_grain(r) * GT_STRIDE;
    const P3 x = lattice_pos(G, rec_sx(r), rec_sy(r), rec_sz(r), rec_dir(r), D.adj_sfin[i]);
    xN[3 * i] = x.x;
    xN[3 * i + 1] = x.y;
    xN[3 * i + 2] = x.z;
  }
}

// Reverse sweep, one thread per tracked particle.  Each checkpoint segment
// of K steps is recomputed from its checkpoint into seg[j][i] (step-major,
// coalesced) with the forward's own arithmetic, then walked backwards.
// Per-block FP64 partial sums go to part[block][3].
template <class Bind>
__global__ __launch_bounds__(TPB) void k_adj_backward(Bind Bd, uint32_t n, int32_t n_steps,
                                                      int32_t K, const float* linc, float dt,
                                                      const float* dLdx, float* seg,
                                                      double* part, uint32_t* mismatch) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  __shared__ double s_red[3][TPB / 64];
  double ga0 = 0.0, ga1 = 0.0, gth = 0.0;
  uint32_t bad = 0;
  for (uint32_t i = V.b * TPB + threadIdx.x; i < n; i += V.G * TPB) {
    const uint4 r = D.adj_rec[i];
    const int32_t nact = D.adj_nact[i];
    if (nact <= 0) continue;
    const float* G = D.gtab + (size_t)rec_grain(r) * GT_STRIDE;
    const int d = rec_dir(r), sx = rec_sx(r), sy = rec_sy(r), sz = rec_sz(r);
    // u = R e_d: column axis(d) of R (rows at G[4..12]), with the sign of d.
    const int ax = d >> 1;
    const float sg = (d & 1) ? -1.0f : 1.0f;
    const P3 u = {sg * G[4 + ax], sg * G[7 + ax], sg * G[10 + ax]};
    float lam = (dLdx[3 * i] * u.x + dLdx[3 * i + 1] * u.y) + dLdx[3 * i + 2] * u.z;
    const int32_t nck = (n_steps + K - 1) / K;
    for (int32_t c = nck - 1; c >= 0; --c) {
      const int32_t k0 = c * K;
      if (k0 >= nact) continue;
      const int32_t k1 = min(k0 + K, nact);
      float s = D.adj_ck[(size_t)c * D.adj_ncap + i];
      for (int32_t k = k0; k < k1; ++k) {
        seg[(size_t)(k - k0) * n + i] = s;
        const P3 x = lattice_pos(G, sx, sy, sz, d, s);
        const float dT = field_at(D, x, linc[k]) - D.theta;
        s = s + velocity(D, dT) * dt;
      }
      if (k1 == nact && s != D.adj_sfin[i]) bad += 1;
      for (int32_t k = k1 - 1; k >= k0; --k) {
        const float sk = seg[(size_t)(k - k0) * n + i];
        const P3 x = lattice_pos(G, sx, sy, sz, d, sk);
        const float dT = field_at(D, x, linc[k]) - D.theta;
        const float vp = velocity_slope(D, dT);
        if (dT > 0.0f) {
          const double w = (double)lam * (double)dt;
          if (D.kin_poly) {
            const double t2 = (double)dT * (double)dT;
            ga0 += w * t2;
            ga1 += w * t2 * (double)dT;
          } else {
            ga0 += w * pow((double)dT, (double)D.kb[0]);
            ga1 += w * pow((double)dT, (double)D.kb[1]);
          }
        }
        gth -= (double)lam * (double)dt * (double)vp;
        const P3 gF = field_grad(D, x);
        const float du = (gF.x * u.x + gF.y * u.y) + gF.z * u.z;
        lam = lam * fmaf(dt * vp, du, 1.0f);
      }
    }
  }
  // Fixed-order block reduction: wave sums, then the waves in order.
  double v[3] = {ga0, ga1, gth};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double x = v[q];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
    if (lane_id() == 0) s_red[q][threadIdx.x >> 6] = x;
  }
  if (bad) atomicAdd(mismatch, bad);
  __syncthreads();
  if (threadIdx.x < 3) {
    double x = 0.0;
    for (int w = 0; w < TPB / 64; ++w) x += s_red[threadIdx.x][w];
    part[(size_t)V.b * 3 + threadIdx.x] = x;
  }
}

// Sum of the per-block partials in a fixed order: lane l of wave q adds
// blocks l, l + 64, ... of component q, then a fixed shuffle tree.
__global__ void k_adj_reduce(const double* part, uint32_t nblocks, double* out) {
  const int q = threadIdx.x >> 6, l = lane_id();
  if (q >= 3) return;
  double x = 0.0;
  for (uint32_t b = (uint32_t)l; b < nblocks; b += 64u) x += part[(size_t)b * 3 + q];
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
  if (l == 0) out[q] = x;
}


// Order-independent digest of the state: wrap-around sums of a hash of each
// active record, each stopped record (flags other than the state cleared)
// and each occupied claim slot (claimed and reached masks).
__device__ __forceinline__ unsigned long long rec_digest(uint4 r) {
  const unsigned long long lo = ((unsigned long long)r.y << 32) | r.x;
  const unsigned long long hi = ((unsigned long long)(r.w & 0x3FFFFu) << 32) | r.z;
  return mix64(lo ^ mix64(hi + 0x9e3779b97f4a7c15ull));
}

template <class Bind>
__global__ __launch_bounds__(TPB) void k_digest(Bind Bd, unsigned long long* out) {
  Dev D;
  VGrid V;
  Bd.bind(D, V);
  const uint32_t na = D.cnt->n_active, ns = min(D.cnt->n_stopped, D.cap_s);
  unsigned long long a = 0, b = 0, c = 0;
  for (uint32_t i = V.b * TPB + threadIdx.x; i < na; i += V.G * TPB) {
    const uint4 r = D.A[i];
    if ((rec_fl(r) & 3u) == ST_ACTIVE) a += rec_digest(r);
  }
  for (uint32_t j = V.b * TPB + threadIdx.x; j < ns; j += V.G * TPB) {
    const uint4 r = D.S[j];
    if ((rec_fl(r) & 3u) != ST_RETIRED) b += rec_digest(r);
  }
  for (uint64_t k = (uint64_t)V.b * TPB + threadIdx.x; k <= D.cmask; k += (uint64_t)V.G * TPB) {
    const unsigned long long key = D.ckeys[k];
    if (key == CLAIM_EMPTY) continue;
    unsigned long long h = mix64(key);
    for (int w = 0; w < 16; ++w) h = mix64(h ^ D.cbits[k * 24 + w]);
    c += h;
  }
  if (a) atomicAdd(&out[0], a);
  if (b) atomicAdd(&out[1], b);
  if (c) atomicAdd(&out[2], c);
}

// ============================================================ launchers ===
static inline unsigned grid_for(uint64_t n, unsigned cap = 65535u) {
  uint64_t g = (n + TPB - 1) / TPB;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// Default launch schedule: for each tunable kernel, as many blocks as the
// device keeps resident at once (a chunked kernel whose last blocks wait for
// a second round takes about two block durations), a multiple of the 8 XCDs,
// at most STREAM_GRID.
hipError_t resident_grids(Dev& d) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  auto family = [&](std::initializer_list<const void*> ks, uint32_t& grid) -> hipError_t {
    int per_cu = 1 << 20;
    for (const void* k : ks) {
      int nb = 0;
      const hipError_t r = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, TPB, 0);
      if (r != hipSuccess) return r;
      per_cu = std::min(per_cu, nb);
    }
    uint32_t g = (uint32_t)std::max(1, per_cu) * (uint32_t)std::max(1, cus);
    g = std::min<uint32_t>(g, (uint32_t)STREAM_GRID);
    grid = g >= 8u ? g / 8u * 8u : g;
    return hipSuccess;
  };
  const void* ks[TK_N] = {(const void*)k_advance<Plain, 0>, (const void*)k_branch<Plain>, (const void*)k_cellscan<Plain>,
                          (const void*)k_scatter<Plain>, (const void*)k_scatter_children<Plain>,
                          (const void*)k_dirty<Plain>, (const void*)k_contain<Plain, 0>,
                          (const void*)k_stoplink<Plain>};
  for (int t = 0; t < TK_N && e == hipSuccess; ++t) e = family({ks[t]}, d.sched[t]);
  return e;
}

void launch_advance(const Dev& d, float dt, hipStream_t s) {
  if (d.periodic) k_advance<Plain, 1><<<d.sched[TK_ADVANCE], TPB, 0, s>>>(Plain{d}, dt);
  else k_advance<Plain, 0><<<d.sched[TK_ADVANCE], TPB, 0, s>>>(Plain{d}, dt);
  k_spawn_scan<<<1, 1024, 0, s>>>(Plain{d});
}
void launch_branch(const Dev& d, hipStream_t s) { k_branch<<<d.sched[TK_BRANCH], TPB, 0, s>>>(Plain{d}); }
static void scan_bricks(const Dev& d, int mode, hipStream_t s) {
  const uint32_t ntiles = (uint32_t)((d.n_bricks + SCAN_TILE - 1) / SCAN_TILE);
  k_scan_reduce<<<ntiles, TPB, 0, s>>>(Plain{d}, mode);
  k_scan_top<<<1, TPB, 0, s>>>(Plain{d}, mode);
  k_scan_write<<<ntiles, TPB, 0, s>>>(Plain{d}, mode);
  k_cellscan<<<mode == 0 ? d.sched[TK_CELLSCAN] : (uint32_t)STREAM_GRID, TPB, 0, s>>>(Plain{d}, mode);
}
void launch_scan(const Dev& d, hipStream_t s) { scan_bricks(d, 0, s); }
void launch_scatter(const Dev& d, hipStream_t s) { k_scatter<<<d.sched[TK_SCATTER], TPB, 0, s>>>(Plain{d}); }
void launch_scatter_children(const Dev& d, hipStream_t s) {
  k_scatter_children<<<d.sched[TK_CHILDREN], TPB, 0, s>>>(Plain{d});
}
void launch_dirty(const Dev& d, hipStream_t s) {
  k_dirty<<<d.sched[TK_DIRTY], TPB, 0, s>>>(Plain{d});
}
void launch_contain(const Dev& d, hipStream_t s) {
  if (d.periodic) k_contain<Plain, 1><<<d.sched[TK_CONTAIN], TPB, 0, s>>>(Plain{d});
  else k_contain<Plain, 0><<<d.sched[TK_CONTAIN], TPB, 0, s>>>(Plain{d});
}
void launch_stoplink(const Dev& d, hipStream_t s) {
  k_stoplink<<<d.sched[TK_STOPLINK], TPB, 0, s>>>(Plain{d});
}
void launch_nucleate(const Dev& d, hipStream_t s) {
  if (d.n_sites == 0) return;
  k_nuc_test<<<grid_for(d.n_sites, 1024), TPB, 0, s>>>(Plain{d});
  k_nuc_fire<<<1, TPB, 0, s>>>(Plain{d});
}
void launch_finish(const Dev& d, double dt, hipStream_t s) { k_finish<<<1, 1, 0, s>>>(Plain{d}, dt); }
void launch_reset_stats(const Dev& d, hipStream_t s) { k_reset_stats<<<1, 1, 0, s>>>(Plain{d}); }
void launch_stopped_rebuild(const Dev& d, hipStream_t s) {
  k_srb_count<<<STREAM_GRID, TPB, 0, s>>>(Plain{d});
  scan_bricks(d, 1, s);
  k_srb_scatter<<<STREAM_GRID, TPB, 0, s>>>(Plain{d});
  k_srb_finish<<<1, 1, 0, s>>>(Plain{d});
}
void launch_resample(const Dev& d, hipStream_t s) {
  const uint64_t total = (uint64_t)d.fn[0] * d.fn[1] * d.fn[2];
  k_resample<<<grid_for(total, 8192), TPB, 0, s>>>(Plain{d});
}
void launch_solute_nodes(const double* T, const double* w, double liq_T, double liq_m,
                         uint64_t n, float* out, hipStream_t s) {
  k_solute_nodes<<<grid_for(n, 8192), TPB, 0, s>>>(T, w, liq_T, liq_m, n, out);
}
void launch_deposit_all(const Dev& d, hipStream_t s) {
  k_deposit_all<<<grid_for((d.cmask + 1) * 8, 16384), TPB, 0, s>>>(Plain{d});
}
void launch_mushy_fraction(const uint32_t* cnt, uint64_t n, double site_over_cell, float* out,
                           hipStream_t s) {
  k_mushy_fraction<<<grid_for(n, 8192), TPB, 0, s>>>(cnt, n, site_over_cell, out);
}
void launch_melt(const Dev& d, hipStream_t s) {
  if (d.fkind == F_GRID || d.fkind == F_ROSENTHAL) {
    const uint64_t c[3] = {(uint64_t)d.fn[0] - 1, (uint64_t)d.fn[1] - 1, (uint64_t)d.fn[2] - 1};
    k_field_cellmin<<<grid_for(c[0] * c[1] * c[2], 8192), TPB, 0, s>>>(Plain{d});
    k_field_coarsemin<<<grid_for(((c[0] + 3) >> 2) * ((c[1] + 3) >> 2) * ((c[2] + 3) >> 2), 2048),
                        TPB, 0, s>>>(Plain{d});
  }
  k_melt_sites<<<grid_for(d.cmask + 1, 16384), TPB, 0, s>>>(Plain{d});
  k_walkback<<<1024, TPB, 0, s>>>(Plain{d});
  k_melt_grains<<<grid_for(d.cap_grains, 256), TPB, 0, s>>>(Plain{d});
  k_melt_stopped<<<STREAM_GRID, TPB, 0, s>>>(Plain{d});
}
void launch_count_reached(const Dev& d, hipStream_t s) {
  (void)hipMemsetAsync(d.greach, 0, 4 * (size_t)d.cap_grains, s);
  k_count_reached<<<grid_for(d.cmask + 1, 16384), TPB, 0, s>>>(Plain{d});
  k_count_finish<<<grid_for(std::max<uint64_t>(d.cap_grains, d.n_sites), 256), TPB, 0, s>>>(Plain{d});
}
void launch_init_workspace(const Dev& d, hipStream_t s) {
  k_fill_bmeta<<<grid_for(d.n_bricks, 8192), TPB, 0, s>>>(Plain{d});
}
void launch_classify_new(const Dev& d, uint32_t first, uint32_t count, bool exit_rule,
                         hipStream_t s) {
  if (count == 0) return;
  k_classify_new<<<grid_for(count, 4096), TPB, 0, s>>>(Plain{d}, first, count, exit_rule ? 1 : 0);
}
void launch_claim_ball(const Dev& d, uint32_t grain, int32_t r, hipStream_t s) {
  const uint64_t w = 2ull * (uint64_t)r + 1ull;
  k_claim_ball<<<grid_for(w * w * w, 8192), TPB, 0, s>>>(Plain{d}, grain, r);
}
void launch_claim_list(const Dev& d, const int32_t* grain, const int32_t* site,
                       const uint8_t* flags, uint32_t n, hipStream_t s) {
  if (n == 0) return;
  k_claim_list<<<grid_for(n, 8192), TPB, 0, s>>>(Plain{d}, grain, site, flags, n);
}
void launch_claim_slots(const Dev& d, const void* slots, uint32_t n, hipStream_t s) {
  if (n == 0) return;
  k_claim_slots<<<grid_for(n, 8192), TPB, 0, s>>>(Plain{d}, (const SlotOut*)slots, n);
}
void launch_export_slots(const Dev& d, uint32_t* counter, void* out, uint32_t cap_out,
                         hipStream_t s) {
  k_export_slots<<<grid_for(d.cmask + 1, 16384), TPB, 0, s>>>(Plain{d}, counter, (SlotOut*)out,
                                                               cap_out);
}
static Window make_window(const float* win) {
  Window w;
  w.on = win ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    w.lo[a] = win ? win[a] : 0.0f;
    w.hi[a] = win ? win[3 + a] : 0.0f;
  }
  return w;
}
void launch_export_particles(const Dev& d, uint32_t* counter, void* out, uint32_t cap_out,
                             const float* win, hipStream_t s) {
  k_export_particles<<<1024, TPB, 0, s>>>(Plain{d}, counter, (PartOut*)out, cap_out, make_window(win));
}
// ------------------------------------------- allocation-free particle query --
// Scratch of ge_query_particles_noalloc: a 256-byte header (the append
// counter of the export) and staging for NOALLOC_RECORDS exported particles,
// in a static device array (each device holds its own copy until the process
// ends).  Host code reaches it only through the address that
// hipGetSymbolAddress gives on each device.
constexpr size_t NOALLOC_HEADER = NOALLOC_RECORDS_OFFSET;
static __device__ __align__(256) unsigned char scratch[NOALLOC_HEADER + NOALLOC_RECORDS * sizeof(PartOut)];

__global__ void k_zero_word(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0u;
}

hipError_t noalloc_scratch(void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

void launch_export_particles_staged(const Dev& d, void* scratch_ptr, const float* win,
                                    hipStream_t s) {
  uint32_t* counter = (uint32_t*)scratch_ptr;
  k_zero_word<<<1, 64, 0, s>>>(counter);
  k_export_particles<<<1024, TPB, 0, s>>>(Plain{d}, counter,
                                          (PartOut*)((char*)scratch_ptr + NOALLOC_HEADER),
                                          (uint32_t)NOALLOC_RECORDS, make_window(win));
}
void launch_export_claims(const Dev& d, uint32_t* counter, void* out, uint32_t cap_out,
                          const float* win, hipStream_t s) {
  k_export_claims<<<4096, TPB, 0, s>>>(Plain{d}, counter, (ClaimOut*)out, cap_out, make_window(win));
}
void launch_grain_map(const Dev& d, const int32_t n[3], const float origin[3],
                      const float spacing[3], uint32_t* out, hipStream_t s) {
  const uint64_t total = (uint64_t)n[0] * n[1] * n[2];
  k_grain_map<<<grid_for(total, 8192), TPB, 0, s>>>(Plain{d}, n[0], n[1], n[2], origin[0], origin[1],
                                                    origin[2], spacing[0], spacing[1], spacing[2],
                                                    out);
}
void launch_digest(const Dev& d, unsigned long long* out, hipStream_t s) {
  k_digest<<<2048, TPB, 0, s>>>(Plain{d}, out);
}
void launch_adj_init(const Dev& d, uint32_t n, int32_t n_steps, hipStream_t s) {
  if (n) k_adj_init<<<grid_for(n, 4096), TPB, 0, s>>>(Plain{d}, n, n_steps);
}
void launch_adj_final(const Dev& d, hipStream_t s) { k_adj_final<<<4096, TPB, 0, s>>>(Plain{d}); }
void launch_adj_positions(const Dev& d, uint32_t n, float* xN, hipStream_t s) {
  if (n) k_adj_positions<<<grid_for(n, 4096), TPB, 0, s>>>(Plain{d}, n, xN);
}
void launch_adj_backward(const Dev& d, uint32_t n, int32_t n_steps, int32_t K, const float* linc,
                         float dt, const float* dLdx, float* seg, double* part, double* grad_out,
                         uint32_t* mismatch, hipStream_t s) {
  k_adj_backward<<<ADJ_BLOCKS, TPB, 0, s>>>(Plain{d}, n, n_steps, K, linc, dt, dLdx, seg, part, mismatch);
  k_adj_reduce<<<1, 192, 0, s>>>(part, ADJ_BLOCKS, grad_out);
}


// ------------------------------------------------------ batched launches --
static inline Batch bind_of(const BatchLaunch& L, int site) {
  return Batch{L.tab, L.base, L.site[site].map, L.site[site].gsz};
}

void launch_batch_reset_stats(const BatchLaunch& L, hipStream_t s) {
  k_reset_stats<<<L.site[BS_ONE].total, 1, 0, s>>>(bind_of(L, BS_ONE));
}

// One step of every context of the batch: the launches of a plain step, each
// covering all contexts.  The re-sort kernels run every step; each context's
// device step count decides whether its stopped store is re-sorted.
void launch_batch_step(const BatchLaunch& L, double dt, hipStream_t s) {
  const uint32_t one = L.site[BS_ONE].total, tiles = L.site[BS_TILES].total;
  if (L.site[BS_RESAMPLE].total)
    k_resample<<<L.site[BS_RESAMPLE].total, TPB, 0, s>>>(bind_of(L, BS_RESAMPLE));
  if (L.any_periodic)
    k_advance<Batch, 2><<<L.site[BS_ADVANCE].total, TPB, 0, s>>>(bind_of(L, BS_ADVANCE), (float)dt);
  else
    k_advance<Batch, 0><<<L.site[BS_ADVANCE].total, TPB, 0, s>>>(bind_of(L, BS_ADVANCE), (float)dt);
  k_spawn_scan<<<one, 1024, 0, s>>>(bind_of(L, BS_ONE));
  k_branch<<<L.site[BS_BRANCH].total, TPB, 0, s>>>(bind_of(L, BS_BRANCH));
  k_scan_reduce<<<tiles, TPB, 0, s>>>(bind_of(L, BS_TILES), 0);
  k_scan_top<<<one, TPB, 0, s>>>(bind_of(L, BS_ONE), 0);
  k_scan_write<<<tiles, TPB, 0, s>>>(bind_of(L, BS_TILES), 0);
  k_cellscan<<<L.site[BS_CELLSCAN].total, TPB, 0, s>>>(bind_of(L, BS_CELLSCAN), 0);
  k_scatter<<<L.site[BS_SCATTER].total, TPB, 0, s>>>(bind_of(L, BS_SCATTER));
  k_scatter_children<<<L.site[BS_CHILDREN].total, TPB, 0, s>>>(bind_of(L, BS_CHILDREN));
  k_dirty<<<L.site[BS_DIRTY].total, TPB, 0, s>>>(bind_of(L, BS_DIRTY));
  if (L.any_periodic) k_contain<Batch, 2><<<L.site[BS_CONTAIN].total, TPB, 0, s>>>(bind_of(L, BS_CONTAIN));
  else k_contain<Batch, 0><<<L.site[BS_CONTAIN].total, TPB, 0, s>>>(bind_of(L, BS_CONTAIN));
  k_stoplink<<<L.site[BS_STOPLINK].total, TPB, 0, s>>>(bind_of(L, BS_STOPLINK));
  if (L.site[BS_NUCTEST].total) {
    k_nuc_test<<<L.site[BS_NUCTEST].total, TPB, 0, s>>>(bind_of(L, BS_NUCTEST));
    k_nuc_fire<<<L.site[BS_NUCFIRE].total, TPB, 0, s>>>(bind_of(L, BS_NUCFIRE));
  }
  k_finish<<<one, 1, 0, s>>>(bind_of(L, BS_ONE), dt);
  k_srb_count<<<L.site[BS_RESORT].total, TPB, 0, s>>>(bind_of(L, BS_RESORT));
  k_scan_reduce<<<tiles, TPB, 0, s>>>(bind_of(L, BS_TILES), 1);
  k_scan_top<<<one, TPB, 0, s>>>(bind_of(L, BS_ONE), 1);
  k_scan_write<<<tiles, TPB, 0, s>>>(bind_of(L, BS_TILES), 1);
  k_cellscan<<<L.site[BS_RESORT].total, TPB, 0, s>>>(bind_of(L, BS_RESORT), 1);
  k_srb_scatter<<<L.site[BS_RESORT].total, TPB, 0, s>>>(bind_of(L, BS_RESORT));
  k_srb_finish<<<one, 1, 0, s>>>(bind_of(L, BS_ONE));
}

}  // namespace ge
