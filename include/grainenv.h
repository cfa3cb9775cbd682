/*
 * grainenv — MI355X (gfx950) implementation of the per-step update of the
 * particle-based grain-envelope method for solidification microstructures
 * (Mosbah, Gomez Vazquez, Zenz, Tourret, Otto, arXiv:2504.12858).
 *
 * One step of the method, for every tracking particle of every grain:
 *   - undercooling at the particle from the thermal field (Sec. 2.3: the
 *     field is interpolated at particle positions),
 *   - growth velocity from the kinetic law Eq. (1)/(2) (Sec. 2.1.2),
 *   - advance along the grain's rotated <100> direction (Sec. 2.1.2),
 *   - branching into outer directions after lambda0 of travel (Sec. 2.1.2,
 *     Fig. 2),
 *   - rebinning into a uniform cell list and deactivation of particles that
 *     meet another grain's particles (grain-boundary formation, Sec. 2.1.2;
 *     neighbour search, Sec. 2.3),
 *   - nucleation of liquid sites whose undercooling reaches their drawn
 *     threshold (Sec. 2.1.1).
 *
 * Conventions
 *   - SI units.  Undercooling dT = T_L - T in kelvin, minus the offset theta.
 *   - Every function returns a ge_status; nothing throws across the ABI.
 *   - A context owns no device memory: the caller passes a workspace of
 *     ge_workspace_size() bytes (device memory) and a HIP stream; every
 *     device operation of the context is issued on that stream.
 *   - Host arrays passed in are copied before the call returns.  Device
 *     arrays passed in are read in stream order: keep them alive until the
 *     stream has passed the call.
 *   - One context per stream; a context is not thread-safe.
 *   - Errors found on the device (capacity, non-finite values, CFL) are
 *     sticky: they surface at the next call that synchronises (ge_step with
 *     non-null stats, ge_query_envelope) and leave the context unusable for
 *     further steps (GE_ESTATE).  Recover by re-creating the context with
 *     larger capacities and reloading a saved state.
 */
#ifndef GRAINENV_H
#define GRAINENV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ge_status;
#define GE_OK 0
#define GE_EINVAL (-1)     /* invalid argument or parameter set */
#define GE_ECAPACITY (-2)  /* a capacity of the context was exceeded */
#define GE_ENUMERIC (-3)   /* non-finite undercooling or travel */
#define GE_ECFL (-4)       /* v dt > rc / 2, or travel >= 2 lambda0 before branching */
#define GE_EDEVICE (-5)    /* HIP runtime error */
#define GE_ESTATE (-6)     /* context unusable after an earlier device error */

/* Thermal field kinds (values of ge_field.kind). */
#define GE_FIELD_UNIFORM 0   /* dT(x, t) = dT */
#define GE_FIELD_LINEAR 1    /* dT(x, t) = dT0 + grad . x + rate t */
#define GE_FIELD_GRID 2      /* trilinear interpolation of node values */
#define GE_FIELD_ROSENTHAL 3 /* LINEAR background minus a moving point source,
                                resampled onto the node grid every step */
#define GE_FIELD_SOLUTE 4    /* temperature and solute node values: the local
                                undercooling is taken with respect to the local
                                liquidus, dT = liq_T + liq_m w - T (Sec. 3.4) */

/* Particle states in exported records. */
#define GE_ACTIVE 0
#define GE_STOPPED 1
#define GE_RETIRED 2

/* Nucleation-site states. */
#define GE_SITE_DORMANT 0
#define GE_SITE_FIRED 1
#define GE_SITE_ENGULFED 2 /* inside a grain's claims: can never fire */

/*
 * Model and capacity parameters.
 *
 * Kinetic law, Eq. (2) (Sec. 2.1.2):  v = a[0] dT^b[0] + a[1] dT^b[1] for
 * dT > 0, v = 0 otherwise (Eq. (1) is a[1] = 0).  Exponents (2, 3) take a
 * polynomial path, any other exponents the power path.
 *
 * Geometry: the box is [lo, hi); the cell list has cells of edge h covering
 * it (ceil((hi - lo) / h) per axis), grouped in bricks of 4^3 cells.  The
 * contact radius rc must satisfy rc <= h and rc <= lambda0; with rc <= h/2
 * the containment test visits 2^3 cells per particle, otherwise 3^3.
 * Lattice sites must stay within +-16000 of a grain's centre:
 * (box diagonal) / lambda0 < 16000, the extent of a periodic axis counted
 * twice.  Dense per-cell tables take 24 bytes per cell (padded to whole
 * bricks).
 *
 * Periodic axes (Sec. 3.4 imposes periodic conditions on the faces normal
 * to x and y): bit a of `periodic` makes axis a repeat with period
 * L = hi - lo, which must be a whole number (at least 3) of cells h.
 * Particles never leave through such faces (box_exit concerns the other
 * axes); positions stay lattice-anchored (unwrapped: a grain grows on
 * across the face), and the field, the cell of a particle, the deposition
 * cell and the grain map take the position wrapped into the box.  Two
 * particles meet when their nearest periodic images are closer than rc and
 * they belong to different grains, or to one grain through a non-zero
 * period shift (a grain that has grown around the period meets itself).  A
 * nucleation site is inside a grain when one of its periodic images is.
 * cap_grains must then stay below 2^26 - 8 (the image of a position is kept
 * in the upper bits of its grain word).
 */
typedef struct ge_params {
  double lo[3], hi[3];   /* box [m] */
  double lambda0;        /* branching spacing: distance between tracking points [m] */
  double h;              /* cell edge [m] */
  double rc;             /* contact radius: particles of two grains closer than rc meet [m] */
  double a[2], b[2];     /* kinetic law coefficients [m s^-1 K^-b] and exponents */
  double theta;          /* undercooling offset [K], subtracted from the field */
  int32_t branching;     /* 1: particles branch after lambda0 of travel; 0: they never do */
  int32_t box_exit;      /* 1: particles leaving the box stop */
  int64_t cap_particles; /* capacity of the active particle store */
  int64_t cap_stopped;   /* capacity of the stopped particle store */
  int32_t cap_grains;    /* maximum number of grains (< 2^28 - 1) */
  int32_t cap_sites;     /* maximum number of nucleation sites */
  int64_t cap_claim_bricks; /* slots of the claim hash (rounded up to a power of two,
                               at most 2^31); each slot holds 8^3 lattice sites of
                               one grain */
  int32_t field_n[3];    /* largest field grid the context will hold (nodes per axis) */
  int32_t resort_every;  /* steps between re-sorts of the stopped store by cell (0: 16) */
  int32_t periodic;      /* bit a (a = 0, 1, 2 for x, y, z): axis a is periodic */
} ge_params;

/* Thermal field (Sec. 2.3 interpolation; Sec. 3.1 / 3.4 imposed fields). */
typedef struct ge_field {
  int32_t kind;
  double dT;                /* UNIFORM */
  double dT0, grad[3], rate;/* LINEAR, and ROSENTHAL background [K, K/m, K/s] */
  int32_t n[3];             /* GRID / ROSENTHAL: nodes per axis (>= 2, <= field_n) */
  double origin[3];         /* node (0,0,0) [m] */
  double spacing[3];        /* node spacing [m] */
  const float* data;        /* GRID: node values, index (k*ny + j)*nx + i */
  int32_t data_on_device;   /* 1: data is device memory read in stream order */
  /* ROSENTHAL source: dT -= q / (2 pi r) exp(-U (xi + r) / (2 alpha)),
     r = max(|x - x_s(t)|, r_min), xi = signed distance along the travel
     direction; the source rasters back and forth along x between x_start
     and x_end at speed U, at (y, z) = (ys, zs); dT is floored at dT_min. */
  double q, U, alpha, x_start, x_end, ys, zs, r_min, dT_min;
  /* SOLUTE: temperature T [K] and solute concentration w of every node of the
     grid (n, origin, spacing), FP64, index (k*ny + j)*nx + i, host or device
     memory (data_on_device); liquidus T_L(w) = liq_T + liq_m w [K, K per unit
     of w].  The node undercooling T_L(w) - T is formed in FP64 and stored in
     FP32; the liquidus being linear in w, its trilinear interpolant is the
     liquidus of the interpolated concentration minus the interpolated
     temperature. */
  const double* T;
  const double* w;
  double liq_T, liq_m;
} ge_field;

/* Counters of a ge_step call (sums over its steps) and the state after it. */
typedef struct ge_step_stats {
  int64_t n_active;   /* active particles after the last step */
  int64_t n_stopped;  /* stopped particles after the last step */
  int64_t n_grains;
  int64_t n_claim_bricks;
  int64_t advanced;   /* particle updates: active particles advanced */
  int64_t exited;     /* particles stopped by leaving the box */
  int64_t spawners;   /* particles that reached their target */
  int64_t children;   /* particles created by branching */
  int64_t contained;  /* particles stopped by meeting another grain */
  int64_t nucleated;  /* sites fired */
  double max_step;    /* largest v dt of the call [m] */
  double t;           /* time after the call [s] */
  int64_t step;       /* steps taken since creation or the last state load */
  int64_t pair_tests; /* candidate particles examined by the containment test (a particle's
                         candidates are examined until it is found to meet another grain:
                         the count depends on timing and on the order within a cell, and
                         is not reproducible) */
  int64_t dirty_tests;/* active particles given the containment test: those of the cells
                         of dirty bricks whose 3x3x3 cell neighbourhood reaches a brick
                         that holds another grain */
  int64_t melted;     /* melting: reached sites melted */
  int64_t removed;    /* melting: particles removed with their melted departure sites */
  int64_t reactivated;/* melting: particles re-activated next to melted sites (walk-back) */
  int64_t grains_melted; /* melting: grains melted entirely */
} ge_step_stats;

/* Query kinds of ge_query_envelope. */
#define GE_QUERY_COUNTS 0    /* out: ge_step_stats (counters zero) */
#define GE_QUERY_PARTICLES 1 /* out: ge_particle_rec[n_active + n_stopped] */
#define GE_QUERY_GRAIN_MAP 2 /* out: uint32 labels [n2][n1][n0], 0 = liquid, g + 1 = grain g */
#define GE_QUERY_CLAIMS 3    /* out: ge_claim_rec[...] */
#define GE_QUERY_SITES 4     /* out: int32 site states [n_sites] */
#define GE_QUERY_GRAINS 5    /* out: float [n_grains][24]: centre, pad, R (row-major), lambda0 R */
#define GE_QUERY_DIGEST 6    /* out: uint64 [3]: order-independent digests of the active
                                particles, the stopped particles and the claims (equal
                                states give equal digests) */
#define GE_QUERY_MUSHY_COUNTS 7 /* out: uint32 [n2][n1][n0]: reached lattice sites per cell
                                   of the deposition grid (EINVAL if none is set) */
#define GE_QUERY_MUSHY 8     /* out: float [n2][n1][n0]: mushy-zone fraction per cell,
                                g^m = min(1, count lambda0^3 / cell volume) */

/* Exported particle: position computed on the device, binning cell. */
typedef struct ge_particle_rec {
  float x, y, z;     /* position [m]; on periodic axes unwrapped (lattice-anchored) */
  float s;           /* travel since the departure site [m] */
  int32_t site[3];   /* departure lattice site (crystal frame) */
  uint32_t grain;
  uint8_t dir;       /* 0..5 = +x,-x,+y,-y,+z,-z of the crystal frame */
  uint8_t state;     /* GE_ACTIVE / GE_STOPPED */
  uint16_t pad;
  int32_t cell[3];   /* cell of the uniform cell list holding the particle */
} ge_particle_rec;   /* 48 bytes */

/* Exported claimed lattice site. */
typedef struct ge_claim_rec {
  uint32_t grain;
  int32_t site[3];
  uint32_t flags;    /* 1 = claimed as a target, 2 = reached */
} ge_claim_rec;      /* 20 bytes */

/* Arguments of GE_QUERY_GRAIN_MAP: voxel centre = origin + (i + 1/2) spacing.
   A voxel takes the grain whose reached lattice site nearest to the voxel
   centre is the voxel's own rounded site (Voronoi interpolation, Sec. 2.3). */
typedef struct ge_query_args {
  int32_t n[3];
  double origin[3];
  double spacing[3];
} ge_query_args;

/* Full state for ge_load_state (host arrays). */
typedef struct ge_state_in {
  int32_t n_grains;
  const double* centre;    /* [n_grains][3] */
  const double* quat;      /* [n_grains][4] (w, x, y, z), crystal -> world */
  int64_t n_particles;
  const int32_t* grain;    /* [n] */
  const int32_t* site;     /* [n][3] */
  const int32_t* dir;      /* [n] */
  const float* s;          /* [n] travel, finite, 0 <= s < 2 lambda0 (EINVAL otherwise) */
  const int32_t* state;    /* [n] GE_ACTIVE / GE_STOPPED (GE_RETIRED entries are dropped) */
  int64_t n_claims;
  const int32_t* c_grain;  /* [m] */
  const int32_t* c_site;   /* [m][3] */
  const uint8_t* c_flags;  /* [m] */
  int32_t n_sites;         /* must equal the number of registered sites */
  const int32_t* site_state; /* [n_sites] */
  double t;
  int64_t step;
} ge_state_in;

typedef struct ge_ctx ge_ctx;

/* Bytes of device workspace the parameters need.  EINVAL on invalid params. */
ge_status ge_workspace_size(const ge_params* p, size_t* bytes);

/* Checks the parameters without touching a device. */
ge_status ge_validate_params(const ge_params* p);

/* Creates a context over a caller-owned device workspace of at least
   ge_workspace_size() bytes (256-byte aligned) and a caller-owned HIP stream
   (hipStream_t, may be NULL for the null stream).  The workspace is
   initialised on the stream. */
ge_status ge_create(const ge_params* p, void* workspace, size_t bytes, void* stream,
                    ge_ctx** out);

/* Destroys the context (host memory only; the workspace stays the caller's). */
ge_status ge_destroy(ge_ctx* ctx);

/* Text of the last error of the context ("" if none).  With ctx == NULL: why
   the last ge_create of the calling thread failed ("" if it did not). */
const char* ge_last_error(const ge_ctx* ctx);

/* Appends n grains (Sec. 2.1.2).  shell_r[i] = 0: a nucleus of six particles
   at the centre moving along the six <100> directions (Step 0 of Fig. 2),
   the centre site claimed.  shell_r[i] = r > 0: an octahedral envelope of L1
   radius r lattice steps: one particle per lattice site of the L1 shell r,
   moving along its axis of largest |offset| (lowest axis on ties), all sites
   of the L1 ball r claimed as reached.  Particles outside the box start
   stopped.  first_id (nullable) receives the index of the first new grain.
   ECAPACITY when a capacity would be exceeded. */
ge_status ge_init_grains(ge_ctx* ctx, int32_t n, const double* centre /*[n][3]*/,
                         const double* quat /*[n][4]*/, const int32_t* shell_r /*[n]*/,
                         uint32_t* first_id);

/* Mushy-zone deposition (Sec. 2.2: the mushy zone is the volume inside the
   grain envelopes, and its fraction g^m per volume element is what the
   coupled solver needs from the envelopes, Eqs. (4)-(5)).  The inside of a
   grain's envelope is taken as the lattice sites it has reached, each
   standing for its crystal-frame cube of edge lambda0.  A reached site counts
   in the cell of the deposition grid that holds its centre; cell (i, j, k) is
   the box of half-width spacing / 2 around node origin + (i, j, k) spacing
   (index floor((x - origin) / spacing + 1/2) per axis in FP32; sites outside
   every cell are not counted).  g^m = min(1, count lambda0^3 / cell volume)
   (GE_QUERY_MUSHY; GE_QUERY_MUSHY_COUNTS gives the counts).
   ge_set_deposition_grid sets the grid (at most field_n nodes per axis,
   EINVAL otherwise) and counts every site reached so far; from then on each
   step adds the sites it reaches (branching, nucleation, new grains), and
   ge_load_state counts the loaded claims again.  n = NULL or a zero entry
   turns the deposition off. */
ge_status ge_set_deposition_grid(ge_ctx* ctx, const int32_t* n /*[3]*/, const double* origin /*[3]*/,
                                 const double* spacing /*[3]*/);

/* Melting by walk-back (Sec. 2.1.3), off by default.  With melting on,
   every step starts, with the field of that step (dT = field - theta), by:
     1. a reached lattice site S of a grain with dT(x_S) < 0 melts: it is no
        longer claimed or reached;
     2. a particle, active or stopped, whose departure site melted is
        removed, and an active one's target is released;
     3. walk-back: for each site T melted in this step, the first direction
        d (0..5) for which S = T - e_d is a reached site of the grain gives
        an active particle at S moving towards T (travel 0), and T is claimed
        as its target: the solid sites next to the melt are re-activated;
     4. a grain left without reached sites has melted entirely, and its
        nucleation site, if it has one, is dormant again and may fire anew
        (as a new grain) once its nucleation undercooling is reached.
   Sites inside claims are then tested again every step.  The counts of a
   step call are in ge_step_stats.  Not available with an adjoint recording
   or in batched steps (EINVAL there). */
ge_status ge_set_melting(ge_ctx* ctx, int32_t on);

/* Sets the thermal field used from the next step on (undercooling values).
   ENUMERIC on non-finite scalars; EINVAL on a grid larger than field_n or
   missing node arrays.  GRID node values are copied as given: a non-finite
   node is found by the step that interpolates an undercooling from it (at an
   active particle or a dormant nucleation site), which then fails with
   ENUMERIC.  Host node arrays are copied before return; device
   node arrays are read in stream order (the caller keeps them until the
   stream has passed this call).  A new field of the same kind and geometry
   (new node values, or new scalars of the same kind) keeps the recorded step
   sequence of ge_step valid, so a coupled solver can hand over a field every
   step at the cost of one copy. */
ge_status ge_set_thermal_field(ge_ctx* ctx, const ge_field* f);

/* Registers n dormant nucleation sites (Sec. 2.1.1): position, nucleation
   undercooling and orientation.  A site fires inside ge_step when the
   undercooling at the site reaches its threshold and the site is liquid (no
   particle within rc, not inside any grain's claims); it then becomes a new
   grain with six particles at the site.  Sites fired in the same step get
   grain ids in site order.  ECAPACITY when cap_sites would be exceeded. */
ge_status ge_nucleate(ge_ctx* ctx, int32_t n, const double* xyz /*[n][3]*/,
                      const double* dT_nuc /*[n]*/, const double* quat /*[n][4]*/);

/* Advances n_steps steps of dt seconds on the context's stream.  Returns at
   once unless stats is non-null; then it synchronises, fills stats and
   returns any sticky device error: ECAPACITY, ENUMERIC (a non-finite
   undercooling at an active particle or a dormant site, or a non-finite
   travel), ECFL.  After one the context refuses further steps (ESTATE). */
ge_status ge_step(ge_ctx* ctx, double dt, int32_t n_steps, ge_step_stats* stats);

/* Exports part of the state into a caller-owned buffer (host or device).
   With out == NULL (or out_bytes too small) only *needed is set.  The call
   synchronises when out is host memory.  For PARTICLES and CLAIMS, non-null
   args select a window: only particles (claimed sites) whose world position
   (wrapped into the box on periodic axes) lies in [origin, origin + n *
   spacing) are exported; with args == NULL everything is.  GRAIN_MAP
   requires args. */
ge_status ge_query_envelope(ge_ctx* ctx, int32_t kind, const ge_query_args* args, void* out,
                            size_t out_bytes, size_t* needed);

/* Allocation-free variant of ge_query_envelope(GE_QUERY_PARTICLES), for
   callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): it calls no
   hipMalloc or hipFree.  The particles of the window `args` (NULL: all) are
   exported into a static scratch array of the library (one per device, kept
   until the process ends: a 256-byte counter and staging for at most
   1,048,576 records of 48 bytes, about 48 MiB), then copied to `out` (host
   or device memory, at least *needed bytes; out == NULL or out_bytes too
   small: only *needed is set).  Records are those of GE_QUERY_PARTICLES, in
   no particular order.  A window holding more than 1,048,576 particles is
   refused with GE_ECAPACITY (*needed still set).  Every call on one device
   shares that device's scratch: calls that overlap on one GPU (contexts on
   different streams or threads) race and must be serialised by the caller.
   Synchronises the context's stream. */
ge_status ge_query_particles_noalloc(ge_ctx* ctx, const ge_query_args* args, void* out,
                                     size_t out_bytes, size_t* needed);

/* Replaces grains, particles, claims, site states, time and step.  Particles
   keep the states they are given (an active particle outside the box stays
   active until its next advance, as in the step that produced it). */
ge_status ge_load_state(ge_ctx* ctx, const ge_state_in* st);

/* ------------------------------------------------------ saved states ---
   Checkpoint and resume of the whole state of the method (Sec. 2.1: grains
   with their orientation, the tracking particles, the lattice sites each
   grain has claimed or reached, the nucleation sites, the time), as one
   versioned, self-checking blob in host memory.  A context restored from a
   blob steps exactly like the context that saved it: the same particles,
   claims, grain rows (formed again from the FP64 centres and quaternions)
   and site states, so equal inputs give bitwise equal states afterwards.
   The usual use: save, re-create the context with larger capacities after a
   capacity error, restore.

   Layout (little-endian; every section starts on an 8-byte boundary):
     ge_state_header
     grains     n_grains    x ge_state_grain     (FP64 centre and quaternion)
     sites      n_sites     x ge_state_site      (FP64 position, threshold,
                                                  quaternion; state)
     particles  n_particles x ge_state_particle  (active and stopped)
     claims     n_claim_bricks x ge_state_claims (the claimed and reached
                masks of one grain's brick of 8 x 8 x 8 lattice sites)
   checksum: 64-bit FNV-1a over everything after the header, taken as
   little-endian 64-bit words (h = (h ^ word) * 0x100000001b3, starting from
   0xcbf29ce484222325).

   ge_save_state (synchronises): writes the blob to host memory `out`.  With
   out == NULL or out_bytes too small only *needed is set (GE_OK).  The
   sticky device error of a context in error is returned instead (a state
   taken after an error is not a state of the method).
   ge_state_check (no device needed): validates a blob (magic, version,
   sizes, section counts, checksum) and copies its header to hdr
   (nullable).  GE_EINVAL on any mismatch.
   ge_restore_state: checks the blob, then replaces the context's state like
   ge_load_state.  The blob must come from a context with the same lambda0
   and box (GE_EINVAL otherwise).  Its nucleation sites are registered when
   the context has none; otherwise the registered sites must equal the
   blob's (GE_EINVAL).  GE_ECAPACITY when a capacity of the context is too
   small for the blob. */
#define GE_STATE_MAGIC 0x54534547u /* "GEST" */
#define GE_STATE_VERSION 1u
typedef struct ge_state_header {
  uint32_t magic;          /* GE_STATE_MAGIC */
  uint32_t version;        /* GE_STATE_VERSION */
  uint64_t bytes;          /* size of the whole blob */
  uint64_t checksum;       /* of the sections after the header */
  double lambda0;          /* of the context that saved the state [m] */
  double lo[3], hi[3];     /* its box [m] */
  double t;                /* time [s] */
  int64_t step;            /* steps taken */
  int64_t n_grains, n_sites, n_particles, n_claim_bricks;
} ge_state_header;         /* 128 bytes */
typedef struct ge_state_grain {
  double centre[3];
  double quat[4];          /* (w, x, y, z), crystal -> world */
} ge_state_grain;          /* 56 bytes */
typedef struct ge_state_site {
  double xyz[3];
  double dT_nuc;
  double quat[4];
  int32_t state;           /* GE_SITE_DORMANT / FIRED / ENGULFED */
  int32_t pad;
} ge_state_site;           /* 72 bytes */
typedef struct ge_state_particle {
  float s;                 /* travel since the departure site [m] */
  uint32_t grain;
  int32_t site[3];         /* departure lattice site */
  uint8_t dir;             /* 0..5 */
  uint8_t state;           /* GE_ACTIVE / GE_STOPPED */
  uint16_t pad;
} ge_state_particle;       /* 24 bytes */
typedef struct ge_state_claims {
  uint32_t grain;
  int32_t brick[3];        /* sites 8 brick .. 8 brick + 7 along each axis */
  uint64_t claimed[8];     /* word z & 7, bit (x & 7) | (y & 7) << 3 */
  uint64_t reached[8];
} ge_state_claims;         /* 144 bytes */
ge_status ge_save_state(ge_ctx* ctx, void* out, size_t out_bytes, size_t* needed);
ge_status ge_state_check(const void* blob, size_t bytes, ge_state_header* hdr);
ge_status ge_restore_state(ge_ctx* ctx, const void* blob, size_t bytes);

/* Phase timing of ge_step with HIP events recorded on the context's stream
   between the phases of every step.
   ge_profile(ctx, 1) starts recording and clears the totals; ge_profile(ctx, 0)
   stops.  ge_profile_read synchronises and returns, per phase, the summed
   GPU time in milliseconds and the number of steps recorded.  Phases: field
   resample, advance (with the reached-site marks), branch, brick and cell
   scan, scatter, child scatter, dirty-brick pass, containment, stop linking,
   nucleation, finish, stopped-store re-sort. */
#define GE_N_PHASES 12
ge_status ge_profile(ge_ctx* ctx, int32_t on);
ge_status ge_profile_read(ge_ctx* ctx, double* ms /*[GE_N_PHASES]*/, int64_t* steps);
const char* ge_phase_name(int32_t phase);
/* Times one phase alone (0 <= phase < GE_N_PHASES; -1 stops), with two HIP
   events per step around it on the context's stream, instead of one between
   every two phases: the rest of the step runs without events in between.
   Steps run plain while it is on (HIP does not time events recorded inside a
   graph).  Clears the totals, which ge_profile_read returns (zero for the
   other phases); ge_profile ends it.  GE_EINVAL for a phase out of range. */
ge_status ge_profile_phase(ge_ctx* ctx, int32_t phase);

/* Recorded step sequences.  With graphs on (the default), a ge_step call of
   at least 2 resort_every steps runs plain steps up to a step count that is
   a multiple of resort_every, then replays a recorded hipGraph of
   resort_every steps (one launch each), then the remaining steps plain.
   Every argument of every kernel is the same from step to step (the step
   state lives in device memory), so replays give the same results as plain
   steps.  The recording is made again after any change of the launch
   arguments (schedule, model, field, sites, time step).  Phase profiling
   (ge_profile, ge_profile_phase) runs plain steps.  ge_use_graphs(ctx, 0)
   turns it off. */
ge_status ge_use_graphs(ge_ctx* ctx, int32_t on);
/* Records the step sequence for time step dt now, so that the next ge_step
   call with that dt starts replaying at once. */
ge_status ge_prepare_step(ge_ctx* ctx, double dt);

/* Holds (on = 1) or releases (on = 0) a context: while held, its steps
   change nothing (time and step count included); a held context is not in
   error.  Used to freeze some contexts of a batch while the others go on. */
ge_status ge_hold(ge_ctx* ctx, int32_t on);

/* Launch schedule: the number of thread blocks (256 threads each) of every
   tunable kernel of ge_step.  Kernels: advance, branch, cell scan, scatter,
   child scatter, dirty-brick pass, containment, stop linking.  The schedule changes only speed, never results.  The default,
   set by ge_create, is the number of blocks the device keeps resident at
   once for each kernel.
   ge_get_schedule writes the current schedule.  ge_set_schedule takes a new
   one; an entry of 0 keeps the current value; EINVAL for an entry outside
   [1, GE_MAX_BLOCKS].
   ge_autotune searches the schedule kernel by kernel: for each candidate
   (1 to 8 blocks per compute unit) it runs steps_per_trial real steps timed
   with the phase profiler, scores each by its phase time per particle
   update and keeps the best.  With a snapshot buffer (device memory of at
   least ge_workspace_size bytes, owned by the caller, used only during the
   call; EINVAL if smaller) the context's device state is copied to it
   first, every trial starts from that state and the state is restored at
   the end, so the call changes nothing but the schedule.  With snapshot =
   NULL the trials advance the state (by at most 8 * GE_N_TUNABLE *
   steps_per_trial steps in all).  It leaves the best schedule set, writes
   it to blocks_out (nullable), and leaves phase profiling off. */
#define GE_N_TUNABLE 8
#define GE_MAX_BLOCKS 2048
ge_status ge_get_schedule(ge_ctx* ctx, int32_t* blocks /*[GE_N_TUNABLE]*/);
ge_status ge_set_schedule(ge_ctx* ctx, const int32_t* blocks /*[GE_N_TUNABLE]*/);
ge_status ge_autotune(ge_ctx* ctx, double dt, int32_t steps_per_trial, void* snapshot,
                      size_t snapshot_bytes,
                      int32_t* blocks_out /*[GE_N_TUNABLE], nullable*/);
const char* ge_tunable_name(int32_t k);

/* ------------------------------------------------------------ model ---
   Replaces the kinetic law (Eq. (2): coefficients a, exponents b), the
   undercooling offset theta and the branching switch between steps.  The
   same checks as ge_validate_params apply (EINVAL). */
ge_status ge_set_model(ge_ctx* ctx, const double a[2], const double b[2], double theta,
                       int32_t branching);

/* ----------------------------------------------------------- adjoint ---
   Gradients of the final positions of the envelope particles with respect
   to the kinetic coefficients a[0], a[1] (Eq. (2)) and the undercooling
   offset theta, with the deactivation masks frozen from a recorded run.

   Under frozen masks a particle's travel obeys
     s_{k+1} = s_k + dt v(dT(x(s_k), t_k) - theta)   for its first nact steps,
   x(s) = c + R (lambda0 site + s e_d) (Sec. 2.1.2), and particles do not
   interact, so reverse mode runs per particle.  lambda = dL/ds is FP32;
   the three parameter gradients are accumulated in FP64 and reduced in a
   fixed order (bitwise reproducible).

   ge_adjoint_workspace_size: device bytes of the adjoint workspace for a
   run of n_steps steps with a checkpoint of the travel every ckpt_every
   steps (about 56 + 4 (ckpt_every + n_steps / ckpt_every) bytes per
   particle of cap_particles).  The caller owns the workspace (256-byte
   aligned) and keeps it until the last call that reads the run.

   ge_adjoint_forward: tracks the records of the active store at the call
   (n_tracked of them, in storage order: particle i of the tracked set) and
   runs n_steps ordinary steps (ge_step) while recording, per tracked
   particle, the number of steps in which it advanced (its mask: it stops at
   most once, by containment or by leaving the box) and its travel every
   ckpt_every steps.  Requires branching off (ge_set_model) and a field fixed
   in time (UNIFORM, LINEAR or GRID; LINEAR may cool at a constant rate):
   EINVAL otherwise.  Synchronises; surfaces sticky device errors.

   ge_adjoint_positions: final positions x_N of the tracked particles,
   float [n_tracked][3] (particles that stopped keep their stop position),
   to device or host memory.

   ge_adjoint_tracked: the tracked set (host copy): identity, travel at the
   start, mask and final travel.

   ge_adjoint_backward: grad = (dL/da0, dL/da1, dL/dtheta) for
   L = sum_i <dLdx_i, x_N,i>, i.e. for any loss whose gradient with respect
   to the final positions is dLdx (float [n_tracked][3], device memory when
   on_device, else host).  Reads the context's grains, field and model:
   ESTATE when the replay of the recorded run from its checkpoints does not
   reproduce the recorded final travel bit for bit (they changed since the
   run).  Synchronises. */
typedef struct ge_adjoint_rec {
  uint32_t grain;
  int32_t site[3];   /* departure lattice site */
  uint8_t dir;       /* 0..5 */
  uint8_t state0;    /* state at the start: GE_ACTIVE or GE_STOPPED */
  uint16_t pad;
  float s0;          /* travel at the start [m] */
  float s_final;     /* travel after the run or at its stop [m] */
  int32_t nact;      /* steps in which the particle advanced */
} ge_adjoint_rec;    /* 32 bytes */

ge_status ge_adjoint_workspace_size(const ge_ctx* ctx, int32_t n_steps, int32_t ckpt_every,
                                    size_t* bytes);
ge_status ge_adjoint_forward(ge_ctx* ctx, double dt, int32_t n_steps, int32_t ckpt_every,
                             void* workspace, size_t bytes, int64_t* n_tracked);
ge_status ge_adjoint_positions(ge_ctx* ctx, float* xN, size_t bytes, int32_t on_device);
ge_status ge_adjoint_tracked(ge_ctx* ctx, ge_adjoint_rec* out, size_t bytes);
ge_status ge_adjoint_backward(ge_ctx* ctx, const float* dLdx, int32_t on_device, double grad[3]);

/* ------------------------------------------------------------ batches ---
   Many independent contexts (for instance realisations of one problem with
   different nucleation sites and orientations, and uneven particle counts)
   advanced together: each phase of a step is one launch covering every
   context, whose blocks are shared out among the contexts in proportion to
   their active particles (at least 8 blocks each).  Steps of whole
   resort_every sequences are replayed from a recorded hipGraph.  Results
   are those of plain ge_step calls on each context, bit for bit.

   ge_batch_workspace_size / ge_batch_create: n contexts with parameters
   params[i] (different sizes allowed), in one caller-owned device workspace
   (256-byte aligned), all on one stream.  1 <= n <= 4096.
   ge_batch_member: context i, a full ge_ctx (initialise, load states, query
   and step it alone with the ordinary calls; it stays owned by the batch).
   ge_batch_step: n_steps steps of every context; stats (nullable) receives
   one ge_step_stats per context.  Synchronises.  On a device error of a
   context the first such status is returned (ge_batch_last_error names the
   context) and that context is unusable.
   ge_batch_get_blocks / ge_batch_set_blocks: total blocks of each shared
   launch, indexed like the schedule of ge_get_schedule (kernels without a
   shared launch: 0; at most 65536 each; a context gets at most 2048 blocks of
   a launch).  ge_batch_autotune: coordinate search of those totals
   (1 to 8 blocks per compute unit) scored by batched step time per active
   particle; its trials run real steps (steps_per_trial per candidate), from
   a snapshot of the whole batch workspace restored at the end when
   `snapshot` (at least ge_batch_workspace_size bytes of device memory) is
   given, else advancing every context.
   ge_batch_use_graphs: replays on (default) or off. */
typedef struct ge_batch ge_batch;
ge_status ge_batch_workspace_size(int32_t n, const ge_params* params /*[n]*/, size_t* bytes);
ge_status ge_batch_create(int32_t n, const ge_params* params /*[n]*/, void* workspace, size_t bytes,
                          void* stream, ge_batch** out);
ge_status ge_batch_destroy(ge_batch* b);
ge_status ge_batch_member(ge_batch* b, int32_t i, ge_ctx** out);
const char* ge_batch_last_error(const ge_batch* b);
ge_status ge_batch_step(ge_batch* b, double dt, int32_t n_steps, ge_step_stats* stats /*[n]*/);
ge_status ge_batch_use_graphs(ge_batch* b, int32_t on);
ge_status ge_batch_get_blocks(ge_batch* b, int32_t* blocks /*[GE_N_TUNABLE]*/);
ge_status ge_batch_set_blocks(ge_batch* b, const int32_t* blocks /*[GE_N_TUNABLE]*/);
ge_status ge_batch_autotune(ge_batch* b, double dt, int32_t steps_per_trial, void* snapshot,
                            size_t snapshot_bytes,
                            int32_t* blocks_out /*[GE_N_TUNABLE], nullable*/);

#ifdef __cplusplus
}
#endif

#endif /* GRAINENV_H */
