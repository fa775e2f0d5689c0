/* tpc.h -- C ABI of the MI355X TPC track-reconstruction library (gfx950, HIP).
 *
 * The method: per TPC sector, cellular-automaton seeding (neighbour links between
 * clusters on adjacent pad rows, mutual cleaning, chains of >= 3 clusters) followed
 * by Kalman-filter track following, ownership arbitration, track selection, a
 * Kalman refit and the merge of track pieces across neighbouring sectors.  The
 * paper (arXiv 2402.01205) establishes that this step dominates the synchronous
 * processing (section 5 and Table 1: TPC processing 99.37% of the time; Table 2:
 * TPC tracking 61.41% of the asynchronous time), that it must track every
 * collision because track-model compression stores cluster-to-track residuals
 * (section 5), that its cost is linear in the number of TPC hits (section 6), and
 * that it runs on GPUs (sections 6-7).  The paper does not spell the algorithm
 * out; the library implements a fixed reading of it whose constants are the
 * fields of tpc_params.  The rest of the paper's GPU chain for the TPC is here
 * too (section 5): cluster finding from zero-suppressed digits before the
 * tracking (tpc_find_clusters), and after it the track-model compression of
 * the clusters against the tracks (tpc_compress / tpc_decompress) and the rANS
 * entropy coder (tpc_rans_encode / tpc_rans_decode).
 *
 * Conventions
 *  - Pointers are DEVICE pointers unless marked [host].  The caller owns every
 *    buffer: inputs, outputs and the workspace (tpc_bind_workspace).  The library
 *    allocates device memory only when no workspace was bound (then it grows its
 *    own at tpc_grid_build).
 *  - Stage calls enqueue work on the context's HIP stream and return without
 *    synchronising; counts stay on the device.  Call tpc_sync() to wait and to
 *    collect errors found by the kernels.
 *  - Cluster indices in every output are 0-based indices into the caller's
 *    cluster arrays.  Results do not depend on the input order except through the
 *    index tie-breaks that define them.
 *  - Units: cm, GeV/c, tesla, microseconds.  Track parameters (y, z, sin(phi),
 *    tan(lambda), q/pT) are in the frame of the track's sector at plane x_ref.
 *  - Return values: TPC_OK (0) or a negative TPC_E_* code; tpc_last_error()
 *    describes the last failure of the context.
 */
#ifndef TPC_H
#define TPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPC_OK 0
#define TPC_E_ARG (-1)      /* invalid argument (null pointer, size, order of calls) */
#define TPC_E_RANGE (-2)    /* a cluster had sector >= 36, row outside 0..151 or a non-finite
                               y/z; such clusters are excluded from tracking */
#define TPC_E_CAPACITY (-3) /* workspace or output capacity exceeded; results truncated */
#define TPC_E_HIP (-4)      /* HIP runtime error; see tpc_last_error */

#define TPC_N_SECTORS 36
#define TPC_N_ROWS 152

/* Every constant of the method.  tpc_params_default() fills the reading used by
 * the library's tests; changing a field changes the computed result.        */
typedef struct {
  float win_dy_slope, win_dy_const;  /* up-neighbour window in y: slope*dx + const, cm */
  float win_dz_slope, win_dz_const;  /* up-neighbour window in z, cm                   */
  float link_cut;                    /* max second difference of a link triplet, cm;  */
                                     /* > 0 with link_cut^2 a normal float             */
  float cy0, cz0, cs0, ct0, ck0;     /* tracklet Kalman priors (diagonal)              */
  float cy1, cz1, cs1, ct1, ck1;     /* refit Kalman priors (diagonal)                 */
  float sigma_y, sigma_z;            /* cluster errors, cm                             */
  float nwin;                        /* following window in sigmas                     */
  float chi2_follow;                 /* max 2-D chi2 of a followed cluster             */
  int32_t max_miss;                  /* consecutive empty rows that end the following  */
  int32_t min_hits;                  /* hits of a valid tracklet / accepted track      */
  float smax;                        /* limit of |sin(phi)|                            */
  float bz;                          /* solenoid field along +z, tesla                 */
  float merge_edge;                  /* distance to the sector edge of merge pieces, cm;*/
                                     /* negative: no merge across sectors              */
  float chi2_merge;                  /* max 5-D chi2 of a merged pair                  */
  float merge_dz;                    /* max |z| gap between the pieces' ends, cm        */
  float v_drift;                     /* drift velocity, cm/us (collision times)         */
  int32_t ext_down;                  /* 1: extend the tracks below their innermost hit, */
                                     /* 0 (default): no extension (see tpc_fit_merge)   */
  int32_t merge_membrane;            /* 1: merge pieces across the central membrane,   */
                                     /* 0 (default): no such merge (see tpc_fit_merge)  */
} tpc_params;

/* Tunable launch shapes.  Results are identical for every valid setting.     */
typedef struct {
  float cells_per_cluster;  /* grid cells per cluster of a row (search accelerator) */
  int32_t block_links;      /* threads per workgroup of the neighbour kernel (64..256)*/
  int32_t block_tracklets;  /* threads per workgroup of the tracklet kernel (64..256)*/
  int32_t persistent_waves; /* resident waves per CU of persistent kernels (0 = off)  */
  int32_t use_graph;        /* capture the batched stage chain into a hipGraph        */
  int32_t tracklet_order;   /* work order of the tracklet kernel: 0 = tracklet id,    */
                            /* 1 = grid position of the start cluster                */
  int32_t persistent_refill;/* persistent tracklet kernel: 1 = a lane whose tracklet  */
                            /* ended takes the next one, 0 = a wave takes 64 at once */
} tpc_tuning;

/* Cluster list [n] in caller order.  sector: 0..35 (0..17 side A, z >= 0);
 * row: pad row 0..151; y: sector-local y; z; time: arrival time (carried, unused
 * by the tracking).                                                           */
typedef struct {
  int32_t n;
  const uint8_t* sector;
  const int16_t* row;
  const float* y;
  const float* z;
  const float* time;
} tpc_clusters;

/* Independent tracking jobs: job j owns clusters [job_off[j], job_off[j+1]).
 * Tracking is per (job, sector); pieces merge across adjacent sectors of jobs
 * with the same event id (job_event NULL: every job is its own event).
 * job_off_host is the same table in host memory (required).                   */
typedef struct {
  int32_t n_jobs;
  const int32_t* job_off;       /* [n_jobs+1] device */
  const int32_t* job_off_host;  /* [n_jobs+1] [host] */
  const int32_t* job_event;     /* [n_jobs] device, or NULL */
} tpc_jobs;

/* Collision time t0 of a track (continuous read-out, section 2: the detector is read
 * out continuously and the data come in time frames, so a track's collision time is
 * not known in advance).  Measured z is the drift distance recomputed from the
 * arrival time, so a collision t0 after the frame start shifts every z by v_drift*t0
 * towards the far side of the central membrane (z - v_drift*t0 on side A,
 * z + v_drift*t0 on side C).  A primary comes from the nominal vertex (z = 0) on the
 * beam line, the plane x = 0 of its sector frame: the fitted state is transported
 * along the helix (state only, FP32) from x_ref to x = 0 and t0 = -z/v_drift on side
 * A, +z/v_drift on side C.  A track merged across the central membrane
 * (merge_membrane = 1) reports instead the time its two sides' z offset gives,
 * which does not assume the vertex at z = 0.  NaN where the fit failed or the
 * transport fails.                                                              */
/* Output tracks (after tpc_fit_merge).  Capacities are [host] values; counts
 * are written on the device.  hits: CSR of cluster indices ordered along the
 * track (inner piece rows ascending, then the outer piece).  When a capacity
 * is too small, tpc_sync returns TPC_E_CAPACITY, n_tracks still holds the
 * number of tracks found, the tracks and hits that fit are written and nothing
 * beyond the capacities; if the tracks fit, hit_off[n_tracks] holds the number
 * of hits needed.                                                            */
typedef struct {
  int32_t cap_tracks, cap_hits;   /* [host] */
  int32_t* n_tracks;              /* [1] */
  int32_t* hit_off;               /* [cap_tracks+1] */
  int32_t* hits;                  /* [cap_hits] */
  float* param;                   /* [cap_tracks][5] y, z, sin(phi), tan(lambda), q/pT */
  float* cov;                     /* [cap_tracks][15] lower triangle, row-major        */
  float* x_ref;                   /* [cap_tracks] plane of the parameters              */
  float* chi2;                    /* [cap_tracks]                                      */
  int32_t* ndf;                   /* [cap_tracks] 2n-5, or -1 if the fit failed       */
  int32_t* sector;                /* [cap_tracks] sector of param (innermost piece)    */
  int32_t* job;                   /* [cap_tracks]                                      */
  int32_t* tracklet;              /* [cap_tracks] id of the innermost piece's tracklet */
  float* t0;                      /* [cap_tracks] collision time, us, or NULL (below)  */
} tpc_tracks;

typedef struct tpc_ctx tpc_ctx;

/* Launch modes: how the stage entry points launch their kernels.             */
#define TPC_MODE_PLAIN 0      /* one launch sequence per job (per sector-job)           */
#define TPC_MODE_BATCHED 1    /* one launch per kernel over all jobs                    */
#define TPC_MODE_PERSISTENT 2 /* batched, the tracklet stage as resident waves taking   */
                              /* work from a device queue; the other stages stay one   */
                              /* launch over all jobs, whose items (clusters, tracks)  */
                              /* outnumber the resident waves many times over          */

int tpc_params_default(tpc_params* p);
/* Cut sets of the two processing phases (section 2: the synchronous phase uses
 * different cuts to speed up the processing).  TPC_PRESET_ASYNC is the default
 * reading plus the merge across the central membrane (merge_membrane = 1), which
 * joins the two sides of a track from a vertex off z = 0 and measures its
 * collision time from their z offset.  TPC_PRESET_SYNC serves the synchronous
 * phase, whose tracks feed the
 * track-model compression (section 5): that attaches a cluster to any piece of
 * its track, so the pieces are not merged across sector edges (merge_edge < 0
 * disables the merge), and it codes the clusters on tracks as small residuals,
 * so the tracks are extended below their innermost hits (ext_down = 1); every
 * other field is the default.  TPC_E_ARG for another preset.                  */
#define TPC_PRESET_ASYNC 0
#define TPC_PRESET_SYNC 1
int tpc_params_preset(tpc_params* p, int preset);
int tpc_tuning_default(tpc_tuning* t);

/* Create a context on `device`, enqueueing on `hip_stream` (a hipStream_t; NULL =
 * the null stream).  Copies *p (NULL = defaults).  TPC_E_ARG if a field of *p is
 * not finite or outside its domain (sigma_y, sigma_z, nwin, v_drift > 0;
 * 0 < smax < 1; min_hits >= 3; max_miss >= 1; merge_dz >= 0; ext_down 0 or 1). */
int tpc_ctx_create(tpc_ctx** ctx, int device, void* hip_stream, const tpc_params* p);
void tpc_ctx_destroy(tpc_ctx* ctx);
int tpc_set_stream(tpc_ctx* ctx, void* hip_stream);
int tpc_set_mode(tpc_ctx* ctx, int mode);
int tpc_set_tuning(tpc_ctx* ctx, const tpc_tuning* t);
/* Text of the context's last failure; with ctx = NULL, the reason of this thread's
 * last failed tpc_ctx_create.                                                  */
const char* tpc_last_error(const tpc_ctx* ctx);

/* Device bytes of the workspace for n_clusters clusters in n_jobs jobs [host].
 * Used by callers for admission control; exact for the current tuning.      */
size_t tpc_workspace_size(const tpc_ctx* ctx, int64_t n_clusters, int32_t n_jobs);
/* Bind caller-owned device memory as the workspace (>= tpc_workspace_size). */
int tpc_bind_workspace(tpc_ctx* ctx, void* dev_ptr, size_t bytes);

/* a1: validate the clusters and bin them into per-(job, sector, row) grids.
 * The arrays in *c and *j must stay valid until tpc_fit_merge returns.       */
int tpc_grid_build(tpc_ctx* ctx, const tpc_clusters* c, const tpc_jobs* j);
/* a2+a3: neighbour links and cleaning.  up/down ([n] device or NULL) receive the
 * clean links as cluster indices (-1 = none).                                */
int tpc_find_neighbours(tpc_ctx* ctx, int32_t* up, int32_t* down);
/* a4: tracklet construction.  n_tracklets ([1] device or NULL) receives T.   */
int tpc_construct_tracklets(tpc_ctx* ctx, int32_t* n_tracklets);
/* a5: selection.  n_selected ([1] device or NULL) receives K.                */
int tpc_select_tracks(tpc_ctx* ctx, int32_t* n_selected);
/* a6: refit, downward extension, merges across sector edges and the central
 * membrane, merged refit; writes *out.
 * Membrane merge (merge_membrane = 1): a track from a vertex off z = 0 whose z
 * changes sign inside the chamber leaves one piece on each side, in the same
 * sector frame, whose measured z differ by twice the drift of the collision time
 * in a time frame.  An inner piece heading for the membrane is compared with the
 * pieces of the same sector on the other side that start beyond its end and whose
 * innermost z mirrors its end z (|z_A + z_B| <= merge_dz): after transport, the
 * mean of the two z (the true z there) must lie within merge_edge of the
 * membrane and the chi2 over y, sin(phi), tan(lambda), q/pT within chi2_merge;
 * such pairs compete with the sector pairs for the mutual best.  The merged refit
 * moves z across the membrane by twice the drift of the link's time.             
 * Downward extension (ext_down = 1): a track's chain need not start at the
 * track's first row, and the following (section 6's tracking on the GPU) only
 * visits the rows above the chain, so every track whose fit succeeded continues
 * below its innermost hit, row by row inwards in its sector, with the following's
 * window, chi2 cut and miss limit, taking only clusters that no selected track
 * owns; a cluster found by several tracks goes to the one with more hits (then
 * the smaller track id), a track keeps its found clusters up to the first one it
 * lost, and its fit continues over them.  More clusters end up on tracks, which
 * the track-model compression (section 5) codes as small residuals.           */
int tpc_fit_merge(tpc_ctx* ctx, tpc_tracks* out);
/* Run a1..a6 in order (graph-captured in TPC_MODE_BATCHED/PERSISTENT when the
 * tuning asks for it).                                                        */
int tpc_run(tpc_ctx* ctx, const tpc_clusters* c, const tpc_jobs* j, tpc_tracks* out);

/* Per-kernel timing with HIP events recorded on the context's stream around the
 * launches of: the neighbour kernel (index 0), the tracklet kernel (1), the grid
 * build (2), the selection (3), fit + merge (4), tpc_compress (5),
 * tpc_decompress (6), tpc_rans_encode (7), tpc_rans_decode (8),
 * tpc_find_clusters (9) and tpc_pair_legs (10).  While
 * enabled, tpc_run does
 * not use a graph.  tpc_profile_read waits for the stream and returns the summed
 * milliseconds and the number of timed launches per index since the last reset. */
#define TPC_PROF_LINKS 0
#define TPC_PROF_TRACKLETS 1
#define TPC_PROF_GRID 2
#define TPC_PROF_SELECT 3
#define TPC_PROF_FIT_MERGE 4
#define TPC_PROF_COMPRESS 5   /* tpc_compress (all its kernels)   */
#define TPC_PROF_DECOMPRESS 6 /* tpc_decompress (all its kernels) */
#define TPC_PROF_RANS_ENCODE 7
#define TPC_PROF_RANS_DECODE 8
#define TPC_PROF_CLUSTERS 9   /* tpc_find_clusters (all its kernels) */
#define TPC_PROF_LEGS 10      /* tpc_pair_legs (all its kernels)     */
#define TPC_PROF_KERNELS 11
int tpc_profile(tpc_ctx* ctx, int enable);
int tpc_profile_read(tpc_ctx* ctx, double* ms, int32_t* launches, int32_t n, int32_t reset);

/* Track-model compression (section 5: the clusters are stored as residuals to
 * the fitted tracks instead of as absolute coordinates, which is why every
 * collision must be tracked).  One record per stored cluster:
 *   rs = row | sector << 8 | absolute << 15, and codes ey, ez (int16) in units
 *   of the quantisation steps q_y, q_z (cm).
 * Records 0 .. H-1 (H = hit_off[n_tracks]) are the track hits in track order:
 * residual codes e = rint((v - p) / q) against the track's predicted position p
 * at the cluster's pad row (the fitted state turned sector by sector to the
 * cluster's sector, same side only, then transported along the helix to the
 * row's plane; all FP32, round-half-even, q applied as the FP32 product with
 * 1/q).  A hit whose track fit failed (ndf < 0), whose prediction fails, or
 * whose residual code exceeds +-32767 is stored with absolute codes
 * e = rint(v / q) and the absolute bit.  Records H .. are the clusters in no
 * track, in input order, with absolute codes.  Absolute codes saturate at
 * +-32767.  Time frames (continuous read-out, section 2) put the drift-shifted z
 * of a 1 ms frame as far as +-2580 cm from the membrane: with ez_hi non-NULL an
 * absolute z code has 24 bits, e = rint(z * (1/q_z)) saturated at +-(2^23 - 1),
 * stored as its low 16 bits in ez and its signed high byte in ez_hi
 * (e = ez_hi * 65536 + (uint16_t)ez); ez_hi is 0 for residual and invalid
 * records, and decoding reads it the same way.  An invalid cluster (sector >= 36, row outside 0..151, non-finite y
 * or z) or a hit index outside 0..n-1 is stored as rs = 0x7FFF with zero codes.
 * Both raise TPC_E_RANGE at tpc_sync.
 * Decoding gives v = p + e*q for residual codes and v = e*q for absolute ones
 * (each operation rounded once in FP32), so |v' - v| <= q/2 up to FP32
 * rounding; the decoded clusters come in record order.                     */
typedef struct {
  int32_t cap;          /* [host] capacity of the record arrays                     */
  int32_t* n_codes;     /* [1] records needed: track hits + clusters in no track    */
  int32_t* n_attached;  /* [1] records of track hits, H                             */
  uint16_t* rs;         /* [cap]                                                   */
  int16_t* ey;          /* [cap]                                                   */
  int16_t* ez;          /* [cap]                                                   */
  int8_t* ez_hi;        /* [cap] or NULL: high byte of 24-bit absolute z codes     */
} tpc_codes;

/* Encodes the clusters `c` (device) against tracks `t` (device arrays as written
 * by tpc_fit_merge; n_tracks is read on the device and clamped to cap_tracks).
 * Uses the context's workspace, so it needs a preceding tracking run (any
 * stage) over at least c->n clusters; TPC_E_ARG otherwise, or for q <= 0.
 * When the records exceed out->cap, nothing is written beyond it, *n_codes
 * still holds the number needed and tpc_sync returns TPC_E_CAPACITY; track
 * hits beyond t->cap_hits are not read (TPC_E_CAPACITY as well, and their
 * clusters count as clusters in no track).  Runs on the context's stream.    */
int tpc_compress(tpc_ctx* ctx, const tpc_clusters* c, const tpc_tracks* t, float q_y, float q_z,
                 tpc_codes* out);
/* Decodes min(*n_codes, cap) records of `in` against the same tracks (only
 * n_tracks, hit_off, param, x_ref, sector and ndf are read) into sector, row,
 * y, z [in->cap] (device).  An invalid record decodes to sector 255, row -1,
 * y = z = NaN; a residual record without a prediction (a stream that does not
 * belong to these tracks) to NaN coordinates and TPC_E_RANGE at tpc_sync.    */
int tpc_decompress(tpc_ctx* ctx, const tpc_tracks* t, const tpc_codes* in, float q_y, float q_z,
                   uint8_t* sector, int16_t* row, float* y, float* z);

/* Looper legs (section 5: every collision is reconstructed in full).  A particle
 * whose circle turns back inside the chamber (2R < 245 cm / cos 10 deg, pT below
 * about 0.19 GeV at 0.5 T) crosses the pad rows twice and leaves two tracks, the
 * return leg followed against the particle's momentum: the same circle with the
 * signs of sin(phi), tan(lambda) and q/pT flipped.  leg[i] ([t->cap_tracks],
 * device) receives the output index of track i's other leg, or -1; entries from
 * min(*n_tracks, cap_tracks) on are -1.  Two fitted tracks (ndf >= 0) of one
 * event (job_event[job], or the job when job_event is NULL) and one z side pair
 * when their circles turn inside the chamber, their signed curvatures and
 * tan(lambda) have opposite signs, and their circle centres (global x, y) and z
 * carried along the helix to the circle's point farthest from the beam line
 * agree within 3 cm each; the score is the sum of the three squared differences
 * and pairs are mutual best ones (ties: the smaller index).  Which leg left the
 * vertex is not decided.  Reads n_tracks, param, x_ref, sector, ndf and job of
 * `t` (as written by tpc_fit_merge; no tracking run is needed on this context,
 * whose field sets the curvature).  ws: device memory of at least
 * tpc_pair_legs_workspace_size(t->cap_tracks) bytes, 256-byte aligned, owned by
 * the caller and free again when the stream has passed the call.  TPC_E_ARG for
 * a null or negative argument, a missing, small or unaligned workspace, or more
 * than 2^28 track slots (the size function returns 0 then).  Runs on the
 * context's stream.                                                            */
size_t tpc_pair_legs_workspace_size(int32_t cap_tracks);
int tpc_pair_legs(tpc_ctx* ctx, const tpc_tracks* t, const int32_t* job_event, void* ws, size_t ws_bytes,
                  int32_t* leg);

/* rANS entropy coding (section 5: every detector's data, the TPC's after the
 * track-model compression, goes through a common rANS coder; Tables 1 and 2
 * time the TPC encoding and decoding).  Static range ANS on a stream of n
 * 16-bit symbols (e.g. one field of the compression records):
 *  - model: freq[s] over 2^16 slots, f_s = max(1, floor(c_s (2^16 - K) / n))
 *    for the K symbols that occur (c_s = count), 0 for the others, and the
 *    remainder 2^16 - sum to the most frequent symbol (ties: the smaller).
 *  - coder: 32-bit state in [2^16, 2^32) starting at 2^16, 16-bit words;
 *    encoding s emits the low word and shifts when x >= f_s 2^16, then sets
 *    x = floor(x / f_s) 2^16 + (x mod f_s) + C_s (C_s = sum of f below s).
 *  - lanes: chunks of 64 x 512 symbols; lane l of chunk k codes symbols
 *    k*32768 + l + 64 m with its own state, last symbol first.  A lane's words
 *    in decoding order: final state (high, low word), then the emitted words,
 *    last emitted first; a lane without symbols has none.  lane_off[l] is the
 *    word offset of lane l, lane_off[lanes] the total.
 * tpc_rans_lanes(n) = 64 * ceil(n / 32768) is the number of lanes.  The words
 * needed are at most n + 2 * lanes.  Both calls use the context's workspace, so
 * they need a preceding tracking run over at least n clusters (TPC_E_ARG
 * otherwise); they run on the context's stream.  Encoding writes freq,
 * lane_off and *n_words in full and the words that fit in cap_words (else
 * TPC_E_CAPACITY at tpc_sync).  Decoding reads only what lane_off and
 * cap_words bound; a stream that runs short raises TPC_E_RANGE.             */
#define TPC_RANS_LANE_SYMBOLS 512
typedef struct {
  int32_t cap_words;   /* [host] capacity of words                              */
  int32_t* n_words;    /* [1] words of the coded stream                         */
  uint32_t* freq;      /* [65536] model (written by encode, read by decode)     */
  uint32_t* lane_off;  /* [tpc_rans_lanes(n) + 1]                               */
  uint16_t* words;     /* [cap_words]                                           */
} tpc_rans;
int64_t tpc_rans_lanes(int64_t n);
int tpc_rans_encode(tpc_ctx* ctx, const uint16_t* sym, int32_t n, tpc_rans* out);
int tpc_rans_decode(tpc_ctx* ctx, const tpc_rans* in, int32_t n, uint16_t* sym);

/* tpc_rans_encode for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same model, lanes and words as tpc_rans_encode, bit for bit, but every
 * intermediate buffer lives in a fixed device array of the library (10 MiB per
 * device, held until the process ends) instead of the context's workspace, so
 * it needs no tracking run and calls no hipMalloc, hipFree or allocating
 * library routine.  The caller still passes the stream and the outputs.
 * n > TPC_RANS_STATIC_MAX_SYMBOLS: TPC_E_ARG, nothing enqueued.  Capacity:
 * as tpc_rans_encode (*n_words holds the words needed; TPC_E_CAPACITY at the
 * context's next tpc_sync).  Every call on a device shares that device's array:
 * calls that overlap on one device (other streams or contexts) race and give
 * wrong results; serialise them.  TPC_E_HIP if the array's device address
 * could not be obtained when the context was created.                     */
#define TPC_RANS_STATIC_MAX_SYMBOLS 4194304
int tpc_rans_encode_static(tpc_ctx* ctx, const uint16_t* sym, int32_t n, tpc_rans* out);

/* Cluster finding (section 5: the TPC clusters are found on the GPUs from the
 * zero-suppressed digits, ahead of the tracking).  Pad plane: row r holds
 * P_r = 2 ceil(x_r tan 10 deg / pad_pitch) pads (x_r = 85 + r 160/151 cm, in
 * double), pad p centred at y = (p + 1/2) pad_pitch - P_r pad_pitch / 2; time
 * bins of time_bin cm of |z|, bin t centred at |z| = (t + 1/2) time_bin.
 * The ADC counts of the digits are summed per (sector, row, pad, time) cell
 * (digits outside the plane are dropped: TPC_E_RANGE in *status).  A digit is
 * a peak when its cell's charge q >= q_min and, over the 8 neighbouring cells
 * of its row (cells off the plane count 0), q > q_n for the neighbours that
 * come earlier in (pad, time) order and q >= q_n for the later ones.  Its
 * cluster, over the 3 x 3 cells: Q = sum q and the integer moments
 * S_p = sum q dp, S_pp = sum q dp^2 (and in time); in FP32
 * pad = p + S_p / Q, sigma_pad = sqrt(max(0, S_pp / Q - (S_p / Q)^2)),
 * y = (pad + 1/2) pad_pitch - P_r pad_pitch / 2 (last term rounded once),
 * z = (time + 1/2) time_bin, negative on side C (sectors 18..35).
 * Clusters come in the order of their peak digits; each copy of a duplicated
 * peak digit reports it.  Errors found on the device go to out->status
 * (TPC_E_RANGE / TPC_E_CAPACITY bits as in TPC_STATUS_*), not to tpc_sync;
 * beyond out->cap nothing is written and *n_clusters holds the number found.
 * The caller provides a 256-byte aligned device workspace of at least
 * tpc_cf_workspace_size() bytes (a uint32 charge map of all cells, about
 * 1.3 GB for the defaults); the call needs no tracking run before it.  The
 * call leaves the map zero: a following call on the same context with the
 * same workspace pointer and pad plane skips clearing it, so the caller must
 * not write to the workspace between such calls.                           */
#define TPC_STATUS_RANGE 1
#define TPC_STATUS_CAPACITY 2
typedef struct {
  float pad_pitch;  /* cm, >= 0.05                         */
  float time_bin;   /* cm of drift per time bin            */
  int32_t n_time;   /* time bins per row, 1..32767         */
  int32_t q_min;    /* minimum charge of a peak, ADC, >= 1 */
} tpc_cf_params;
typedef struct {
  int32_t n;
  const uint8_t* sector;
  const int16_t* row;
  const int16_t* pad;
  const int16_t* time;
  const uint16_t* adc;
} tpc_digits;
typedef struct {
  int32_t cap;            /* [host] */
  int32_t* n_clusters;    /* [1] */
  int32_t* status;        /* [1] TPC_STATUS_* bits */
  int32_t* digit;         /* [cap] index of the peak digit */
  uint8_t* sector;        /* [cap] */
  int16_t* row;           /* [cap] */
  float* y;               /* [cap] cm, sector frame */
  float* z;               /* [cap] cm */
  uint32_t* q_tot;        /* [cap] ADC over the 3 x 3 cells */
  uint32_t* q_max;        /* [cap] ADC of the peak cell */
  float* sigma_pad;       /* [cap] pads */
  float* sigma_time;      /* [cap] time bins */
} tpc_cf_clusters;
int tpc_cf_params_default(tpc_cf_params* p);  /* 0.5 cm, 0.5 cm, 500 bins, 10 ADC */
size_t tpc_cf_workspace_size(const tpc_cf_params* p, int32_t n_digits);  /* 0: invalid */
int tpc_find_clusters(tpc_ctx* ctx, const tpc_cf_params* p, const tpc_digits* d, void* ws, size_t ws_bytes,
                      tpc_cf_clusters* out);

/* Wait for the context's stream; returns TPC_E_RANGE / TPC_E_CAPACITY if the
 * kernels reported one since the last tpc_grid_build, else TPC_OK.           */
int tpc_sync(tpc_ctx* ctx);

/* Enqueues on the context's stream a copy of six counters of the last run into
 * dst[6] (device memory or pinned host memory), without synchronising:
 *   dst[0] status bits since the last tpc_grid_build (TPC_STATUS_RANGE,
 *          TPC_STATUS_CAPACITY: the conditions tpc_sync reports),
 *   dst[1] tracklets, dst[2] selected tracks, dst[3] their hits,
 *   dst[4] output tracks (= *n_tracks), dst[5] their hits (hit_off[n_tracks]).
 * For callers with several runs in flight on different streams that check each
 * run's status when its results arrive.  TPC_E_ARG before the first run.      */
int tpc_counts(tpc_ctx* ctx, int32_t* dst);

/* Test hooks (stage outputs, device pointers, sizes n or capacities):        */
/* raw links before cleaning, as cluster indices                             */
int tpc_get_links_raw(tpc_ctx* ctx, int32_t* up_raw, int32_t* down_raw);
/* row membership: slot_off [n_jobs*36*152+1] and members sorted per slot by
 * the grid order (cell order; within a cell any order)                       */
int tpc_get_rows(tpc_ctx* ctx, int32_t* slot_off, int32_t* members);
/* tracklets: [host] counts, then device arrays of capacity >= T / sum of hits:
 * start[T], off[T+1], hits[sum], state[T][21] (y z s t k, C[15], x)          */
int tpc_get_tracklet_counts(tpc_ctx* ctx, int32_t* n_tracklets, int64_t* n_hits);
int tpc_get_tracklets(tpc_ctx* ctx, int32_t* start, int32_t* off, int32_t* hits, float* state,
                      uint64_t* hit_weight);
/* selected tracks before the fit: [host] counts then CSR (cluster indices)  */
int tpc_get_selected_counts(tpc_ctx* ctx, int32_t* n_selected, int64_t* n_hits);
int tpc_get_selected(tpc_ctx* ctx, int32_t* tracklet, int32_t* off, int32_t* hits);

/* Streaming copy of `bytes` (multiple of 16) from src to dst on the context's
 * stream: the achievable-bandwidth probe of the roofline and the reference for
 * calibrating hardware traffic counters.                                      */
int tpc_copy_probe(tpc_ctx* ctx, const void* src, void* dst, size_t bytes);

/* Unit hooks of the device track model (tests): n rows, device arrays.
 * propagate: in [n][22] = (y, z, sin phi, tan lambda, q/pT, C[15], x1, x2),
 *            out [n][26] = (ok, state hi[5], state lo[5], C[15]).
 * update:    in [n][27] = (hi[5], lo[5], C[15], y_meas, z_meas),
 *            out [n][27] = (ok, hi[5], lo[5], C[15], chi2).                  */
int tpc_debug_propagate(tpc_ctx* ctx, const float* in, float* out, int32_t n);
int tpc_debug_update(tpc_ctx* ctx, const float* in, float* out, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* TPC_H */
