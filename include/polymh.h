/*
 * polymh.h -- C ABI of libpolymh, a gfx950 (MI355X) implementation of the
 * PolyMinHash signing and search path (Subedi, Pokharel, Puri,
 * "PolyMinHash: Efficient Area-Based MinHashing of Polygons for Approximate
 * Nearest Neighbor Search", SIGSPATIAL'25, arXiv 2511.16576).
 *
 * Conventions for every call below:
 *  - Array arguments are DEVICE pointers (memory of the current HIP device)
 *    unless the comment says "host".  The caller owns every buffer; the
 *    library keeps no pointer after a call returns and never allocates or
 *    frees device memory inside these calls (scratch comes from caller
 *    workspaces sized by the *_workspace_size functions).
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *    stream-ordered: they enqueue work and return; buffers must stay alive
 *    until the stream has passed the call.  Calls that synchronise say so.
 *  - Scalar arguments are validated before anything is enqueued; a failed
 *    validation returns a negative status and enqueues nothing.  A failed
 *    kernel launch returns POLYMH_EDEVICE.  polymh_last_error() gives the
 *    calling thread's text for the last failure.
 *  - Polygons are CSR: polygon p has vertices xy[2*offsets[p] ..
 *    2*offsets[p+1]) as interleaved int32 (x, y) pairs, the ring implicitly
 *    closed (no repeated closing vertex), either orientation.  The method
 *    treats a polygon as the set of lattice points its crossing-number test
 *    accepts (see polymh_sign).
 */
#ifndef POLYMH_H
#define POLYMH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t polymh_status;
#define POLYMH_OK 0
#define POLYMH_EINVAL (-1)    /* null pointer, bad size or count          */
#define POLYMH_ERANGE (-2)    /* empty or inverted sampling box           */
#define POLYMH_EDEVICE (-3)   /* HIP launch or runtime error              */
#define POLYMH_ECAPACITY (-4) /* a caller buffer or workspace is too small */
#define POLYMH_ENOTSUP (-5)   /* current device is not gfx950             */

/* Text of the calling thread's last failure ("" if none).  Host string owned
 * by the library, valid until the thread's next failing call. */
const char *polymh_last_error(void);

/* ABI version of this header (major * 100 + minor). */
int32_t polymh_version(void);

/* Checks that the current HIP device is a gfx950; POLYMH_ENOTSUP if not.
 * Synchronous (queries device properties). */
polymh_status polymh_check_device(void);

/* Inclusive lattice box [xmin, xmax] x [ymin, ymax]: the global MBR B of
 * Sec. 3.1 that every hash samples (Sec. 3.2).  Requires xmin <= xmax and
 * ymin <= ymax. */
typedef struct {
    int32_t xmin, ymin, xmax, ymax;
} polymh_box;

/* n CSR polygons (device pointers): offsets has n + 1 entries, offsets[0] = 0,
 * non-decreasing; xy has 2 * offsets[n] entries. */
typedef struct {
    const int32_t *xy;
    const int64_t *offsets;
    int64_t n;
} polymh_polys;

/* ---------------------------------------------------------------------------
 * polymh_prepare -- per-polygon staging (Sec. 3.1 "global MBR" preprocessing
 * and Alg. 1's "compute local MBR of P").
 *   mbr   [n][4] int32 out: (xmin, ymin, xmax, ymax) of polygon p's vertices
 *                 (all zero for a polygon with no vertex).
 *   area2 [n]    int64 out (nullable): twice the signed shoelace area, exact.
 *   flags [n]    uint32 out (nullable): bit 0 = fewer than 3 vertices, bit 1 =
 *                 all vertices collinear (empty interior), bit 2 = MBR wider
 *                 or taller than 2^26 (signing then uses 128-bit integer
 *                 orientation instead of exact FP64).
 * Stream-ordered. */
polymh_status polymh_prepare(const polymh_polys *polys, int32_t *mbr, int64_t *area2,
                             uint32_t *flags, void *stream);

/* polymh_centre -- Sec. 3.1 centring: every polygon translated so that its
 * area centroid, rounded to the lattice, is the origin (the paper centres
 * polygons before hashing, for a translation-invariant shape search).
 *   The centroid is the area-weighted mean of the signed fan triangles,
 *   computed exactly in 128-bit integers; each coordinate is rounded by
 *   floor(c + 1/2), which commutes with integer translations, so a polygon
 *   and any integer translate of it centre to identical vertices.  Polygons
 *   with fewer than 3 vertices or zero area are not moved.
 *   xy_out     [V][2] int32 out: the translated vertices (same offsets as
 *               `polys`; may not alias polys->xy).
 *   shift      [n][2] int32 out (nullable): the rounded centroid removed.
 *   range_flag int32 (nullable, caller-zeroed): set to 1 if a translated
 *               coordinate leaves int32 (a polygon spanning 2^31 or more).
 * Recompute B of the centred set with polymh_box_of.  Stream-ordered. */
polymh_status polymh_centre(const polymh_polys *polys, int32_t *xy_out, int32_t *shift,
                            int32_t *range_flag, void *stream);

/* polymh_box_of -- the global MBR of all vertices of `polys` (Sec. 3.1),
 * written to *out_host.  `ws` must hold polymh_box_of_workspace_size() bytes.
 * SYNCHRONISES the stream.  POLYMH_EINVAL if the set has no vertex. */
size_t polymh_box_of_workspace_size(void);
polymh_status polymh_box_of(const polymh_polys *polys, void *ws, size_t ws_bytes,
                            polymh_box *out_host, void *stream);

/* ---------------------------------------------------------------------------
 * polymh_sign -- Alg. 1 / Def. 2: the MinHash signature of every polygon.
 *
 *   sig[p*k + i] (uint32, [n][k]) = the 1-based index of the first sample of
 *   stream i that lands inside polygon p, or 0 if none of the first `cap`
 *   samples does (Alg. 1's initial value; the paper's loop has no cap).
 *
 *   Stream i (Sec. 3.2's fixed-seed generators; SplitMix64 of Steele, Lea and
 *   Flood): key_i = mix64(seed + (i+1)*G) and sample j >= 0 is the lattice
 *   point of r = mix64(key_i + (j+1)*G), G = 0x9E3779B97F4A7C15,
 *     x = B.xmin + ((r >> 32) * Wx >> 32),  y = B.ymin + ((r & 0xffffffff) * Wy >> 32),
 *   Wx = B.xmax - B.xmin + 1, Wy likewise (products in 64-bit unsigned).
 *   Every polygon walks the same streams (required by Thm. 1).
 *
 *   A sample outside the polygon's MBR is rejected (Alg. 1's MBR check), else
 *   it is inside iff the crossing-number test accepts it: edge (x0,y0)->(x1,y1)
 *   counts iff (y0 > y) != (y1 > y) and o = (x1-x0)(y-y0) - (x-x0)(y1-y0) has
 *   the sign of y1 - y0 (exact); an odd count is inside.  A boundary point is
 *   thus inside iff it is inside after an infinitesimal move up and right.
 *   Polygons with < 3 vertices or collinear vertices have no interior and get
 *   all-zero rows.
 *
 *   k >= 1, cap >= 1, n >= 0 (n = 0 is a no-op).  `ws` must hold
 *   polymh_sign_workspace_size(n, cfg) bytes; its contents are scratch.
 *   `cfg` (host, nullable = defaults) selects the launch shape; every shape
 *   gives the same bits.  Stream-ordered.
 */
typedef struct {
    int32_t persistent;       /* 1: one persistent launch popping (polygon, hash
                                 block) items longest-expected-first from a
                                 device queue; 0: one workgroup per item.   */
    int32_t block_threads;    /* 64..1024, multiple of 64                     */
    int32_t hash_block;       /* hashes per work item (1..k; 0 = all k)       */
    int32_t lds_edges;        /* polygons with more edges stream them from
                                 global memory instead of LDS (64..8192)     */
    int32_t samples_per_lane; /* 1 or 2 draws per lane per tile step          */
    int32_t blocks_per_cu;    /* persistent grid = blocks_per_cu * CU count   */
} polymh_sign_config;

void polymh_sign_default_config(polymh_sign_config *cfg_host);
size_t polymh_sign_workspace_size(int64_t n, const polymh_sign_config *cfg_host);
polymh_status polymh_sign(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                          uint32_t cap, uint32_t *sig, const polymh_sign_config *cfg_host,
                          void *ws, size_t ws_bytes, void *stream);

/* polymh_sign_static -- polymh_sign without a caller workspace, for callers
 * that cannot allocate device memory (code under graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The staging polymh_sign
 * keeps in `ws` lives instead in a static device array of the library
 * (about 8 MiB, room for POLYMH_SIGN_STATIC_MAX_POLYS polygons), one copy per
 * GPU, held until the process ends; the call allocates and frees nothing.
 *   n > POLYMH_SIGN_STATIC_MAX_POLYS: POLYMH_EINVAL (use polymh_sign).
 *   Every call on a GPU shares that GPU's array, and the kernels set every
 *   word they read from it: calls that overlap on one GPU (other streams,
 *   other host threads) race and give wrong signatures, so callers must
 *   serialise them.  The first call on a device looks up the array's device
 *   address (hipGetSymbolAddress, not a stream operation).
 * Otherwise exactly polymh_sign (same arguments, bits and errors).
 * Stream-ordered. */
#define POLYMH_SIGN_STATIC_MAX_POLYS 262144
polymh_status polymh_sign_static(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                 uint32_t cap, uint32_t *sig, const polymh_sign_config *cfg_host,
                                 void *stream);

/* polymh_join_rings -- polygons with holes and multipolygons (the shapes of
 * the paper's real datasets, Sec. 5.1) as single rings that every call of
 * this library takes as they are.  Input: shape p owns rings
 * poly_rings[p] .. poly_rings[p+1]-1, ring r is vertices
 * ring_offsets[r] .. ring_offsets[r+1]-1 of xy (int32 pairs); filled rings
 * counter-clockwise and holes clockwise (or every ring reversed), rings
 * non-overlapping.  Output: each shape's rings joined through bridges to
 * the first ring's first vertex v0 (R0, v0, R1, R1[0], v0, ..., Rk, Rk[0],
 * closing to v0); a bridge's two edges coincide with opposite directions,
 * so membership (crossing parity over all rings, Alg. 1's test), areas,
 * centroids and the refinement's boundary sums are those of the even-odd
 * region.  A one-ring shape is copied unchanged.
 *   xy [n_vertices][2], ring_offsets [n_rings+1], poly_rings [n_polys+1]:
 *   device, caller-owned.
 *   out_xy [out_capacity][2] int32 (polymh_join_rings_size(V, R, N) vertices
 *   suffice), out_offsets [N+1] int64, device, caller-owned; shape p's
 *   joined ring starts at ring_offsets[poly_rings[p]] + 2 (poly_rings[p] - p).
 *   bad_flag  nullable device int32, set to 1 (never cleared) if a shape has
 *   no ring, indices out of range or more output than out_capacity (such a
 *   shape is skipped and its offsets are meaningless), or a ring has fewer
 *   than 3 vertices.
 * POLYMH_EINVAL for NULL arrays, negative sizes or out_xy == xy.
 * Stream-ordered. */
int64_t polymh_join_rings_size(int64_t n_vertices, int64_t n_rings, int64_t n_polys);
polymh_status polymh_join_rings(const int32_t *xy, int64_t n_vertices, const int64_t *ring_offsets,
                                int64_t n_rings, const int64_t *poly_rings, int64_t n_polys, int32_t *out_xy,
                                int64_t out_capacity, int64_t *out_offsets, int32_t *bad_flag, void *stream);

/* polymh_sign_binned -- the same signatures as polymh_sign, bit for bit,
 * computed from shared samples: every polygon reads the same point stream
 * per hash (Sec. 3.2's fixed-seed generators; Def. 2), so for every hash the
 * samples j < horizon are drawn once, in chunks of C = 2^clamp(2 bin_bits,
 * 8, 12), and each chunk's samples are grouped by cell of a 2^bin_bits x
 * 2^bin_bits grid over B.  A (polygon, hash) takes the smallest j of the
 * first chunk whose samples in the cells under its MBR include one inside
 * the polygon; units with no such sample below the horizon (and polygons
 * needing them) are walked as in polymh_sign.  Work per unit is then about
 * the samples that fall in its cells instead of the N_B / N_P draws of a
 * walk (Thm. 2).
 *   horizon  samples drawn per hash (clamped to cap); a horizon of about 16
 *            times the largest N_B / N_P of the set leaves almost no walk.
 *   bin_bits grid side 2^bin_bits, 0..6 (cells near the typical MBR size).
 *   walk_ratio polygons with |B| < walk_ratio * area (an expected first hit
 *            near N_B / N_P below walk_ratio) are walked whole instead, and
 *            so are those whose walk is expected to cost fewer edge tests
 *            than their lookup (many edges and an MBR holding many of a
 *            chunk's samples); 0 bins every polygon.  A few hundred suits
 *            the walk's cost per draw.  The signatures do not depend on it.
 *   cfg      as polymh_sign for the walk of the polygons left to it (its
 *            persistent form, at most 16 hashes a work item); lds_edges is
 *            also the lookup's edge cache (polygons beyond it are walked
 *            when walk_ratio > 0).
 *   ws       polymh_sign_binned_workspace_size(...) bytes: about
 *            10 * k * horizon bytes of binned samples.
 * POLYMH_EINVAL for k > 65535, bin_bits outside 0..6, horizon < 1 or a
 * negative walk_ratio.
 * Stream-ordered. */
size_t polymh_sign_binned_workspace_size(int64_t n, int32_t k, uint32_t cap, uint32_t horizon, int32_t bin_bits,
                                         const polymh_sign_config *cfg);
polymh_status polymh_sign_binned(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                 uint32_t cap, uint32_t horizon, int32_t bin_bits, double walk_ratio, uint32_t *sig,
                                 const polymh_sign_config *cfg, void *ws, size_t ws_bytes, void *stream);

/* polymh_sign_binned_prebinned -- polymh_sign_binned without drawing and
 * binning the samples: ws must hold the bins of an earlier
 * polymh_sign_binned call on this device with the same workspace, polygon
 * count, box, seed, k, cap, horizon, bin_bits and cfg (only the polygons'
 * coordinates may differ), as a batch of queries signed again and again.
 * The bins depend on none of the polygons, so the signatures equal
 * polymh_sign's.  Not checked: a workspace without those bins gives wrong
 * signatures (every read stays inside the workspace).  Stream-ordered. */
polymh_status polymh_sign_binned_prebinned(const polymh_polys *polys, polymh_box box, uint64_t seed, int32_t k,
                                           uint32_t cap, uint32_t horizon, int32_t bin_bits, double walk_ratio,
                                           uint32_t *sig, const polymh_sign_config *cfg, void *ws, size_t ws_bytes,
                                           void *stream);

/* ---------------------------------------------------------------------------
 * polymh_band -- LSH band keys over the signatures (Sec. 3.2 puts polygons in
 * a hashmap keyed by their MinHash code; the banded form follows the MMDS
 * banding technique the paper cites).
 *   keys[p*b + t] (uint64, [n][b]): F_0 = mix64(band_seed + (t+1)*G),
 *   F_{u+1} = mix64(F_u XOR sig[p*k + t*r + u]) for u < r, key = F_r.
 *   Requires b >= 1, r >= 1, b*r <= k.  Stream-ordered.
 */
polymh_status polymh_band(const uint32_t *sig, int64_t n, int32_t k, int32_t b, int32_t r,
                          uint64_t band_seed, uint64_t *keys, void *stream);

/* ---------------------------------------------------------------------------
 * polymh_index_build -- the bucket table of Sec. 3.2's hashmap: all n*b
 * (band key, entry) pairs, entry = p*b + t for band t of polygon p, sorted by
 * key (ties by ascending entry, i.e. stable), so that one key's bucket is a
 * contiguous range; polymh_query keeps only entries of the query's band.
 *   sorted_keys [n*b] uint64 out, sorted_ids [n*b] int32 out (entry index).
 *   Requires n*b < 2^31.  ws: polymh_index_workspace_size(n, b) bytes of
 *   scratch.  Stream-ordered.
 */
size_t polymh_index_workspace_size(int64_t n, int32_t b);
polymh_status polymh_index_build(const uint64_t *keys, int64_t n, int32_t b, void *ws,
                                 size_t ws_bytes, uint64_t *sorted_keys, int32_t *sorted_ids,
                                 void *stream);

/* ---------------------------------------------------------------------------
 * polymh_query -- candidate generation: for query q, every dataset polygon p
 * that shares at least one band key with it (key_t(p) == qkeys[q*b + t] for
 * some band t), deduplicated, ascending id.  Two phases:
 *   cand_ids == NULL: count phase; writes cand_off[0..nq] (exclusive prefix
 *     of the per-query counts, int64) and nothing else.
 *   cand_ids != NULL: fill phase with the cand_off of the count phase (the
 *     same inputs); writes cand_ids[cand_off[q] .. cand_off[q+1]).
 *     cand_cap is the capacity of cand_ids; if cand_off[nq] > cand_cap the
 *     call returns POLYMH_ECAPACITY after a SYNCHRONOUS read of cand_off[nq];
 *     pass cand_cap < 0 to skip that read (the caller guarantees capacity).
 *   n_data is the number of indexed polygons (ids are < n_data).
 *   ws: polymh_query_workspace_size(n_data, nq) bytes (device, caller-owned,
 *   contents overwritten): a bitmap row of n_data bits per query plus two
 *   words per query.  When the rows add up to 1 GiB or more (rows of at
 *   least 16 KB), a query whose buckets hold at most 4096 entries gathers
 *   and sorts them on chip and leaves its row unused; the others (and every
 *   query of a smaller call) set bits in their row.  The lists are the same
 *   either way.  Stream-ordered except the
 *   capacity check above.
 */
size_t polymh_query_workspace_size(int64_t n_data, int64_t nq);
polymh_status polymh_query(const uint64_t *sorted_keys, const int32_t *sorted_ids,
                           int64_t n_entries, int64_t n_data, const uint64_t *qkeys, int64_t nq,
                           int32_t b, void *ws, size_t ws_bytes, int64_t *cand_off,
                           int32_t *cand_ids, int64_t cand_cap, void *stream);

/* polymh_query_capped -- both phases of polymh_query in one stream-ordered
 * call with no host synchronisation (so it can be captured in a graph):
 * cand_off and cand_ids as above; if the total exceeds cand_cap, *overflow
 * (device int32) is set to 1, every cand_off entry is set to 0 (later stages
 * then see no candidates) and cand_ids is untouched; otherwise *overflow = 0.
 * The caller re-runs with a larger capacity after reading the flag. */
polymh_status polymh_query_capped(const uint64_t *sorted_keys, const int32_t *sorted_ids,
                                  int64_t n_entries, int64_t n_data, const uint64_t *qkeys, int64_t nq,
                                  int32_t b, void *ws, size_t ws_bytes, int64_t *cand_off,
                                  int32_t *cand_ids, int64_t cand_cap, int32_t *overflow, void *stream);

/* ---------------------------------------------------------------------------
 * polymh_refine -- exact Jaccard of each candidate pair (Sec. 1: area of the
 * intersection over area of the union; Table 2's refinement phase).
 *   cand_j[c] (double) = J(data[cand_ids[c]], queries[q]) for
 *   cand_off[q] <= c < cand_off[q+1].  Intersection area by Green's theorem
 *   over the two boundaries split at their crossings, with exact orientation
 *   predicates under a consistent symbolic perturbation; FP64 accumulation
 *   relative to a local origin.  Disjoint MBRs give 0 without clipping.
 *   Relative error of the area is about 1e-13 or better for the workloads'
 *   sizes.  Stream-ordered.
 */
polymh_status polymh_refine(const polymh_polys *data, const polymh_polys *queries,
                            const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                            int64_t n_cand, double *cand_j, void *stream);

/* polymh_refine_ws -- polymh_refine (stats nullable, as polymh_refine_stats)
 * with a workspace of polymh_refine_workspace_size() bytes (device,
 * caller-owned, contents overwritten).  With it, every pair that
 * polymh_refine computes by the general form (every edge of one polygon
 * against every edge of the other, one wavefront per pair: a polygon beyond
 * 512 edges) is deferred to further launches:
 *   - with coordinate spans below 2^26, it takes the tiled form of the
 *     smaller pairs (only edges whose boxes meet are tested), both polygons
 *     passing through on-chip memory in windows of 1024 edges; a pair
 *     spanning more than two window pairs is split into up to 512 units of
 *     one wavefront each (windows of 128 to 1024 edges of the staged
 *     polygon, each against the other's windows together or one at a
 *     time), whose shared quantities (areas, anchors, carries) are found
 *     once per pair, and the partial sums are added in window order (up to
 *     2^20 list entries and 4096 split pairs per call);
 *   - with wider spans (128-bit signs), a pair with n m >= 2^17 edge pairs
 *     is split over 128 wavefronts of the general form (up to 8192 pairs),
 * so the few large pairs of a batch no longer set the call's duration.  The
 * values are those of polymh_refine within the refinement's rounding (the
 * same intersection area summed in another order; deterministic); pairs
 * beyond the caps run in place.  ws NULL is polymh_refine.  Stream-ordered
 * and graph-capturable; two calls sharing a workspace must not overlap. */
size_t polymh_refine_workspace_size(void);
polymh_status polymh_refine_ws(const polymh_polys *data, const polymh_polys *queries, const int64_t *cand_off,
                               const int32_t *cand_ids, int64_t nq, int64_t n_cand, double *cand_j,
                               uint64_t *stats, void *ws, size_t ws_bytes, void *stream);

/* polymh_refine_stats -- polymh_refine that also adds its work counts to
 * stats [4] (device uint64, caller-zeroed): pairs refined by the tiled form,
 * edge pairs that form tested (8 per kept (P chunk, Q edge) unit), edge
 * pairs tested by the general form, and pairs skipped because their MBRs are
 * disjoint.  Stream-ordered. */
polymh_status polymh_refine_stats(const polymh_polys *data, const polymh_polys *queries,
                                  const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                                  int64_t n_cand, double *cand_j, uint64_t *stats, void *stream);

/* ---------------------------------------------------------------------------
 * polymh_topk -- Def. 1 / K-ANN: per query the `topk` candidates with the
 * largest J, ties by ascending id; rows padded with id -1 and J 0.
 *   top_ids [nq][topk] int32 out, top_j [nq][topk] double out.
 *   1 <= topk <= 1024 (topk passes over each query's candidates: meant for
 *   the K of a recall@K, not for sorting whole lists).  Stream-ordered.
 */
polymh_status polymh_topk(const int64_t *cand_off, const int32_t *cand_ids, const double *cand_j,
                          int64_t nq, int32_t topk, int32_t *top_ids, double *top_j,
                          void *stream);

/* ---------------------------------------------------------------------------
 * Graph capture (batching form): record the stream-ordered libpolymh calls a
 * caller issues on `stream` between polymh_graph_begin and polymh_graph_end
 * into a HIP graph, then replay it with polymh_graph_launch (same buffers,
 * new contents).  Other streams join the capture by waiting on an event
 * recorded on `stream` (and must be joined back the same way before
 * polymh_graph_end); their branches run concurrently on replay.  The capture
 * is thread-local: calls from other threads are not recorded.  Calls that
 * synchronise (polymh_box_of, polymh_query with a capacity check,
 * polymh_rank_refine) must not be captured; use polymh_query_capped and
 * polymh_rank_refine_ordered.  The handle is owned by the caller and
 * released by polymh_graph_destroy.  Errors: POLYMH_EINVAL for a null
 * stream or output, POLYMH_EDEVICE when HIP refuses the capture, its end or
 * the instantiation (nothing is then returned). */
typedef struct polymh_graph_t *polymh_graph;
polymh_status polymh_graph_begin(void *stream);
polymh_status polymh_graph_end(void *stream, polymh_graph *out_host);
polymh_status polymh_graph_launch(polymh_graph graph, void *stream);
void polymh_graph_destroy(polymh_graph graph);

/* ---------------------------------------------------------------------------
 * Learned candidate scorer (an AI-systems form beside the method; not in the
 * paper).  A small MLP predicts a pair's Jaccard from its 256 signature
 * collisions (each a Bernoulli(J) draw by Thm. 1) and shape features, so that
 * refinement can visit candidates best-first and stop early; full refinement
 * stays the fallback.  Network: 288 inputs -> 256 -> 256 -> 1, GELU (tanh
 * form) after both hidden layers, sigmoid output, MSE loss; BF16 weights and
 * activations on the MFMA units with FP32 accumulation; Adam on FP32 master
 * weights.
 *
 * Parameter block (FP32, polymh_mlp_param_count() floats):
 *   W1 [256][288] row-major (out, in) | b1 [256] | W2 [256][256] | b2 [256] |
 *   w3 [256] | b3 [1].
 * BF16 copy (polymh_mlp_bf16_count() uint16 bit patterns): W1 then W2,
 * refreshed by polymh_mlp_sync_bf16 and by every polymh_mlp_adam.
 * Inputs X: [B][288] BF16 rows (polymh_pair_features); B a multiple of 32.
 * ------------------------------------------------------------------------- */
int64_t polymh_mlp_param_count(void);
int64_t polymh_mlp_bf16_count(void);
/* Bytes of the activation buffer (z1, z2 FP32; h1, h2 BF16; y) for batch B. */
size_t polymh_mlp_acts_size(int64_t B);
/* Bytes of the backward scratch for batch B. */
size_t polymh_mlp_scratch_size(int64_t B);
/* wbf16 <- BF16(W1), BF16(W2).  Stream-ordered. */
polymh_status polymh_mlp_sync_bf16(const float *params, uint16_t *wbf16, void *stream);
/* y [B] (nullable: kept in acts) = sigmoid(w3 . gelu(W2 gelu(W1 x + b1) + b2) + b3);
 * acts receives the activations the backward pass needs.  Stream-ordered. */
polymh_status polymh_mlp_forward(const uint16_t *X, int64_t B, const float *params,
                                 const uint16_t *wbf16, float *y, void *acts, size_t acts_bytes,
                                 void *stream);
/* After polymh_mlp_forward on the same X and acts: grad [param_count] <- the
 * gradient of the batch loss mean_r (y_r - label_r)^2, *loss (device float)
 * <- that loss.  Stream-ordered. */
polymh_status polymh_mlp_backward(const uint16_t *X, int64_t B, const float *params,
                                  const uint16_t *wbf16, void *acts, size_t acts_bytes,
                                  const float *label, float *grad, float *loss, void *scratch,
                                  size_t scratch_bytes, void *stream);
/* One Adam step (step counts from 1, bias-corrected moments m, v) on the FP32
 * parameters, then the BF16 copy is refreshed.  Stream-ordered. */
polymh_status polymh_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t step,
                              float lr, float beta1, float beta2, float eps, uint16_t *wbf16,
                              void *stream);
/* C [M][N] (FP32, row-major) = A B with BF16 operands read as
 * A(i, k) = A[i*a_row_stride + k*a_k_stride], B(k, j) = B[j*b_col_stride +
 * k*b_k_stride]; M, N multiples of 32, K of 16.  The product the scorer's
 * layers use, exported for direct checks.  Stream-ordered. */
polymh_status polymh_gemm_bf16(const uint16_t *A, int64_t a_row_stride, int64_t a_k_stride,
                               const uint16_t *B, int64_t b_col_stride, int64_t b_k_stride,
                               int64_t M, int64_t N, int64_t K, float *C, void *stream);

/* Per-polygon shape features, feats [n][12] FP32: ln(A)/ln(N_B),
 * ln(P^2/(4 pi A))/4, ln(MBR w/h)/2, ln(n)/9, (area centroid - MBR centre)/sqrt(A)
 * in x and y, A, 0, MBR (x0, y0, x1 + 1, y1 + 1).  N_B = area of the box.
 * Stream-ordered. */
polymh_status polymh_poly_features(const polymh_polys *polys, polymh_box box, float *feats,
                                   void *stream);
/* Scorer input rows X [R_pad][288] BF16 for pairs (li[r], ri[r]) of a left
 * table (signatures lsig [.][256], features lfeat [.][12]) and a right table:
 * 256 collision bits [lsig == rsig], the 6 left and 6 right shape features,
 * ln(A_l/A_r)/4, min/max area ratio, MBR intersection-over-union, collision
 * fraction, then zeros; rows R..R_pad-1, and rows whose li or ri is negative
 * (empty head slots), are zero.  k must be 256.
 * Stream-ordered. */
polymh_status polymh_pair_features(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                   const float *rfeat, int32_t k, const int32_t *li,
                                   const int32_t *ri, int64_t R, int64_t R_pad, uint16_t *X,
                                   void *stream);
/* rows[c] = q for cand_off[q] <= c < cand_off[q+1] (the query of each
 * candidate).  Stream-ordered. */
polymh_status polymh_csr_rows(const int64_t *cand_off, int64_t nq, int32_t *rows, void *stream);
/* out[r] = fraction of the k hashes on which lsig[li[r]] and rsig[ri[r]]
 * agree: the unbiased estimate of J of Thm. 1.  Stream-ordered. */
polymh_status polymh_jhat(const uint32_t *lsig, const uint32_t *rsig, int32_t k, const int32_t *li,
                          const int32_t *ri, int64_t R, float *out, void *stream);

/* The head of each query's candidate order: order [n_cand] (int32) receives
 * each query's candidate positions sorted by decreasing score (ties by
 * position; sorted_ok [nq] = 0 marks queries beyond 8192 candidates, left in
 * their given order); head_off [nq+1] (int64, CSR) with head_query (int32
 * query), head_cand (int64 global candidate index) and head_id (int32 data
 * polygon) list the first min(M, C_q) candidates of each query.  A cascade
 * uses it to re-score only the most promising candidates with the scorer.
 * The head arrays hold at most nq * M entries.  Stream-ordered. */
polymh_status polymh_rank_head(const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                               const float *score, int32_t M, int32_t *order, uint8_t *sorted_ok,
                               int64_t *head_off, int32_t *head_query, int64_t *head_cand,
                               int32_t *head_id, void *stream);
/* score[idx[i]] = val[i] for i < n with idx[i] >= 0 (negative indices, the
 * empty slots of polymh_rank_head_fixed, are skipped).  Stream-ordered. */
polymh_status polymh_scatter_scores(const int64_t *idx, const float *val, int64_t n, float *score,
                                    void *stream);

/* Ordered refinement with early stop.  Each query's candidates are visited in
 * decreasing score (predicted J; ties by position) and refined (as
 * polymh_refine) in rounds of F per query; a query stops once it holds topk
 * results and its topk-th exact J >= next score + margin, or when its
 * candidates are exhausted (margin = +inf refines everything: the fallback,
 * equal to polymh_refine + polymh_topk).  Queries with more than 8192
 * candidates are refined fully in their given order.  top_ids/top_j as in
 * polymh_topk.  If max_rounds rounds pass with queries still active, one
 * finishing pass refines all the candidates those queries have left (so the
 * top-k is always complete; only the work saved by early stop is lost).
 * *n_refined_host and *rounds_host (nullable, host) receive the number of
 * refined pairs and of rounds taken before the finishing pass.
 * SYNCHRONISES the stream once per round (the stop test of the round is read
 * back); polymh_rank_refine_ordered is the form without host reads.  Each
 * round refines as polymh_refine_ws (pairs beyond 512 edges on the windowed
 * tiled form).  ws: polymh_rank_workspace_size(nq, n_cand, F) bytes (it
 * includes the refinement's workspace). */
size_t polymh_rank_workspace_size(int64_t nq, int64_t n_cand, int32_t F);
polymh_status polymh_rank_refine(const polymh_polys *data, const polymh_polys *queries,
                                 const int64_t *cand_off, const int32_t *cand_ids,
                                 const float *score, int64_t nq, int64_t n_cand, int32_t topk,
                                 int32_t F, float margin, int32_t max_rounds, void *ws,
                                 size_t ws_bytes, int32_t *top_ids, double *top_j,
                                 int64_t *n_refined_host, int32_t *rounds_host, void *stream);

/* polymh_rank_jhat_order -- the collision fraction of every candidate pair
 * (Thm. 1: each hash collides with probability J, so the share of agreeing
 * hashes is an unbiased estimate of J) and each query's best-first order in
 * one pass.
 *   qsig [nq][k], dsig [n_data][k]: signatures of the queries and of the
 *   indexed polygons; cand_off/cand_ids: the candidate CSR of polymh_query.
 *   score [C] float out: agreeing hashes / k for candidate c.
 *   order [C] int32 out: per query, the positions (0-based, within the query's
 *   list) sorted by decreasing score, ties by position; sorted_ok [nq] uint8
 *   out: 0 for a query beyond 8192 candidates (left in its given order).
 * Stream-ordered, no host reads (graph-capturable). */
polymh_status polymh_rank_jhat_order(const uint32_t *qsig, const uint32_t *dsig, int32_t k,
                                     const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                                     float *score, int32_t *order, uint8_t *sorted_ok, void *stream);

/* polymh_sig_pack_stride -- bytes a row of the saturated signature table
 * takes for k hashes (2k), or 0 when k is not a multiple of 4 in [4, 256]. */
size_t polymh_sig_pack_stride(int32_t k);

/* polymh_sig_pack -- the saturated signature table of sig [n][k], the layout
 * polymh_rank_jhat_order_packed reads: uint16 [n][k], entry i of row r =
 * min(sig[r][i], 65535).  With sig it decides equality exactly: two values
 * are equal when their entries are equal and below 65535, or both entries
 * are 65535 and the values themselves are equal.  First hits (Def. 2)
 * average 1/S_p draws (Thm. 2), so at the configured data sets' shares
 * almost every value lies below 65535.
 *   sig: device, 16-byte aligned; packed: device, n * 2k bytes, 8-byte
 *   aligned, owned by the caller.  Errors: POLYMH_EINVAL for k not a
 *   multiple of 4 in [4, 256], n < 0, or NULL or misaligned arrays.
 *   Stream-ordered. */
polymh_status polymh_sig_pack(const uint32_t *sig, int64_t n, int32_t k, void *packed, void *stream);

/* polymh_rank_jhat_order_packed -- polymh_rank_jhat_order (the same score,
 * order and sorted_ok, bit for bit) reading the indexed signatures as the
 * saturated table `packed` that polymh_sig_pack made from dsig: a candidate
 * costs 2k bytes instead of 4k, and dsig is read only where the query's and
 * the candidate's entries are both 65535.  k a multiple of 4 in [4, 256];
 * qsig and dsig 16-byte aligned, packed 8-byte aligned.  Errors as
 * polymh_rank_jhat_order, and POLYMH_EINVAL for another k or a misaligned
 * array.  Stream-ordered, no host reads (graph-capturable). */
polymh_status polymh_rank_jhat_order_packed(const uint32_t *qsig, const void *packed, const uint32_t *dsig,
                                            int32_t k, const int64_t *cand_off, const int32_t *cand_ids,
                                            int64_t nq, float *score, int32_t *order, uint8_t *sorted_ok,
                                            void *stream);

/* polymh_rank_order -- order and sorted_ok as polymh_rank_jhat_order, from
 * scores the caller provides (e.g. the network's predictions written into
 * the collision fractions by polymh_scatter_scores).  Stream-ordered. */
polymh_status polymh_rank_order(const int64_t *cand_off, int64_t nq, const float *score,
                                int32_t *order, uint8_t *sorted_ok, void *stream);

/* polymh_rank_head_fixed -- the first M candidates of each query's order in
 * fixed slots s = q*M + t (t < M): head_query[s] = q, head_cand[s] = global
 * candidate index (int64) and head_id[s] = data polygon of the t-th best
 * candidate, or -1 in both when the query has t or fewer candidates (an empty
 * slot; polymh_pair_features gives it a zero row and polymh_scatter_scores
 * skips it).  Arrays of nq*M entries; the size does not depend on the
 * lookup's counts, so a captured graph can hold the call.  Stream-ordered. */
polymh_status polymh_rank_head_fixed(const int64_t *cand_off, const int32_t *cand_ids, int64_t nq,
                                     const int32_t *order, int32_t M, int32_t *head_query,
                                     int64_t *head_cand, int32_t *head_id, void *stream);

/* polymh_rank_reorder_head -- the order after the first min(M, C_q)
 * candidates of each query's order_in (sorted by the scores they had) were
 * given new scores in `score` (the rest unchanged): equal to
 * polymh_rank_order on the new scores, computed by sorting the re-scored
 * head and merging it with the unchanged rest (work in proportion to the
 * list, not a full sort).  1 <= M <= 64; order_out must not alias order_in.
 * Queries with sorted_ok 0 are copied unchanged.  Stream-ordered. */
polymh_status polymh_rank_reorder_head(const int64_t *cand_off, int64_t nq, const float *score,
                                      const int32_t *order_in, int32_t M, const uint8_t *sorted_ok,
                                      int32_t *order_out, void *stream);

/* polymh_mlp_score_pairs -- the scorer's prediction for pairs (li[r], ri[r])
 * in one launch: each pair's input row (as polymh_pair_features builds it)
 * assembled on chip, both hidden layers on the matrix cores (BF16 operands,
 * FP32 accumulation, BF16 activations between the layers, as
 * polymh_mlp_forward), the output layer and the sigmoid; nothing in between
 * goes through memory.
 *   lsig/rsig [.][256] uint32, lfeat/rfeat [.][12] (polymh_poly_features),
 *   li, ri [R] int32; a row with li[r] < 0 or ri[r] < 0 is skipped.
 *   out_idx [R] int64 (nullable): the prediction goes to out[out_idx[r]]
 *   (skipped where out_idx[r] < 0), e.g. into a candidate's score; without
 *   it to out[r].
 * Equal to polymh_pair_features + polymh_mlp_forward up to the order of the
 * FP32 additions of the output layer.  k must be 256; signatures and
 * weights 16-byte aligned.  Stream-ordered. */
polymh_status polymh_mlp_score_pairs(const uint32_t *lsig, const float *lfeat, const uint32_t *rsig,
                                     const float *rfeat, int32_t k, const int32_t *li, const int32_t *ri,
                                     const int64_t *out_idx, int64_t R, const float *params,
                                     const uint16_t *wbf16, float *out, void *stream);

/* polymh_rank_refine_ordered -- polymh_rank_refine without host reads, so
 * that a whole query batch (signing, lookup, scoring, ordered refinement)
 * can be captured in one graph.  The order comes from the caller
 * (polymh_rank_jhat_order or polymh_rank_order on the same scores); exactly
 * `rounds` rounds run: rounds 0 and 1 refine up to F more candidates of each
 * active query, round r >= 2 up to F * 2^(r-1), so a query still active after
 * r >= 1 rounds has had F * 2^(r-1) candidates refined (a round with no
 * active query refines nothing); then the finishing pass of
 * polymh_rank_refine completes every query still active.  With rounds = 1
 * the result equals polymh_rank_refine's with max_rounds = 1; the stop test
 * after each round is the same.
 *   counts [2] int64 device out (nullable): pairs refined, and queries the
 *   finishing pass completed.
 * ws: polymh_rank_workspace_size(nq, n_cand, F) bytes; n_cand is the size
 * of cand_ids (a bound on the lookup's total, e.g. its capacity).
 * Stream-ordered, no host reads; calls sharing ws must not overlap. */
polymh_status polymh_rank_refine_ordered(const polymh_polys *data, const polymh_polys *queries,
                                         const int64_t *cand_off, const int32_t *cand_ids,
                                         const float *score, const int32_t *order,
                                         const uint8_t *sorted_ok, int64_t nq, int64_t n_cand,
                                         int32_t topk, int32_t F, int32_t rounds, float margin,
                                         void *ws, size_t ws_bytes, int32_t *top_ids, double *top_j,
                                         int64_t *counts, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* POLYMH_H */
