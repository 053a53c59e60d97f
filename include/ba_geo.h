/*
 * ba_geo.h -- C ABI of the footprint and patch-transfer kernels of the
 * MI355X (gfx950) cluster bundle-adjustment library (libba.so).
 *
 * These are the steps on either side of the cluster solve that Sec. 3.1 of
 * the paper describes: each image's footprint on the digital surface model
 * (the four image corners' rays intersected with the DSM), the comparison of
 * footprints that finds overlapping images, within and across flight strips,
 * for a cluster's membership, and the GNSS/IMU-based patch transfer of
 * Eq. (3), which carries each patch centre of an image into the images that
 * overlap it, with the patch's depth taken from the DSM (Eq. 3 with a known
 * elevation model instead of flat ground) and re-initialisation at the
 * opposite edge for patches that leave the image.
 *
 * Conventions (as in ba.h)
 *   R camera->world rotation, row-major 3x3; T projection centre; camera z
 *   forward, image y down; pixel origin at the image corner.  The camera is
 *   the pinhole K of Eq. (3): focal length f and principal point (cx, cy) in
 *   pixels, no distortion.
 *   DSM: heights on raster nodes (x0 + i cell, y0 + j cell), i < nx, j < ny,
 *   world x, y and height in metres, the same metric frame as the poses (an
 *   ENU frame, or ECEF rotated to a local tangent plane).  Between nodes the
 *   surface is the bilinear interpolation of the four surrounding nodes;
 *   positions outside the raster are clamped to it.
 *   Pixel ray: X(lam) = T + lam R K^-1 (u, v, 1)^T; lam is the depth along
 *   the camera axis (the nominal depth of Eq. 3).
 *   Ray / DSM intersection: the first lam > 0 where the ray meets the
 *   surface.  The ray is sampled between the depths where it passes the
 *   raster's highest and lowest nodes, in n equal steps with n =
 *   ceil(horizontal travel / half a cell), at least 1 and at most 65536;
 *   the first sample at or below the surface and the sample before it
 *   bracket the crossing, which a safeguarded Illinois (modified regula
 *   falsi) iteration narrows to 1e-12 of the depth (at most 64 steps); the
 *   result is the bracket's final upper end.  A ray that does not descend
 *   misses.
 *
 * Memory and threads
 *   Every array is a HOST pointer owned by the caller, read (inputs) or
 *   written (outputs) during the call only.  The context owns its device
 *   memory: the DSM, copied at creation, and work buffers that grow to the
 *   largest call so far and are freed by ba_geo_destroy.  Calls are
 *   synchronous (they return after the results are on the host) and run on
 *   one HIP stream of the context; a context must not be used from two
 *   threads at once.
 *
 * Errors: the BA_E_* codes of ba.h; ba_geo_last_error gives the message of
 * the last failed call on a context.
 */
#ifndef BA_GEO_H
#define BA_GEO_H

#include <stddef.h>
#include <stdint.h>

#include "ba.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_geo ba_geo;

/* A digital surface model raster (Sec. 3.1: TanDEM-X, 12 m; SRTM, 30 m). */
typedef struct {
  int32_t nx, ny;               /* nodes along x and y; both >= 2 */
  double x0, y0;                /* world position of node (0, 0) */
  double cell;                  /* node spacing (m), > 0 */
  const float* h;               /* [ny][nx] heights (m), row j holds y = y0 + j cell; finite */
} ba_dsm;

/* The pinhole camera K of Eq. (3) and the image size. */
typedef struct {
  double f, cx, cy;             /* focal length and principal point (px); f > 0 */
  int32_t width, height;        /* image size (px); > 0 */
} ba_pinhole;

/* Flags of ba_patch_transfer, and status of ba_footprints. */
enum ba_geo_flag { BA_GEO_OK = 0, BA_GEO_MISS = 1, BA_GEO_REINIT = 2 };

/* Create a context on `device` holding a device copy of the DSM.
 * Errors: BA_E_ARG (NULL, nx or ny < 2, cell <= 0, non-finite heights),
 * BA_E_NOMEM, BA_E_DEVICE. */
int ba_geo_create(int32_t device, const ba_dsm* dsm, ba_geo** out);

/* Free the context and its device memory. */
int ba_geo_destroy(ba_geo* ctx);

/* Footprints of n images (Sec. 3.1): the ground points where the rays of the
 * image corners (0, 0), (W, 0), (W, H), (0, H) and of the image centre
 * (W/2, H/2) meet the DSM.  R [9n], T [3n] the images' poses.  Writes
 * ground [15n] (per image five points x, y, z in that order) and status [n]
 * (BA_GEO_OK, or BA_GEO_MISS when one of the image's rays misses; its point
 * is then NaN).  n = 0 does nothing.
 * Errors: BA_E_ARG (NULL arrays with n > 0, n < 0, bad camera), BA_E_NOMEM,
 * BA_E_DEVICE. */
int ba_footprints(ba_geo* ctx, int32_t n, const double* R, const double* T, const ba_pinhole* cam,
                  double* ground, int32_t* status);

/* Overlap of every pair of n footprints (Sec. 3.1: overlapping images,
 * within and across strips, are found by comparing their projected
 * footprints): the area (m^2) of the intersection of the two corner
 * quadrilaterals in the horizontal plane.  ground [15n] as written by
 * ba_footprints (the corners' x, y are used; the quadrilaterals must be
 * convex).  Writes area [n(n-1)/2], the pairs (i, j), i < j, row by row:
 * pair (i, j) at i n - i(i+1)/2 + j - i - 1.  An area is NaN when either
 * quadrilateral is missing (NaN) or not convex.
 * Errors: BA_E_ARG (NULL arrays with n > 1, n < 0, n > 65536), BA_E_NOMEM,
 * BA_E_DEVICE. */
int ba_footprint_overlaps(ba_geo* ctx, int32_t n, const double* ground, double* area);

/* How ba_cluster_membership forms a cluster (Sec. 3.1-3.2). */
typedef struct {
  int32_t max_back;             /* in-strip predecessors of the triggering image, at most (>= 0) */
  int32_t free_back;            /* in-strip predecessors within this many steps stay free (>= 0) */
  int32_t max_cams;             /* images per cluster, at most (1..64) */
  int32_t min_cams;             /* a triggering image with fewer forms no cluster (1..max_cams) */
  double min_overlap;           /* two footprints overlap when their intersection covers at least
                                   this fraction of the smaller one (0..1) */
} ba_cluster_rule;

/* Cluster membership from footprints (Sec. 3.1: the images that overlap an
 * image, within its strip and across strips, are found by comparing
 * footprints; Sec. 3.2: each new image is adjusted in a cluster with its
 * overlapping images, the part adjusted before held fixed).  n images in
 * flight order with footprints ground [15n] (as ba_footprints writes them)
 * and strip [n] (the strip of each image).  Two images overlap when both
 * footprints exist (convex corner quadrilaterals, finite centre point) and
 * the area of their intersection (as ba_footprint_overlaps computes it) is
 * at least rule->min_overlap times the smaller footprint's area.  The
 * cluster triggered by image i holds: i; its in-strip predecessors i-1,
 * i-2, ... (at most max_back, each in i's strip and overlapping the image
 * after it); then the earlier images (index < i) of other strips that
 * overlap i, nearest first by the horizontal distance between footprint
 * centres (ties: lower index); the list cut at max_cams.  With fewer than
 * min_cams images image i forms no cluster.  The fixed images are the other
 * strips' and the in-strip predecessors more than free_back steps back.
 * Writes, for each image i, count [n] (its cluster's size, 0 for none),
 * members [n][max_cams] (the cluster's images in ascending order, -1
 * after the last) and fixed [n][max_cams] (1 = held fixed, aligned with
 * members).  Integer results; calls are synchronous.
 * Errors: BA_E_ARG (NULL arrays with n > 0, n outside 0..65536, a bad rule),
 * BA_E_NOMEM, BA_E_DEVICE. */
int ba_cluster_membership(ba_geo* ctx, int32_t n, const double* ground, const int32_t* strip,
                          const ba_cluster_rule* rule, int32_t* members, uint8_t* fixed, int32_t* count);

/* GNSS/IMU patch transfer, Eq. (3), with the patch depth from the DSM:
 * for each pair p = (src, dst) in pairs [2 n_pairs] (image indices into R, T)
 * and each patch centre q of uv0 [2 n_patch] (pixel coordinates in the source
 * image), the ground point of the source ray through q is projected into
 * image dst:  p^(dst) = pi(K R_dst^T ((T_src + lam R_src K^-1 q) - T_dst)).
 * A result outside [0, W) x [0, H) is re-initialised at the opposite edge
 * (Sec. 3.1): each coordinate is wrapped modulo the image size.
 * R [9 n_img], T [3 n_img].  Writes uv [n_pairs][n_patch][2], flags
 * [n_pairs][n_patch] (BA_GEO_OK, BA_GEO_REINIT, or BA_GEO_MISS when the
 * source ray misses the DSM or the ground point is not in front of image
 * dst: uv NaN), and, if lam is not NULL, lam [n_img][n_patch]: the depth of
 * each patch of each image (NaN for images that are no pair's source).
 * Errors: BA_E_ARG (NULL arrays with work to do, negative counts, an index
 * out of range, bad camera), BA_E_NOMEM, BA_E_DEVICE. */
int ba_patch_transfer(ba_geo* ctx, int32_t n_img, const double* R, const double* T, int32_t n_patch,
                      const double* uv0, int32_t n_pairs, const int32_t* pairs, const ba_pinhole* cam,
                      double* uv, int32_t* flags, double* lam);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the patch
 * transfer of ba_patch_transfer with device-resident inputs and outputs, and
 * no device allocation by the call.  R [9 n_img], T [3 n_img], uv0
 * [2 n_patch], uv [n_pairs][n_patch][2] and flags [n_pairs][n_patch] are
 * DEVICE pointers on the context's device, owned by the caller; pairs
 * [2 n_pairs] and cam are host memory.  The results equal ba_patch_transfer's
 * bit for bit (the same kernels); the depths (lam) are not returned, and a
 * non-finite patch centre gives BA_GEO_MISS instead of an error.  The work
 * buffers (the source list, the pairs grouped by source and the ground point
 * of every source patch) live in a 16 MiB array inside the library that each
 * device holds for the life of the process; a call that needs more
 * (32 bytes per source image and patch, plus 4 bytes per source and 8 per
 * pair, each part rounded up to 256 bytes) is refused with BA_E_ARG before
 * anything runs.  Every call on a device shares that array: calls that
 * overlap on one device (two threads, or two contexts) race.  The call is
 * synchronous on the context's stream; ba_geo_last_ms times it.  It calls no
 * hipMalloc, hipFree or other allocating routine.
 * Errors: BA_E_ARG (NULL arrays with work to do, negative counts, an index
 * out of range, bad camera, scratch too small), BA_E_DEVICE. */
int ba_patch_transfer_noalloc(ba_geo* ctx, int32_t n_img, const double* R, const double* T, int32_t n_patch,
                              const double* uv0, int32_t n_pairs, const int32_t* pairs, const ba_pinhole* cam,
                              double* uv, int32_t* flags);

/* Device time (ms) of the kernels of the last successful ba_footprints,
 * ba_footprint_overlaps or ba_patch_transfer call on the context, measured
 * by HIP events around its launches (transfers excluded): total_ms over all
 * of the call's kernels, last_ms of its last kernel alone (the projection of
 * ba_patch_transfer; the whole call for the one-kernel calls).  Either
 * pointer may be NULL. */
int ba_geo_last_ms(ba_geo* ctx, double* total_ms, double* last_ms);

/* Message of the last failed call on the context. */
const char* ba_geo_last_error(ba_geo* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BA_GEO_H */
