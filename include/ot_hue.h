/*
 * ot_hue.h -- hue image pipeline around the 1D periodic transport (Sec. 5).
 *
 * Sec. 5 transports the normalised hue histograms of two images on the
 * circle with the periodic 1D solver of ot_dyn.h and renders the frame at
 * time t by giving the first image's hue channel the histogram h^t, keeping
 * saturation and value, through a periodic exact histogram specification
 * that the paper cites without formulas.  This library is that rendering
 * stage; the readings it takes:
 *
 *   hue       the HSV hexcone hue in [0, 1) of an 8-bit RGB pixel, in FP32
 *             from the integer channel differences (grey pixels: 0);
 *   bins      floor(hue * n) (FP32 product, at most n - 1) on n periodic bins;
 *   counts    a target density h on the bins becomes integer counts summing
 *             to the pixel count N: N h_k / sum(h) in FP64 (sum in bin order),
 *             floored, the remaining pixels one each to the largest fractional
 *             parts (equal parts: lower bin first); negative and non-finite
 *             entries count as zero, and a density without mass keeps the
 *             source counts;
 *   order     pixels strictly ordered by hue, equal hues by raster index;
 *   shift     s = lower median over the n bin edges of C_s[e] - C_t[e]
 *             (cumulative source minus target counts before bin e), which
 *             minimises the W1 cost on the circle of the rotated monotone map;
 *   map       the pixel of rank r takes the target bin holding position
 *             (r - s) mod N of the target's cumulative counts, so the output
 *             bins have exactly the target counts;
 *   render    hue' = hue + (k_out - k_src) / n wrapped into [0, 1) (FP32), RGB
 *             rebuilt from the hexcone with the pixel's max and min channels
 *             kept, rounded to 8 bits.
 * Every FP32 step is one rounded operation in a fixed order (no fused
 * multiply-add), so results are reproducible bit for bit.
 *
 * Images are device arrays of N pixels x 3 bytes (R, G, B interleaved, raster
 * order), owned by the caller.  Work is ordered on the stream given at
 * creation; one renderer is not to be called from several host threads at
 * once.  Status codes are those of ot_dyn.h.
 */
#ifndef OT_HUE_H
#define OT_HUE_H

#include "ot_dyn.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ot_hue ot_hue;

/* Bytes of device workspace a renderer for images of npix pixels (1 <= npix
 * <= 2^30) on nbins periodic hue bins (2 <= nbins <= 4096) that plans up to
 * max_frames frames per call (1 <= max_frames <= 65535) needs: about 20
 * bytes per pixel (hues, sort keys and indices, ranks), the radix sort's
 * histograms (1 KB per 8192 pixels) and 8 n + 8 bytes per frame.
 * OT_ERR_SHAPE for sizes out of range, OT_ERR_PARAM for a null bytes. */
int ot_hue_workspace_size(long long npix, int nbins, int max_frames, size_t* bytes);

/* A renderer over the caller's device workspace of ws_bytes bytes (256-byte
 * aligned; ot_hue_workspace_size): the library allocates no device memory.
 * stream: a hipStream_t (NULL = default stream).  The workspace must stay
 * allocated until ot_hue_destroy.  OT_ERR_SHAPE for sizes out of range or a
 * missing, small or misaligned workspace, OT_ERR_PARAM for a null out. */
int ot_hue_create(long long npix, int nbins, int max_frames, void* stream, void* workspace,
                  size_t ws_bytes, ot_hue** out);

void ot_hue_destroy(ot_hue* h);

/* The source image (rgb: device, npix x 3 bytes): hues, bins, bin counts, the
 * strict order (a stable radix sort of 24-bit hue keys, three 8-bit passes)
 * and each pixel's rank in it.  The renderer keeps the pointer:
 * every later frame reads the image's max and min channels from it, so it
 * must stay allocated and unchanged until the last frame rendered from it is
 * done (or the next ot_hue_set_source).  Asynchronous.  OT_ERR_PARAM for a
 * null pointer, OT_ERR_HIP if a launch fails. */
int ot_hue_set_source(ot_hue* h, const unsigned char* rgb);

/* The source's hue histogram: counts (device int32 [nbins]) and/or density
 * (device float [nbins], counts * nbins / npix: mean one, the solver's
 * convention); either may be NULL.  Asynchronous.  OT_ERR_STATE before
 * ot_hue_set_source. */
int ot_hue_histogram(ot_hue* h, int* counts, float* density);

/* Frames: the source image with its hue histogram specified to each of
 * `frames` densities (1 <= frames <= max_frames; e.g. the time levels of f
 * along a transport path).  targets: device float [frames][nbins], any scale per
 * frame.  rgb_out: device, frames x npix x 3 bytes, frame after frame (may
 * not alias the source); bins_out: device int32 [frames][npix], each pixel's
 * output bin, or NULL.  Asynchronous.  OT_ERR_STATE before ot_hue_set_source,
 * OT_ERR_PARAM for a null targets or rgb_out or frames < 1, OT_ERR_SHAPE for
 * frames > max_frames, OT_ERR_HIP if a launch fails. */
int ot_hue_render(ot_hue* h, const float* targets, int frames, unsigned char* rgb_out,
                  int* bins_out);

/* The two halves of ot_hue_render, for callers that time or reuse them:
 * ot_hue_plan computes the target counts and the shift of every frame (one
 * kernel, one block per frame); ot_hue_apply writes the frames of the last
 * plan (one pass over the pixels in raster order per frame: 14 bytes of HBM
 * traffic per pixel, 18 with bins_out).  Same arguments and status codes as
 * ot_hue_render; ot_hue_apply before a plan for the current source is
 * OT_ERR_STATE. */
int ot_hue_plan(ot_hue* h, const float* targets, int frames);
int ot_hue_apply(ot_hue* h, unsigned char* rgb_out, int* bins_out);

/* Frame `frame` of the last plan: its target counts (host int32 [nbins], or
 * NULL) and shift s (host, or NULL).  Synchronises the stream.  OT_ERR_STATE
 * before a plan, OT_ERR_PARAM for a frame out of range. */
int ot_hue_plan_info(ot_hue* h, int frame, int* counts, long long* shift);

/* Colour-space conversions of the HSV split (stateless).  ot_hue_rgb_to_hsv:
 * rgb device u8 [npix][3] to hsv device float [npix][3] = (the hue above,
 * saturation (max - min) / max, 0 for black, value max / 255).
 * ot_hue_hsv_to_rgb: the textbook hexcone inverse, h wrapped into [0, 1), s
 * and v clamped to [0, 1], a pixel with a non-finite component black, each
 * channel floor(255 c + 0.5); FP32 in a fixed order, so 8-bit colours round
 * trip exactly.  npix = 0 does nothing.  Asynchronous on `stream` (a
 * hipStream_t, NULL = default stream).  OT_ERR_PARAM for npix < 0 or a null
 * pointer with npix > 0, OT_ERR_HIP if the launch fails. */
int ot_hue_rgb_to_hsv(const unsigned char* rgb, long long npix, float* hsv, void* stream);
int ot_hue_hsv_to_rgb(const float* hsv, long long npix, unsigned char* rgb, void* stream);

#ifdef __cplusplus
}
#endif

#endif  /* OT_HUE_H */
