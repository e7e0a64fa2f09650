/*
 * findpts.h -- C ABI of the MI355X (gfx950) findpts / findpts_eval library.
 *
 * The library locates arbitrary points x* in a mesh of curved isoparametric
 * hexahedral spectral elements of order N and interpolates nodal fields at
 * the located points (Mittal, Dutta & Fischer, "Nonconforming Schwarz-
 * spectral element methods for incompressible flow", Section 2.1: findpts
 * determines the computational coordinates (e, r, s, t) of any x* and tells
 * whether it was found inside an element, on a border, or not at all;
 * findpts_eval interpolates a scalar field at those coordinates; all meshes
 * are posted at setup with a session-id discriminator and a distance-to-
 * boundary discriminator).  The processor index of the paper is dropped:
 * one GPU holds the whole mesh.
 *
 * Conventions for every call:
 *   - Pointers are DEVICE pointers (e.g. the data_ptr of a torch CUDA
 *     tensor) unless the parameter name starts with h_ (host memory).
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue on
 *     it and return without waiting unless stated otherwise.
 *   - Return value: FP_OK (0) or a negative fp_status.  Nothing aborts or
 *     exits; fp_last_error() gives a message for the calling thread.
 *   - A handle is used by one stream at a time.  Calls that overlap on one
 *     handle race (the serving layer below owns concurrency).
 *
 * Node layout of every per-element array (coordinates, fields, delta):
 *   index i + n1*(j + n1*(k + n1*e)), n1 = N + 1, i the r index (fastest),
 *   j the s index, k the t index, e the element id.
 */
#ifndef FINDPTS_H
#define FINDPTS_H

#include <stddef.h>

#ifndef FP_API
#define FP_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fp_handle fp_handle; /* opaque, owned by the library */

enum fp_status {
    FP_OK = 0,
    FP_EINVAL = -1, /* NULL / negative / non-finite argument, bad flag      */
    FP_ENOMEM = -2, /* device allocation failed                              */
    FP_EHIP = -3,   /* a HIP runtime error; text in fp_last_error()          */
    FP_ESTATE = -4, /* call not valid in the handle's current state          */
    FP_ERANGE = -5, /* N outside [1, 15], or a size beyond a stated limit    */
    FP_EBUSY = -6   /* serving: wait timed out / queue full                  */
};

/* Status code per point (Section 2.1: found inside an element, on a border,
 * or not found). */
enum fp_code {
    FP_INSIDE = 0,   /* ||x^e(r) - x*|| <= tol * h_e for the returned element */
    FP_BORDER = 1,   /* candidates exist but none holds x* within tol: the
                        closest point found (r usually on a face of [-1,1]^3) */
    FP_NOT_FOUND = 2 /* no candidate element: el = -1, rst = 0, dist2 = +inf  */
};

enum fp_precision {
    FP_PREC_FP64 = 0, /* every step in binary64                              */
    FP_PREC_MIXED = 1 /* binary32 start search and early Newton iterations;
                         final Newton steps, acceptance, classification,
                         delta and the returned residual in binary64; orders
                         N >= 8 run binary64 throughout                     */
};

/*
 * findpts_setup -- post one mesh (Section 2.1: all meshes are posted to setup
 * together with the session-id and distance discriminators).
 *   h            out: new handle (host pointer to a handle pointer).
 *   x, y, z      node coordinates, each E*(N+1)^3 doubles (layout above).
 *                Copied into handle-owned memory: the caller may free them
 *                once `stream` has passed this call.
 *   E, N         element count (>= 1) and order (1 <= N <= 15).
 *   tol          inside tolerance relative to the element size h_e (the
 *                largest per-axis extent of the element's nodes); a point is
 *                FP_INSIDE when ||x^e(r) - x*|| <= tol * h_e.  0 < tol < 1.
 *   elem_session E ints (session id per element, >= 0) or NULL (all 0).
 *   delta        E*(N+1)^3 nodal values of the distance-to-own-boundary
 *                field, or NULL (then ownership among several inside
 *                candidates goes to the smallest element id).
 *   max_points   largest npts handled in one internal pass (>= 1); larger
 *                findpts / findpts_eval calls are processed in passes.  The
 *                workspace is sized from it at setup.
 *   precision    an fp_precision value.
 * Synchronises `stream` (to size the hash grid and its workspace).
 * Errors: FP_EINVAL (NULL pointers, E < 1, bad tol/precision/max_points,
 * non-finite coordinates, detected on the device), FP_ERANGE (N), FP_ENOMEM,
 * FP_EHIP.  Inverted or degenerate elements are accepted (never rejected).
 */
FP_API int findpts_setup(fp_handle **h, const double *x, const double *y,
                  const double *z, int E, int N, double tol,
                  const int *elem_session, const double *delta,
                  int max_points, int precision, void *stream);

/*
 * findpts_update -- post new node coordinates of the same mesh (same E, N,
 * sessions, tolerance) to a set-up handle, for moving or deforming meshes,
 * whose donor elements must be found again after every timestep (Section 1,
 * the overlapping-grid challenges).  Recomputes, on the device, the packed
 * copies, element boxes and sizes, oriented boxes and the hash grid.
 *   x, y, z  node coordinates, layout as in findpts_setup (copied).
 *   delta    new distance field (E*(N+1)^3) or NULL to keep the current one;
 *            FP_ESTATE if the handle was set up without one.
 * Allocates only when the new hash grid needs more room than any earlier
 * one.  Synchronises `stream` three times.  Calls on the handle that are
 * still in flight must have finished (the serving layer must not be running
 * requests on it; requests queued on it count as in flight: if the update
 * lengthens the longest hash-cell list, such a request later fails with
 * FP_ESTATE instead of running in a workspace sized for the old mesh).  Errors: FP_EINVAL (NULL, non-finite coordinates: the
 * handle must then be updated again before use), FP_ESTATE, FP_ERANGE,
 * FP_EHIP.  Results afterwards equal those of a handle set up on the new
 * coordinates.
 */
FP_API int findpts_update(fp_handle *h, const double *x, const double *y, const double *z,
                          const double *delta, void *stream);

/*
 * findpts -- locate npts points (Section 2.1: hash lookup, elementwise
 * bounding boxes, trust-region Newton on ||x^e(r) - x*||^2 started from the
 * closest mapped GLL node; session exclusion and largest-delta ownership).
 *   pts        npts*3 doubles, x y z interleaved.
 *   pt_session npts ints or NULL.  A point tagged j >= 0 is searched only in
 *              elements whose session differs from j; a negative tag (or
 *              NULL) searches every element.
 *   code       out, npts ints (fp_code).
 *   el         out, npts ints: element id, -1 if not found.
 *   rst        out, npts*3 doubles: reference coordinates in [-1,1]^3.
 *   dist2      out, npts doubles: ||x^e(rst) - x*||^2 (+inf if not found).
 * Outputs are in the caller's point order.  Allocates nothing.  npts == 0 is
 * a no-op.  Non-finite points are FP_NOT_FOUND.
 */
FP_API int findpts(fp_handle *h, int npts, const double *pts, const int *pt_session,
            int *code, int *el, double *rst, double *dist2, void *stream);

/*
 * findpts_eval -- interpolate nfields scalar fields at located points
 * (Section 2.1: f(e, r) = sum_ijk F^e_ijk h_i(r) h_j(s) h_k(t)).
 *   code, el, rst  as returned by findpts (code FP_NOT_FOUND gives NaN).
 *   h_fields       HOST array of nfields device pointers, each to
 *                  E*(N+1)^3 doubles; borrowed for the stream-ordered call.
 *   out            out, nfields*npts doubles, field-major: out[f*npts + p].
 * Allocates nothing.  Errors: FP_EINVAL (NULL, nfields < 1, an element id
 * out of range is NOT checked on the device: el must come from findpts).
 */
FP_API int findpts_eval(fp_handle *h, int npts, const int *code, const int *el,
                 const double *rst, int nfields,
                 const double *const *h_fields, double *out, void *stream);

/*
 * findpts_eval_noalloc -- findpts_eval for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same interpolation, bit-identical
 * results, but the point grouping uses a file-scope device array of 32 MiB
 * per GPU (held by the library until the process ends) instead of the
 * handle's workspace.  Calls no hipMalloc/hipFree and creates no events.
 * Arguments as findpts_eval; any npts (it runs in passes).  FP_ERANGE if the
 * mesh has more elements than the array's per-element counters allow (about
 * 4.19 million).  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads, other handles) race and
 * must be serialised by the caller; each call clears what it uses.
 */
FP_API int findpts_eval_noalloc(fp_handle *h, int npts, const int *code, const int *el,
                                const double *rst, int nfields,
                                const double *const *h_fields, double *out, void *stream);

/* Switch precision (fp_precision) for later calls; FP_EINVAL if unknown.
 * Mixed precision needs no new allocation: the binary32 geometry copy is
 * built at setup. */
FP_API int findpts_set_precision(fp_handle *h, int precision);

/*
 * findpts_stats -- cumulative counters since setup (or the last reset),
 * written to host memory (6 values): h_counts[0] = (point, element) pairs
 * solved by Newton, h_counts[1] = Newton iterations, h_counts[2] = points
 * located, h_counts[3] = candidates of the method (hash cell + axis-aligned
 * element box + session test; the library solves only those whose oriented
 * box also holds the point, then redoes points left without an inside
 * element with all of them), h_counts[4] and h_counts[5] = the pairs and
 * iterations of [0] and [1] that the first-pass Newton launches solved (the
 * rest belong to the second passes).  Synchronises the device.  reset != 0
 * zeroes them afterwards.
 */
FP_API int findpts_stats(fp_handle *h, long long *h_counts, int reset);

/*
 * Per-kernel timing with HIP events recorded on the call's stream.
 * findpts_timing(h, 1) turns recording on; findpts_timing_read fills
 * h_ms[5] with the summed milliseconds and h_n[5] with the launch counts of
 * [0] the first-pass Newton (locate) kernel, [1] the interpolation kernel,
 * [2] whole findpts calls, [3] whole findpts_eval calls, [4] the
 * second-pass Newton kernel, then clears them.
 * findpts_timing_read synchronises the recorded events.
 */
FP_API int findpts_timing(fp_handle *h, int enable);
FP_API int findpts_timing_read(fp_handle *h, double *h_ms, long long *h_n);

/*
 * Read back setup products to host memory (parity tests):
 * h_bbox E*6 doubles (xmin xmax ymin ymax zmin zmax), h_size E doubles (h_e);
 * h_nc[3] hash cells per axis, h_lo[3] grid origin, h_dx[3] cell size,
 * h_meta[3] = {cell count, stored cell entries, largest cell list}.
 * findpts_get_cells copies cell_off (ncell+1 ints) and cell_el (nnz ints).
 * Each synchronises the device.
 */
FP_API int findpts_get_bbox(fp_handle *h, double *h_bbox, double *h_size);
FP_API int findpts_get_hash(fp_handle *h, int *h_nc, double *h_lo, double *h_dx,
                     long long *h_meta);
FP_API int findpts_get_cells(fp_handle *h, int *h_cell_off, int *h_cell_el);

/* Device bytes held by the handle (mesh copy, hash, workspace). */
FP_API int findpts_footprint(const fp_handle *h, size_t *h_bytes);

/* Release the handle after work already enqueued has finished (device-wide
 * synchronisation).  NULL is a no-op. */
FP_API int findpts_free(fp_handle *h);

/*
 * Two dimensions: meshes of curved quadrilateral spectral elements of order
 * N (the method of Section 2.1 on the reference square [-1,1]^2; the
 * paper's Figs. 1 and 6 are two-dimensional overlapping meshes).  Node (i, j)
 * of element e is at flat index i + (N+1) (j + (N+1) e).  Readings as in three
 * dimensions: Bernstein-hull boxes with the same margin, h_e = largest
 * per-axis node extent, closest-node start (smallest index on ties), the same
 * trust-region rules on [-1,1]^2, the same classification and selection (and,
 * as in 3D, an oriented-box first round that never changes a result).
 *
 * findpts2_setup -- like findpts_setup: x, y hold E*(N+1)^2 doubles each,
 * elem_session E ints or NULL, delta E*(N+1)^2 doubles or NULL; all device
 * pointers, copied.  Synchronises `stream`.  Errors: FP_EINVAL, FP_ERANGE,
 * FP_ENOMEM, FP_EHIP.
 */
typedef struct fp2_handle fp2_handle; /* opaque, owned by the library */
FP_API int findpts2_setup(fp2_handle **h, const double *x, const double *y, int E, int N,
                          double tol, const int *elem_session, const double *delta,
                          int max_points, void *stream);

/*
 * findpts2 -- locate npts points: pts npts*2 doubles (x y interleaved),
 * pt_session npts ints or NULL, out code / el (npts ints), rs (npts*2
 * doubles: r, s), dist2 (npts doubles), as for findpts.  Allocates nothing;
 * calls on one handle must not overlap (they share its workspace).
 */
FP_API int findpts2(fp2_handle *h, int npts, const double *pts, const int *pt_session,
                    int *code, int *el, double *rs, double *dist2, void *stream);

/*
 * findpts2_eval -- f(e, r, s) = sum_ij F^e_ij h_i(r) h_j(s) for nfields
 * fields (host array of device pointers, each E*(N+1)^2 doubles) at located
 * points; out nfields*npts doubles, field-major; FP_NOT_FOUND gives NaN.
 * Allocates nothing; shares the handle's workspace with findpts2.
 */
FP_API int findpts2_eval(fp2_handle *h, int npts, const int *code, const int *el,
                         const double *rs, int nfields, const double *const *h_fields,
                         double *out, void *stream);

/* Since setup (h_counts: 3 host long longs): pairs solved, Newton
 * iterations, and the method's candidates (hash + axis-aligned box +
 * session test); reset != 0 zeroes them.  Synchronous. */
FP_API int findpts2_stats(fp2_handle *h, long long *h_counts, int reset);

/* Element boxes (host E*4 doubles: xmin xmax ymin ymax) and sizes h_e (host E
 * doubles).  Synchronous. */
FP_API int findpts2_get_bbox(fp2_handle *h, double *h_bbox, double *h_size);

/* Release a handle (NULL is a no-op); waits for the device first. */
FP_API int findpts2_free(fp2_handle *h);

/* Message of the last error on the calling thread ("" if none). */
FP_API const char *fp_last_error(void);

/*
 * fp_copy -- plain device-to-device copy kernel of `bytes` bytes (multiple
 * of 16, 16-byte aligned pointers), used to calibrate bandwidth and hardware
 * byte counters against a kernel of known traffic.  Enqueued on `stream`.
 */
FP_API int fp_copy(const void *src, void *dst, size_t bytes, void *stream);

/*
 * Interface data (what the Schwarz exchange does with interpolated values).
 *
 * fp_flux_correct -- mass-flux correction of boundary velocity data of one
 * subdomain (Section 2.2, Eqs. 1-3): with F the boundary flux of the
 * tentative velocity (sum of w_p u_p . n_p over all npts boundary points)
 * and A the area of the interpolated part (sum of w_p n_p . n_p over the
 * points with iface[p] != 0), gamma = -F / A (0 if A = 0) and
 * u_p += gamma n_p on the interpolated points, so that the corrected data
 * has zero net flux.
 *   w      npts surface quadrature weights (area elements).
 *   n      unit outward normals, component c of point p at n[c*ldn + p]
 *          (ldn >= npts).
 *   iface  npts ints (non-zero: interpolated point) or NULL (all are).
 *   u      velocity, component c of point p at u[c*ldu + p] (ldu >= npts;
 *          the layout findpts_eval writes, ldu = its npts, so that one
 *          subdomain's points are a slice); corrected in place.
 *   work   device buffer of FP_FLUX_WORK doubles; work[0] receives gamma.
 * Sums in binary64 with a fixed reduction order (bit-reproducible).
 * Allocates nothing.  Errors: FP_EINVAL.
 *
 * fp_extrapolate -- m-th order extrapolation in time of interface data
 * (Section 2: lagged data extrapolated to order m, 1 <= m <= 3, constant time
 * step): out = sum_q beta_q hist[q], weights (1), (2, -1), (3, -3, 1).
 *   h_hist  HOST array of `order` device arrays of n doubles, most recent
 *           first.  out may alias none of them.
 */
#define FP_FLUX_WORK 1024
FP_API int fp_flux_correct(int npts, const double *w, const double *n, long long ldn,
                           const int *iface, double *u, long long ldu, double *work,
                           void *stream);
FP_API int fp_extrapolate(long long n, int order, const double *const *h_hist, double *out,
                          void *stream);

/*
 * Serving layer.  Not a step of the paper's method: Section 2.1 runs one
 * findpts (and findpts_eval per field) per Schwarz exchange over all
 * interface points of a session; this layer serves many such calls, on many
 * resident meshes, as they arrive.
 *
 *   - Meshes stay resident: fps_add_mesh registers a set-up handle and its
 *     fields (borrowed, not copied; they must outlive the serving object).
 *   - A request is (mesh, npts points, optional point sessions, a list of
 *     field ids).  Its workspace (the pair arrays of findpts and the
 *     element counters of both calls, sized for min(npts, 2^20) points per
 *     pass) is carved from one device arena of `hbm_budget_bytes`, reserved
 *     at fps_create.  A request is admitted when a slot (a HIP stream of the
 *     serving object) is free and its workspace fits in the arena; until
 *     then it waits in submission order (a later request that fits may pass
 *     a waiting one, at most 8 times in a row).  Admitted requests run
 *     concurrently on their slots and release slot and workspace when their
 *     stream completes; waiting requests are then admitted.
 *   - Results equal those of findpts + findpts_eval on the request alone
 *     (every point's result depends only on that point and the mesh).
 *   - Latency of a request = host time from fps_submit to the completion of
 *     its last kernel (a host callback on its stream).
 *
 * All request buffers are device pointers owned by the caller: pts (npts x
 * 3), pt_session (npts or NULL), code/el (npts), rst (npts x 3), dist2
 * (npts), out (nfields x npts, field-major; may be NULL when nfields = 0).
 * Inputs must be ready (their producing stream synchronised) before
 * fps_submit; no buffer may be touched until fps_wait returns for the
 * ticket.  Precision is the handle's (findpts_set_precision).
 *
 * fps_create      budget in bytes (> 0), slots in [1, 16].
 * fps_add_mesh    fields: nfields device pointers (E x V doubles each), may
 *                 be 0; *mesh_id receives the id (0, 1, ...).
 * fps_submit      returns FP_ENOMEM if even a 256-point pass of the request
 *                 exceeds the budget, FP_EINVAL for bad ids or sizes;
 *                 *ticket receives a positive id.  Never blocks on the GPU.
 * fps_wait        blocks until the request completed (FP_OK or its error),
 *                 FP_EBUSY if timeout_s (>= 0; < 0 = forever) passes first.
 *                 A ticket can be waited for once.  FP_ESTATE: the mesh was
 *                 updated while the request was queued and its longest
 *                 hash-cell list grew past what the workspace was sized for.
 * fps_latency     p50 / p99 latency (seconds) of the requests completed
 *                 since the last reset, and their points per second over the
 *                 span from the first submission to the last completion;
 *                 h_info[6] (may be NULL): completed requests, requests
 *                 waiting, requests running, peak concurrent requests, peak
 *                 arena bytes in use, admissions that had to wait.
 * fps_destroy     waits for every submitted request, then frees streams and
 *                 the arena.  Handles and fields are not freed.
 */
typedef struct fps fps;

FP_API int fps_create(fps **s, size_t hbm_budget_bytes, int slots);
FP_API int fps_add_mesh(fps *s, fp_handle *h, const double *const *h_fields, int nfields,
                        int *h_mesh_id);
FP_API int fps_submit(fps *s, int mesh_id, int npts, const double *pts, const int *pt_session,
                      int nfields, const int *h_field_ids, int *code, int *el, double *rst,
                      double *dist2, double *out, long long *h_ticket);
FP_API int fps_wait(fps *s, long long ticket, double timeout_s);
FP_API int fps_latency(fps *s, double *h_p50_s, double *h_p99_s, double *h_pts_per_s,
                       long long *h_info, int reset);
FP_API int fps_destroy(fps *s);

#ifdef __cplusplus
}
#endif

#endif /* FINDPTS_H */
