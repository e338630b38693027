/* sphmi.h: C ABI of the MI355X (gfx950) SPH hot-path library libsphmi.so.
 *
 * The library implements the per-particle compute kernels of the SPH code
 * studied in "Compiler-supported reduced precision and AoS-SoA
 * transformations for heterogeneous hardware" (Radtke & Weinzierl):
 *   - cell binning of an array-of-structs particle set,
 *   - the AoS->SoA gather with narrowing and storage below IEEE double
 *     (operators N, C, U of Sec. 4.1) and its inverse,
 *   - the quadratic density and force kernels (Sec. 2.1, Eq. density and
 *     Eq. momentum; Alg. 1 CallQuadratic),
 *   - the linear kick/drift kernel (Alg. 1 CallLinear),
 *   - plain-AoS forms of the three kernels (the GPU-native variant of
 *     Sec. 4.3, Eq. gpu_native),
 *   - FP64 conservation reductions.
 *
 * Conventions
 *   - Every entry point returns sph_status: 0 (SPH_OK) or a negative error.
 *     sph_last_error() returns a thread-local message describing the last
 *     failure on the calling thread; it stays valid until the next call on
 *     that thread. No C++ exception and no HIP error crosses this boundary.
 *   - Pointers are device pointers unless a parameter says "host". The
 *     caller allocates and owns every buffer, including workspaces; the
 *     library allocates no persistent device memory and keeps no global
 *     mutable state.
 *   - Device work is enqueued on the caller's stream and the call returns
 *     without waiting. Kernel-side conditions (NaN positions, smoothing
 *     lengths too large for the cell list) are OR-ed into the optional
 *     device word sph_cells.status; the caller reads it after the stream
 *     has reached the call. Argument errors are detected on the host before
 *     anything is enqueued.
 *   - Particle arrays in an sph_soa are indexed by sorted slot k
 *     (0 <= k < n): slot k holds input particle perm[k], and slots of one
 *     cell are contiguous.
 *   - Floating-point arithmetic and accumulation in the pair kernels is
 *     FP32; positions are FP64 in the AoS record and in the kick view.
 */
#ifndef SPHMI_H
#define SPHMI_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPH_ABI_VERSION 11

typedef int32_t sph_status;
enum {
  SPH_OK = 0,
  SPH_E_INVALID = -1,      /* bad pointer, enum, size or layout            */
  SPH_E_RANGE = -2,        /* n_c < 3, cell count overflow                 */
  SPH_E_NOMEM = -3,        /* workspace smaller than required              */
  SPH_E_HIP = -4,          /* HIP runtime error (message has the details)  */
  SPH_E_UNSUPPORTED = -5   /* valid but unsupported combination            */
};

/* bits OR-ed into *sph_cells.status by kernels */
enum {
  SPH_FLAG_BAD_POSITION = 1,   /* a position was NaN or infinite            */
  SPH_FLAG_H_TOO_LARGE = 2     /* some H_i exceeded the cell side: neighbour
                                  sums may miss particles                   */
};

/* storage formats (Table 2: 64, 32 and 16 total bits; plus bfloat16) */
typedef enum {
  SPH_F64 = 0, SPH_F32 = 1, SPH_F16 = 2, SPH_BF16 = 3, SPH_I32 = 4,
  SPH_TRUNC = 0x100
} sph_dtype;
/* truncate_mantissa storage of T bits in total (Sec. 3.2, Table 2), for
 * the narrowed SoA views, 9 <= T <= 32: the top T bits of the value's IEEE
 * single (T > 16) or half (T <= 16) pattern, the rest of the mantissa cut
 * off (toward zero); T = 32 and 16 are single and half. The codes form one
 * bitstream per field: value k at bits [kT, kT + T) of little-endian 32-bit
 * words. A field buffer holds sph_storage_bytes(n, dtype) bytes. */
#define SPH_TRUNC_BITS(T) (SPH_TRUNC + (T))

/* ------------------------------------------------------------------ */
/* AoS record description (Table 1 fields; "all variants derive from   */
/* one struct declaration", Sec. 4.1). X, V, A are 3 consecutive        */
/* elements. X must be SPH_F64; the other floating fields SPH_F32 or    */
/* SPH_F64; NNGB, NFORCE, CELL are SPH_I32. Unused fields: offset       */
/* SPH_ABSENT. Every present field must lie inside the stride and be    */
/* aligned to its element size.                                         */
/* ------------------------------------------------------------------ */
enum {
  SPH_A_X = 0, SPH_A_V, SPH_A_A, SPH_A_M, SPH_A_H, SPH_A_U, SPH_A_RHO, SPH_A_P,
  SPH_A_C, SPH_A_DU, SPH_A_RHO_DH, SPH_A_WCOUNT, SPH_A_F, SPH_A_VSIG,
  SPH_A_NNGB, SPH_A_NFORCE, SPH_A_CELL, SPH_A_NFIELDS
};
#define SPH_ABSENT 0xffffffffu

typedef struct {
  uint32_t stride;                     /* bytes per record, multiple of 8 */
  uint32_t offset[SPH_A_NFIELDS];      /* byte offset or SPH_ABSENT      */
  int32_t dtype[SPH_A_NFIELDS];        /* sph_dtype of each element      */
} sph_aos_layout;

/* ------------------------------------------------------------------ */
/* Cell list (uniform grid over the periodic unit box) with an optional */
/* finer sub-cell order inside each cell (R = 2^sub_bits sub-cells per  */
/* axis; the sub-cell of x along an axis is floor(x * n_c * R) - c * R, */
/* clamped to [0, R-1]; a cell's particles are ordered by the Morton    */
/* code of their sub-cell (bit b of sx at 3b, sy at 3b+1, sz at 3b+2),  */
/* then by input index).                                                */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t n;              /* particles                                   */
  int32_t n_c;            /* cells per axis, >= 3; cell side 1/n_c must   */
                          /* be >= every support radius H = gamma_k h     */
  int32_t sub_bits;       /* 0..3; n_c^3 * 8^sub_bits < 2^31             */
  int32_t reserved;       /* must be 0                                    */
  int32_t *cell_start;    /* [n_c^3 + 1] slots of cell c: [start[c],     */
                          /* start[c+1])                                  */
  int32_t *perm;          /* [n] input index of sorted slot k             */
  int32_t *cell;          /* [n] cell id cx + n_c (cy + n_c cz) of slot k */
  int32_t *sub_start;     /* [n_c^3 R^3 + 1] slots of sub-cell key        */
                          /* cell * R^3 + morton; required when           */
                          /* sub_bits > 0, else may be NULL               */
  float *hmax;            /* [n_c^3] largest h of each cell (written by   */
                          /* sph_bin when the layout has H; may be NULL)  */
  int32_t *status;        /* [1] optional (may be NULL) SPH_FLAG_* word   */
  uint64_t *tally;        /* [2] optional (may be NULL) work counters of  */
                          /* the pair loops: [0] += candidate pair tests  */
                          /* (particles of a chunk times the candidates   */
                          /* staged for it), [1] += candidates gathered   */
                          /* from the candidate ranges                    */
  int32_t *rebin;         /* [2] optional (may be NULL) validity of the    */
                          /* cell list across steps: [0] counts particles */
                          /* that left their cell or sub-cell since the   */
                          /* list was built (pass &rebin[0] as moved to   */
                          /* sph_kick_drift / _aos); sph_bin keeps the    */
                          /* list when [0] == 0 and otherwise rebuilds it */
                          /* and sets [0] = 0; it sets [1] = 1 when it    */
                          /* rebuilt, 0 when it kept the list, and        */
                          /* sph_worklist / _occupancy rebuild a work     */
                          /* list only when [1] != 0. The caller sets [0] */
                          /* nonzero before the first sph_bin and         */
                          /* whenever the records change otherwise (new   */
                          /* positions or h, another n_c or sub_bits).    */
} sph_cells;

/* Work list of the pair kernels for a launch over all cells of uneven
 * occupancy: (cell, first slot) items of at most `ti` particles each, built
 * by sph_worklist from a cell list, split into 8 contiguous ranges (one per
 * XCD) of about equal estimated cost. The caller allocates `buf` with at
 * least sph_worklist_size(n, n_c, ti) bytes. A work list describes the cell
 * list it was built from: rebuild it after every sph_bin. `sched` picks how
 * workgroups take items; it changes only the timing, never a result.
 * max_cells > 1 (merged items) changes the frame in which the positions of
 * a merged cell's particles are taken (the group's first cell): results
 * then differ from those of an unmerged list by FP32 rounding only. */
enum {
  SPH_SCHED_GRID = 0,     /* one workgroup per item, dispatched by the hardware */
  SPH_SCHED_STATIC = 1,   /* persistent grid, items of an XCD's range in turn  */
  SPH_SCHED_DYNAMIC = 2   /* persistent grid, per-XCD queues with stealing      */
};
typedef struct {
  int32_t ti;             /* particles per item (the tile's ti)           */
  int32_t sched;          /* SPH_SCHED_*                                  */
  void *buf;              /* device buffer: queues, item count, items     */
  size_t bytes;           /* size of buf                                  */
  int32_t max_cells;      /* 0 or 1: an item holds slots of one cell; 2..4: */
                          /* an item may hold all slots of up to that many */
                          /* x-adjacent cells of one row of a 4x4x4 brick  */
                          /* (in the same occupancy class) whose particles */
                          /* fit the tile, so sparse cells share full      */
                          /* tiles and one candidate neighbourhood; needs  */
                          /* n_c^3 < 2^29; only sph_worklist /             */
                          /* _occupancy build merged items                 */
  int32_t reserved;       /* must be 0                                      */
} sph_work;

/* ------------------------------------------------------------------ */
/* SoA buffers (sorted-slot order). One struct names every array a       */
/* kernel may touch; each entry point lists the ones it reads/writes,   */
/* the rest may be NULL.                                                */
/* ------------------------------------------------------------------ */
enum {
  /* narrowed views for the pair kernels, stored in sph_precision formats */
  SPH_S_OFF_X = 0, SPH_S_OFF_Y, SPH_S_OFF_Z,  /* x - cell origin  (pos)   */
  SPH_S_VQ_X, SPH_S_VQ_Y, SPH_S_VQ_Z,         /* velocity         (vel)   */
  SPH_S_M, SPH_S_H, SPH_S_U,                  /* m, h, u          (mhu)   */
  /* kick view: absolute FP64 positions, FP32 velocity and energy        */
  SPH_S_X_X, SPH_S_X_Y, SPH_S_X_Z,            /* double                   */
  SPH_S_V_X, SPH_S_V_Y, SPH_S_V_Z, SPH_S_UK,  /* float                    */
  /* density outputs (float; NNGB int32)                                  */
  SPH_S_RHO, SPH_S_WCOUNT, SPH_S_RHO_DH, SPH_S_F, SPH_S_P, SPH_S_C, SPH_S_NNGB,
  /* force outputs (float; NFORCE int32)                                  */
  SPH_S_A_X, SPH_S_A_Y, SPH_S_A_Z, SPH_S_DU, SPH_S_VSIG, SPH_S_NFORCE,
  /* anchor sub-cell code of each slot (uint8; see sph_precision.pos_anchor) */
  SPH_S_ANC,
  SPH_S_NFIELDS
};

typedef struct {
  void *f[SPH_S_NFIELDS];
} sph_soa;

/* storage precision of the narrowed views. pos, vel and mhu: SPH_F32 |
 * SPH_F16 | SPH_BF16 | SPH_TRUNC_BITS(T). A field with scale s is stored as
 * Q(RNE32(v) * 2^s) and read back as stored * 2^-s (|s| <= 64; exact
 * power-of-two scaling keeps small masses and smoothing lengths in the
 * normal range of FP16); Q rounds to nearest even for the IEEE formats and
 * cuts the mantissa for SPH_TRUNC_BITS. Truncated formats are written by
 * sph_convert only (records of at most 208 bytes), and read by the kernels'
 * run-time format path.
 *
 * Positions are stored as offsets from an anchor that the kernels rebuild
 * from the cell id (Sec. 3.2: a value kept as a quantised difference from an
 * anchor). With x_w the wrapped position of a particle in cell c (per axis):
 *   SPH_ANCHOR_CORNER:  anchor = c / n_c;
 *   SPH_ANCHOR_SUB(b):  anchor = (c 2^b + a + 1/2) / (n_c 2^b), the centre
 *     of the particle's sub-cell of side 1/(n_c 2^b), with the sub-cell
 *     index a = floor(x_w n_c 2^b) - c 2^b clamped to [0, 2^b - 1]
 *     (b = 0: the cell centre; 0 <= b <= 2);
 * all in FP64; OFF = Q_pos(RNE32(x_w - anchor)). Every halving of the
 * anchor's reach halves the largest stored offset and so the position
 * error of a floating storage format. For b >= 1 the SoA field ANC holds
 * each slot's code a_x + 4 a_y + 16 a_z (uint8), written with the offsets
 * and required wherever they are read. The kernels read a position
 * relative to the cell corner as fma(a + 1/2, s 2^-b, off) in FP32 with
 * s = RNE32(1 / n_c). */
#define SPH_ANCHOR_CORNER 0
#define SPH_ANCHOR_SUB(b) (1 + (b))
typedef struct {
  int32_t pos, vel, mhu;
  int32_t scale_m, scale_h, scale_u;
  int32_t pos_anchor;     /* SPH_ANCHOR_CORNER or SPH_ANCHOR_SUB(0..2)    */
  int32_t reserved;       /* must be 0                                    */
} sph_precision;

/* which fields a convert or writeback moves (operator N of Sec. 4.1) */
typedef enum {
  SPH_VIEW_DENSITY = 0,   /* OFF, M, H, U                                 */
  SPH_VIEW_FORCE = 1,     /* OFF, VQ, M, H                                */
  SPH_VIEW_KICK = 2,      /* X, V, UK                                     */
  SPH_VIEW_FULL = 3,      /* all of the above                             */
  /* views of the streaming arrangement (host gather only): the inputs the
   * in-place arrangement keeps resident on the device come from the
   * records instead (host gather and sph_convert_host only) */
  SPH_VIEW_FORCE_IN = 4,  /* FORCE + RHO, F, P, C (FP32)                  */
  SPH_VIEW_KICK_IN = 5    /* KICK + A, DU (FP32)                          */
} sph_view;

/* physics constants: H = gamma_k h; P = (gamma - 1) rho u; viscosity
 * strength alpha and signal-velocity coefficient beta; gradh = 1 applies
 * the grad-h factor f_i, 0 sets f_i = 1; kernel picks the smoothing kernel
 * (Sec. 2.1 names the cubic-spline and Wendland families): SPH_KERNEL_M4,
 * w(u) = 8/pi (1 - 6u^2 + 6u^3) for u < 1/2, 16/pi (1-u)^3 for u < 1
 * (gamma_k = 1.825742), or SPH_KERNEL_WENDLAND_C2,
 * w(u) = 21/(2 pi) (1-u)^4 (1 + 4u) for u < 1 (gamma_k = 1.936492); both
 * normalised on the unit support u = r / H. */
typedef struct {
  double gamma_k, gamma, alpha, beta;
  int32_t gradh;
  int32_t kernel;
} sph_params;

#define SPH_KERNEL_M4 0
#define SPH_KERNEL_WENDLAND_C2 1

/* pair-kernel tiling: ti particles i per work item, k lanes per particle
 * (ti * k threads per workgroup). {0, 0} picks the default. Supported
 * combinations are listed by sph_tile_supported. */
typedef struct {
  int32_t ti, k;
} sph_tile;

/* ------------------------------------------------------------------ */
/* Entry points                                                        */
/* ------------------------------------------------------------------ */

int32_t sph_abi_version(void);

/* Bytes of an SoA field of n values stored in dtype (SPH_F32, SPH_F16,
 * SPH_BF16 or SPH_TRUNC_BITS(T)). */
sph_status sph_storage_bytes(int32_t n, int32_t dtype, size_t *bytes);
const char *sph_last_error(void);

/* 1 if the tiling is compiled in, else 0. */
int32_t sph_tile_supported(sph_tile tile);

/* Workspace bytes sph_bin needs for n particles and n_c cells per axis. */
sph_status sph_bin_workspace_size(int32_t n, int32_t n_c, size_t *bytes);

/* Cell binning (spatial buffers of co-located particles, Sec. 6 setup).
 * For every record i of the AoS (device pointer aos, layout->stride bytes
 * apart, X read as FP64): wrap x into [0,1) as x - floor(x); per axis
 * c = min(floor(x * n_c), n_c - 1) in FP64; id = cx + n_c (cy + n_c cz).
 * Writes cells->cell_start, cells->perm and cells->cell (stable order by
 * (cell id, sub-cell Morton code, input index): bit-identical on every
 * run), cells->sub_start when sub_bits > 0, and cells->hmax (max h of each
 * cell, h read as stored in the record) when it is non-NULL and the layout
 * has H. cells->n, n_c and sub_bits are inputs. Raises
 * SPH_FLAG_BAD_POSITION for non-finite x (such particles go to cell 0). */
sph_status sph_bin(const void *aos, const sph_aos_layout *layout, const sph_cells *cells,
                   void *workspace, size_t workspace_bytes, hipStream_t stream);

/* AoS->SoA gather U o N o C (Sec. 4.1; Eq. gpu_soa_conversion): for every
 * sorted slot k, read record perm[k] and write the view's fields at k.
 * OFF = FP32(x_wrapped - anchor) (FP64 difference, one rounding; anchor as
 * in sph_precision), then the pos format, and ANC for anchors with b >= 1;
 * VQ, M, H, U: RNE to FP32, scale, RNE to the format;
 * X: wrapped FP64 position; V, UK: FP32. */
sph_status sph_convert(const void *aos, const sph_aos_layout *layout, const sph_cells *cells,
                       int32_t view, const sph_precision *prec, const sph_soa *out,
                       hipStream_t stream);

/* Host-side variant (Eq. gpu_soa_conversion_cpu_datamanagement; the
 * soa_conversion_handler(host) semantics of Sec. 3.1): the host bins the
 * host AoS (aos_host, n records) with nthreads worker threads and gathers
 * the view into pinned host staging (staging_host, at least
 * sph_host_staging_size bytes, allocated with hipHostMalloc), then copies
 * the cell list (cell_start, perm, cell and, when non-NULL, hmax with the
 * definition of sph_bin) and the view to the device buffers of cells / out
 * on stream. Returns after the copies are enqueued; staging must stay alive
 * until the stream reaches them. Sub-cell order is built by sph_bin only:
 * cells->sub_bits must be 0 (else SPH_E_UNSUPPORTED). */
sph_status sph_host_staging_size(int32_t n, int32_t n_c, int32_t view,
                                 const sph_precision *prec, size_t *bytes);
sph_status sph_convert_host(const void *aos_host, const sph_aos_layout *layout,
                            const sph_cells *cells, int32_t view, const sph_precision *prec,
                            const sph_soa *out, void *staging_host, size_t staging_bytes,
                            int32_t nthreads, hipStream_t stream);

/* Streaming arrangement (Sec. 6, the pipeline comparison): every kernel
 * call ships only the fields it needs, and all reorganisation happens on
 * the host. A step is sph_bin_host; H2D of the cell list; then per kernel
 * sph_gather_host (view DENSITY, FORCE_IN, KICK_IN), the kernel, and
 * sph_writeback_host of its outputs (view DENSITY, FORCE, KICK).
 *
 * sph_bin_host: the cell list of the host records with the definition of
 * sph_bin for sub_bits = 0 (stable order by (cell id, input index)) into
 * caller-owned host arrays: cell_start[n_c^3 + 1], perm[n], cell[n] and,
 * when non-NULL, hmax[n_c^3] (0 for every cell if the layout has no H).
 * nthreads <= 0: one per hardware thread.
 *
 * sph_gather_host: the view's fields of records perm[k], quantised as in
 * sph_convert (same values bit for bit) into pinned staging (at least
 * sph_host_staging_size bytes, hipHostMalloc), then enqueues their H2D
 * copies into out on stream and returns; staging must stay alive and
 * unchanged until the stream reaches the copies. perm and cell must be a
 * cell list of these records (entries out of range: SPH_E_RANGE).
 *
 * sph_writeback_host: the outputs of a view (DENSITY: rho, wcount, rho_dh,
 * f, P, c, nngb; FORCE: a, du, vsig, nforce; KICK: X, V, UK -> x, v, u) are
 * copied D2H into pinned staging (sph_writeback_host_size bytes) on stream;
 * the call waits for the stream and scatters them into host records
 * perm[k] (FP32 values widened to the record's FP64 fields where the layout
 * says so). Blocking. */
sph_status sph_bin_host(const void *aos_host, const sph_aos_layout *layout, int32_t n, int32_t n_c,
                        int32_t *cell_start, int32_t *perm, int32_t *cell, float *hmax,
                        int32_t nthreads);
sph_status sph_gather_host(const void *aos_host, const sph_aos_layout *layout, int32_t n,
                           int32_t n_c, const int32_t *perm, const int32_t *cell, int32_t view,
                           const sph_precision *prec, const sph_soa *out, void *staging_host,
                           size_t staging_bytes, int32_t nthreads, hipStream_t stream);
sph_status sph_writeback_host_size(int32_t n, int32_t view, size_t *bytes);
sph_status sph_writeback_host(const sph_soa *soa, int32_t n, const int32_t *perm, int32_t view,
                              void *aos_host, const sph_aos_layout *layout, void *staging_host,
                              size_t staging_bytes, int32_t nthreads, hipStream_t stream);

/* SoA->AoS writeback C^AoS_SoA o N^T o U^T (Sec. 4.1): writes the view's
 * state (KICK: X, V, UK -> x, v, u) and the kernel outputs present in soa
 * (DENSITY: rho, wcount, rho_dh, f, P, c, nngb; FORCE: a, du, vsig,
 * nforce; FULL: all plus the cell id) into record perm[k]. */
sph_status sph_writeback(const sph_soa *soa, const sph_cells *cells, int32_t view,
                         void *aos, const sph_aos_layout *layout, hipStream_t stream);

/* Work list for the pair kernels (Alg. 1 CallQuadratic over all cells of
 * uneven occupancy in one launch; the relaxed neighbourhood-neighbourhood
 * checks with interaction masking that Sec. 2.2 describes for
 * accelerators, over chunks of co-located particles as the buffers of
 * Sec. 6 are): one item per chunk of at most ti
 * consecutive slots of a cell, in cell order. The cost of an item is
 * estimated as its particle count times the particle count of the 27 cells
 * around its cell, capped at 27 x 64 (h follows the density, so the
 * candidates a chunk stages stay bounded next to crowded cells); the 8 XCD
 * ranges split the total cost evenly. Items are
 * independent (each writes only its own particles), so no result depends on
 * the schedule. work->sched is not used here. */
sph_status sph_worklist_size(int32_t n, int32_t n_c, int32_t ti, size_t *bytes);
sph_status sph_worklist(const sph_cells *cells, sph_work *work, hipStream_t stream);
/* The same list restricted to the cells holding occ_lo <= count < occ_hi
 * particles: a loop over all cells can run as several launches, each with
 * the tile that suits its occupancy class (results do not depend on the
 * split). Empty or negative ranges: SPH_E_INVALID. */
sph_status sph_worklist_occupancy(const sph_cells *cells, sph_work *work, int32_t occ_lo,
                                  int32_t occ_hi, hipStream_t stream);

/* Density loop (Eq. density; Alg. 1 CallQuadratic over the 27 cells
 * around each particle's cell). For every slot i, over every j with
 * r_ij < H_i, the self pair included (support test in FP32:
 * r2 = fma(dz,dz,fma(dy,dy,dx*dx)) < (gamma_k h_i)^2 with d the difference
 * of the stored positions relative to i's cell corner; a pair decided
 * otherwise than in FP64 lies within FP32 rounding of the support radius):
 *   rho_i = sum m_j W(r_ij, h_i)      wcount_i = (4 pi/3) sum w(r_ij/H_i)
 *   rho_dh_i = sum m_j dW/dh          nngb_i = #j
 *   f_i = 1 / (1 + h_i rho_dh_i / (3 rho_i))   (1 if gradh = 0)
 *   P_i = (gamma-1) rho_i u_i         c_i = sqrt(gamma (gamma-1) u_i)
 * Reads OFF (and ANC), M, H, U; writes RHO, WCOUNT, RHO_DH, F, P, C, NNGB.
 * work == NULL: one workgroup per cell; otherwise one launch over the work
 * list with schedule work->sched (work->ti must equal the tile's ti). Candidates come from
 * the sub-cells (or cells, sub_bits = 0) within the chunk's bounding box
 * widened by its largest support radius. */
sph_status sph_density(const sph_soa *soa, const sph_precision *prec, const sph_cells *cells,
                       const sph_params *params, sph_tile tile, const sph_work *work,
                       hipStream_t stream);

/* Force loop (Eq. momentum and Eq. energy, discrete grad-h form with
 * signal-velocity artificial viscosity). For every slot i, over j != i with
 * r_ij < max(H_i, H_j) (FP32 test as above against both radii):
 *   A = f P / rho^2,  g_k = w'(r/H_k)/H_k^4 if r < H_k else 0,
 *   w = (v_i - v_j).e,  mu = min(w, 0),  vsig_ij = c_i + c_j - beta mu,
 *   Pi = -alpha vsig_ij mu / (rho_i + rho_j),  gbar = (g_i + g_j)/2,
 *   a_i   -= m_j (A_i g_i + A_j g_j + Pi gbar) e
 *   du_i  += m_j (A_i g_i + Pi gbar / 2) w
 *   vsig_i = max_j vsig_ij,  nforce_i = #j
 * A pair at zero separation (coincident stored positions, j != i) has the
 * zero vector as e: it counts, adds nothing to a and du, and has
 * vsig_ij = c_i + c_j (the r -> 0 limit of the pair terms, which vanish
 * with w'(0) = 0).
 * Reads OFF (and ANC), VQ, M, H and RHO, F, P, C; writes A_*, DU, VSIG,
 * NFORCE.
 * Needs cells->hmax (the neighbour bound of each cell); work as above. */
sph_status sph_force(const sph_soa *soa, const sph_precision *prec, const sph_cells *cells,
                     const sph_params *params, sph_tile tile, const sph_work *work,
                     hipStream_t stream);

/* Kick and drift (Alg. 1 CallLinear): v += a dt_kick, u += du dt_kick
 * (FP32), then x += v dt_drift in FP64 with the kicked v and wrap into
 * [0,1). Reads/writes X, V, UK; reads A_*, DU. If moved (device int32)
 * is non-NULL, adds the number of particles whose cell changed or, with
 * cells->sub_bits > 0, whose sub-cell changed (the binning's definitions
 * of both). */
sph_status sph_kick_drift(const sph_soa *soa, const sph_cells *cells, double dt_kick,
                          double dt_drift, int32_t *moved, hipStream_t stream);

/* FP64 reductions over the slots (deterministic order): the conservation
 * checks of the discrete equations of Sec. 2.1 (Eq. momentum: the pair
 * forces are antisymmetric, so sum m a vanishes up to rounding; Eq. energy:
 * sum m (v.a + du/dt) vanishes for the same reason), with the magnitudes
 * they are measured against:
 * out[0..2] = sum m a, out[3] = sum m (v.a + du), out[4] = sum m |a|,
 * out[5] = sum m (|v.a| + |du|), out[6] = sum nngb, out[7] = sum nforce.
 * Reads M (with its scale) or, if NULL, nothing for m (m = 1), V, A, DU,
 * NNGB, NFORCE. out: 8 doubles on the device. workspace: at least
 * sph_reduce_workspace_size bytes. */
sph_status sph_reduce_workspace_size(int32_t n, size_t *bytes);
sph_status sph_reduce(const sph_soa *soa, const sph_precision *prec, const sph_cells *cells,
                      double *out, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* sph_reduce without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the same kernels and the same results bit for
 * bit, with the partial sums in a 64 KiB array the library holds on each
 * device it runs on (kept until the process ends; its address is resolved
 * on the first call on a device). The call allocates nothing. It runs on
 * the current device, and stream must belong to it. Every partial sum is
 * overwritten by each call, so nothing needs clearing; calls that overlap
 * on one device (on different streams or threads) share the array and race.
 * The scratch covers any slot count (SPH_E_NOMEM would report a count
 * beyond it). */
sph_status sph_reduce_static(const sph_soa *soa, const sph_precision *prec,
                             const sph_cells *cells, double *out, hipStream_t stream);

/* Leapfrog kick-drift-kick over several steps (the Kick and Drift kernels
 * of Sec. 6 arranged as the second-order integrator; the paper gives no
 * scheme). A step of size dt: sph_kick_drift(dt/2, dt) and the kick view
 * written back; rebin and convert; sph_predict(dt/2); density and force;
 * sph_kick_drift(dt/2, 0); full writeback (which keeps the rates a, du in
 * the records for the next prediction).
 *
 * sph_predict: the force depends on v (viscosity) and, through the
 * pressure, on u, so the forces at the end of the step are evaluated with
 * v and u predicted by the last rates: for every slot k, with the record
 * perm[k]'s A and DU, VQ = Q_vel(V + a dt_half) and U = Q_mhu((UK + du
 * dt_half) 2^scale_u) in FP32 (fma), where V, UK (the kick view) hold the
 * half-step values. Writes VQ and U only; IEEE storage formats only
 * (SPH_E_UNSUPPORTED for truncated ones).
 *
 * sph_step_totals: out[0..2] = sum m v, out[3] = sum m |v|^2 / 2,
 * out[4] = sum m u, out[5] = sum m (FP64, deterministic order, m and h as
 * stored with their scales, v and u from V and UK), out[6] = the Courant
 * step min over slots with vsig > 0 of c_cfl (gamma_k h) / vsig in FP64
 * (+inf if none), out[7] = number of such slots. workspace: at least
 * sph_reduce_workspace_size bytes; out: 8 doubles on the device. */
sph_status sph_predict(const sph_soa *soa, const sph_precision *prec, const sph_cells *cells,
                       const void *aos, const sph_aos_layout *layout, double dt_half,
                       hipStream_t stream);
sph_status sph_step_totals(const sph_soa *soa, const sph_precision *prec, const sph_cells *cells,
                           const sph_params *params, double c_cfl, double *out, void *workspace,
                           size_t workspace_bytes, hipStream_t stream);

/* Plain-AoS forms (Eq. gpu_native): the same kernels reading and writing
 * the AoS records through the cell list (record perm[k] for slot k),
 * with the identical loop order and arithmetic, so FP32 records give
 * bit-identical results to the FP32 SoA path. */
sph_status sph_density_aos(void *aos, const sph_aos_layout *layout, const sph_cells *cells,
                           const sph_params *params, sph_tile tile, const sph_work *work,
                           hipStream_t stream);
sph_status sph_force_aos(void *aos, const sph_aos_layout *layout, const sph_cells *cells,
                         const sph_params *params, sph_tile tile, const sph_work *work,
                         hipStream_t stream);
/* kick/drift over records 0..n-1 (no cell list needed; cells->n_c is used
 * for the moved count when moved != NULL) */
sph_status sph_kick_drift_aos(void *aos, const sph_aos_layout *layout, const sph_cells *cells,
                              double dt_kick, double dt_drift, int32_t *moved,
                              hipStream_t stream);
/* The FP64 reductions of sph_reduce (the conservation sums of Sec. 2.1,
 * Eq. momentum and Eq. energy, and the neighbour-count totals) over the
 * AoS records through the cell list: slot k reads record perm[k]'s M (1 if
 * the layout has none), V, A, DU, NNGB and NFORCE (0 if absent), in the
 * slot order and summation tree of sph_reduce, so FP32 records give the
 * sums of sph_reduce over FP32 storage bit for bit. Needs the cell list of
 * sph_bin; out: 8 doubles on the device; workspace: at least
 * sph_reduce_workspace_size bytes (caller-owned device memory). */
sph_status sph_reduce_aos(const void *aos, const sph_aos_layout *layout, const sph_cells *cells,
                          double *out, void *workspace, size_t workspace_bytes,
                          hipStream_t stream);

/* Autotuner of the pair loops' cell-to-workgroup tiling (the batched
 * launch over cells of uneven occupancy of Alg. 1 CallQuadratic; Sec. 2.2
 * notes that the right offload granularity is a kernel- and
 * architecture-specific decision, which the paper makes by hand and which
 * this call makes by timing). One candidate is a tile and a
 * schedule: sched = -1 launches one workgroup per cell (no work list),
 * otherwise the work list is built for the tile's ti and taken with that
 * SPH_SCHED_* schedule. */
typedef struct {
  sph_tile tile;
  int32_t sched;          /* -1 or SPH_SCHED_*                              */
  float ms;               /* out: mean time of one launch; -1 if skipped    */
} sph_tune_entry;

/* The default candidate set: every supported tile with each schedule.
 * Writes min(count, max) entries to out (may be NULL when max = 0) and the
 * full count to *count. */
sph_status sph_tune_candidates(sph_tune_entry *out, int32_t max, int32_t *count);

/* Times `reps` launches (after one untimed launch) of sph_density
 * (loop = 0) or sph_force (loop = 1) for each of cand[0..ncand) on the
 * caller's SoA and cell list, with HIP events on `stream`, and stores the
 * mean launch time in cand[i].ms. Candidates whose work list needs more
 * than work_bytes get ms = -1. *best = index of the fastest. The loop's
 * outputs are written as by a normal call, by the last candidate timed;
 * different tiles sum in different orders, so rerun the loop with the
 * chosen candidate where bit-reproducible outputs matter. sph_force reads
 * the density outputs: run the density loop first. Blocking: returns after
 * the stream has drained. work_buf (device, work_bytes) holds each
 * candidate's work list in turn and may be NULL when no candidate uses one. */
sph_status sph_autotune(int32_t loop, const sph_soa *soa, const sph_precision *prec,
                        const sph_cells *cells, const sph_params *params,
                        sph_tune_entry *cand, int32_t ncand, int32_t reps, void *work_buf,
                        size_t work_bytes, int32_t *best, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Cell-pair tasks (serving): the density or force sums of a range of i */
/* particles of one cell over the j particles of one neighbouring cell. */
/* The sum over the 27 cells around ci of a particle's task results is  */
/* its full loop result (counts exactly; floating point up to the order */
/* of summation).                                                       */
/* ------------------------------------------------------------------ */
enum { SPH_TASK_DENSITY = 0, SPH_TASK_FORCE = 1 };
typedef struct {
  int32_t kind;           /* SPH_TASK_DENSITY or SPH_TASK_FORCE             */
  int32_t ci, cj;         /* cell of the i particles; cj is one of the 27   */
                          /* cells around ci (ci itself included)           */
  int32_t i_begin, i_end; /* sorted slots cell_start[ci] <= i_begin <=      */
                          /* i_end <= cell_start[ci + 1]                    */
} sph_task;
#define SPH_TASK_MAX_I 1024   /* largest i_end - i_begin of one task      */

/* One result record per i particle of a task (32 bytes):
 *   density: v = {rho, wcount, rho_dh, 0, 0}, count = nngb  (over j in cj)
 *   force:   v = {a_x, a_y, a_z, du_dt, vsig}, count = nforce
 * with the definitions of sph_density / sph_force restricted to j in cj
 * (rho and rho_dh normalised by h_i as there; vsig is the maximum over
 * the task's pairs, 0 if none). */
typedef struct {
  float v[5];
  int32_t count;
  int32_t pad[2];
} sph_task_result;

/* Tiles of the task kernels (ti particles per workgroup, k lanes each) */
int32_t sph_task_tile_supported(sph_tile tile);

/* One launch per kind over a batch of n_tasks tasks (device arrays), each
 * task one CallQuadratic of Alg. 1 over a cell pair, the unit the paper's
 * host threads offload one loop invocation at a time (Sec. 5, GPU data
 * handling; Sec. 6 gives 16 host cores to offloading): items are
 * (task index, first slot) pairs, one per chunk of at most tile.ti slots
 * of a task, density items first (n_dens of them), then force items
 * (n_force); out_off[t] is the index in `out` of task t's first result;
 * `out` holds n_out records. Reads the view of sph_density (density
 * items) or sph_force (force items) from soa. Every index read from the
 * device arrays is clamped to the cell list and to n_out, so bad entries
 * cannot address memory outside them; the host checks tasks before they
 * reach the device (sph_server_submit). */
sph_status sph_tasks_run(const sph_soa *soa, const sph_precision *prec, const sph_cells *cells,
                         const sph_params *params, sph_tile tile, const sph_task *tasks,
                         int32_t n_tasks, const int32_t *out_off, const int32_t *items,
                         int32_t n_dens, int32_t n_force, sph_task_result *out, int32_t n_out,
                         hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Serving loop: cell-pair tasks over particle state resident in HBM,  */
/* continuously batched. A dispatcher thread takes the tasks whose      */
/* arrival time has passed, in arrival order, as long as their result  */
/* records fit in the device result pool (admission by memory           */
/* footprint), and launches them as one batch on a free stream; up to  */
/* `streams` batches run on the device at once, so tasks that arrive    */
/* while others run are admitted as soon as a stream and pool memory   */
/* free up. A completion thread copies each finished batch's records to */
/* the requests' host buffers, frees its pool memory and time-stamps    */
/* it. A task's records depend only on the task and the resident state, */
/* never on the batch it ran in.                                        */
/* ------------------------------------------------------------------ */
typedef struct sph_server sph_server;   /* opaque */

typedef struct {
  sph_tile tile;          /* task kernel tile ({0, 0}: 64 x 4)              */
  int32_t streams;        /* batches in flight, 1..8                        */
  int32_t max_batch;      /* tasks per batch, 1..4096                       */
  size_t pool_bytes;      /* device bytes for the records of in-flight      */
                          /* tasks (>= SPH_TASK_MAX_I records)              */
} sph_server_config;

typedef struct {
  sph_task task;
  int32_t reserved;       /* must be 0                                      */
  int64_t arrival_ns;     /* sph_now_ns clock; not started before this      */
  sph_task_result *out;   /* host memory for i_end - i_begin records        */
                          /* (pinned recommended), or NULL to drop them     */
} sph_request;            /* 40 bytes */

typedef struct {
  int64_t id;             /* from sph_server_submit                         */
  int64_t arrival_ns, admit_ns, launch_ns, done_ns;
  int32_t batch;          /* batch sequence number                          */
  int32_t batch_tasks;    /* tasks in that batch                            */
} sph_task_done;          /* 48 bytes */

typedef struct {
  int64_t submitted, done, batches;
  int64_t admission_waits;   /* dispatcher rounds that found arrived tasks  */
                             /* but no pool memory for the next one         */
  int32_t max_inflight;      /* most batches on the device at once          */
  int32_t reserved;
  int64_t pool_high_water;   /* most pool bytes in use at once              */
} sph_server_stats;

/* Steady clock of the server, in ns */
int64_t sph_now_ns(void);

/* Device workspace bytes of a server with this configuration (the result
 * pool plus each stream's task descriptors). */
sph_status sph_server_workspace_size(const sph_server_config *cfg, size_t *bytes);

/* Starts a server over the resident state: soa (the views of sph_density
 * and sph_force, density outputs included for force tasks), prec, cells
 * (its cell_start is read once, to check tasks) and params are copied by
 * value, the device buffers they name must stay alive and unchanged until
 * sph_server_destroy. workspace: device, sph_server_workspace_size bytes.
 * Creates its streams (default priority) and pinned staging. */
sph_status sph_server_create(const sph_server_config *cfg, const sph_soa *soa,
                             const sph_precision *prec, const sph_cells *cells,
                             const sph_params *params, void *workspace, size_t workspace_bytes,
                             sph_server **out);

/* Queues n requests (thread-safe); ids are consecutive from *first_id.
 * Every task is checked against the cell list first: a bad one rejects the
 * whole call (SPH_E_INVALID / SPH_E_RANGE, nothing queued). */
sph_status sph_server_submit(sph_server *srv, const sph_request *req, int32_t n,
                             int64_t *first_id);

/* Moves up to max completion records to done (in completion order), waiting
 * up to wait_ms for the first one; *n = records written. A HIP error of the
 * serving threads is reported here (SPH_E_HIP) and stops the server. */
sph_status sph_server_poll(sph_server *srv, sph_task_done *done, int32_t max, int32_t *n,
                           int32_t wait_ms);

sph_status sph_server_get_stats(sph_server *srv, sph_server_stats *stats);

/* Waits until every queued task is done (or timeout_ms passes:
 * SPH_E_RANGE). Completion records stay for sph_server_poll. */
sph_status sph_server_drain(sph_server *srv, int32_t timeout_ms);

/* Stops the threads after the batches in flight finish, releases the
 * streams and pinned memory. Queued tasks that have not started are
 * dropped. */
sph_status sph_server_destroy(sph_server *srv);

/* Smoothing lengths adapted to the local density (Sec. 2.1: h follows the
 * density so that the neighbour number stays about constant): for every
 * slot, the root of h = eta (m / rho(h))^(1/3), rho(h) the density loop's
 * sum at the particle's own h, by Newton steps with the loop's drho/dh
 * (f'(h) = 1 + (h_t / (3 rho)) drho/dh, h_t = eta (m / rho(h))^(1/3); a
 * step f' <= 0 would make is replaced by h_t; each new h is limited to
 * [h/2, 2h] and to h_max, the largest FP32 h whose support radius fits a
 * cell both in the kernels' FP32 test and exactly), starting from the
 * stored H. A particle is done after the first
 * step with |h_new - h| < tol h that the h_max limit did not cut; each pass
 * runs the density loop (tile, work as in sph_density; the work list is
 * rebuilt for the cells that still hold unfinished particles) and then the
 * step. H must be stored in SPH_F32 (prec->mhu). Afterwards cells->hmax
 * (if non-NULL) holds the new per-cell maxima and, if aos is non-NULL, h is
 * written into the records' H field (layout must have H). The density
 * outputs are those of the last pass: run sph_density for values at the
 * final h. *iterations = passes run, *unconverged = particles not done.
 * work is left holding the last pass's list: rebuild it (sph_worklist)
 * before using it for another launch.
 * Blocking: reads the count of unfinished particles after every pass.
 * workspace: device, sph_smoothing_length_workspace_size(n) bytes. */
sph_status sph_smoothing_length_workspace_size(int32_t n, size_t *bytes);
sph_status sph_smoothing_length(const sph_soa *soa, const sph_precision *prec,
                                const sph_cells *cells, const sph_params *params, double eta,
                                double tol, int32_t max_iter, sph_tile tile,
                                const sph_work *work, void *workspace, size_t workspace_bytes,
                                void *aos, const sph_aos_layout *layout, int32_t *iterations,
                                int32_t *unconverged, hipStream_t stream);

/* Streaming probes of the device memory rate: the ceiling against which the
 * streaming kernels (convert, writeback, kick/drift) are measured. One
 * launch moves `bytes` (a multiple of 16, src and dst 16-byte aligned) with
 * 16-byte non-temporal accesses: SPH_PROBE_COPY reads src and writes dst
 * (2 x bytes of traffic), SPH_PROBE_READ reads src (dst: a device float
 * that is written only in a case no finite input produces), SPH_PROBE_WRITE
 * writes dst (src unused). No result beyond the traffic is defined. */
#define SPH_PROBE_COPY 0
#define SPH_PROBE_READ 1
#define SPH_PROBE_WRITE 2
sph_status sph_hbm_probe(int32_t mode, const void *src, void *dst, size_t bytes,
                         hipStream_t stream);

/* hipStreamSynchronize with the error mapped to sph_status */
sph_status sph_sync(hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* SPHMI_H */
