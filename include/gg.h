/*
 * gg.h - C ABI of the MI355X (gfx950) initial-conditions library.
 *
 * The library computes the data-parallel hot path of the Ginnungagap
 * initial-conditions method (arxiv 2511.10353, Sec. 2.1-2.2) on one GPU that
 * holds the whole N^3 lattice:
 *
 *   white noise W (Sec. 2, step 1)
 *   -> forward real-to-complex 3D transform W~
 *   -> Eq. (1)  delta~ = sqrt(P(k) N^3/L^3) W~   and
 *      Eq. (2)  psi~_j = i k_j / k^2 delta~,  j = 0, 1, 2
 *   -> three complex-to-real inverse transforms psi_j
 *   -> Eq. (3)  Zel'dovich positions x_j = q_j + psi_j and velocities
 *               v_j = a H(a) f psi_j at the lattice points q.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Lattice cell (m0, m1, m2), m_i in [0, N), has linear index
 *   c = (m0 N + m1) N + m2: row-major, axis 2 contiguous.
 * - Real field ("R"): N^3 values of the plan's dtype (float or double).
 * - Half spectrum ("H"): N * N * (N/2 + 1) complex values, interleaved
 *   (re, im) of the plan's dtype, mode (k0, k1, k2) at
 *   (k0 N + k1) (N/2 + 1) + k2, k2 in [0, N/2]; the same layout as
 *   numpy.fft.rfftn of the real field.
 * - Forward transform unnormalised, exp(-2 pi i k.m/N); inverse normalised
 *   by 1/N^3, exp(+2 pi i k.m/N).
 * - Signed mode index s(k) = k for k < N/2, k - N above; k_j = 2 pi s_j / L.
 *   The filter zeroes k = 0 and every mode with |s_j| = N/2 on any axis.
 * - Particle arrays: float32, structure of arrays, component j of cell c at
 *   j N^3 + c (3 N^3 values each for positions and velocities).
 * - Noise: cell c is one Philox-4x32-10 call (key = seed, counter =
 *   (c, stream_id, 0)); its words w0, w1 give the cosine branch of the
 *   Box-Muller transform, sqrt(-2 ln u1) cos(2 pi u2), evaluated in binary64
 *   with a fixed operation sequence, so a cell's value depends only on
 *   (seed, stream_id, c).  The float path stores that value rounded once.
 *
 * Memory, streams, errors
 * -----------------------
 * - Every data pointer is a device pointer owned by the caller; the library
 *   never frees it.  Pointers must be 256-byte aligned.  Nothing on the hot
 *   calls allocates memory.
 * - ``stream`` is a hipStream_t passed as void* (NULL = the null stream).
 *   Every launch is asynchronous on that stream; a fault inside a kernel is
 *   reported by the caller's next synchronisation, not by the call.
 * - Arguments are validated before anything is launched: a bad argument
 *   returns GG_ERR_INVALID_ARG and launches nothing.  gg_last_error() then
 *   holds a message (per thread).  No call throws across the ABI.
 * - Failure injection for tests: with the environment variable
 *   GG_FAULT_INJECT=plan_alloc, gg_plan_create fails its last device
 *   allocation (GG_ERR_OUT_OF_MEMORY, the earlier ones freed); with
 *   GG_FAULT_INJECT=launch, gg_make_ic returns GG_ERR_HIP without launching.
 *   The variable is read on each call; unset, it changes nothing.
 * - GG_CUS=k (1 <= k < the device's compute units), read by gg_plan_create:
 *   the plan sizes the grids of its persistent passes (P3 of float plans,
 *   P5) as if the device had k compute units, so that each work-group loops
 *   over more tiles.  Results do not depend on it; tests use it to exercise
 *   those loops at small lattices.
 * - A plan is read-only after gg_plan_create, except for the timing records
 *   of gg_timing_enable.  gg_noise, gg_fft3d, gg_filter and gg_zeldovich on one
 *   plan may run from several streams (each with its own buffers);
 *   gg_make_ic uses a stream and events owned by the plan, so two gg_make_ic
 *   calls on one plan must not be in flight from different host threads.
 */
#ifndef GG_H
#define GG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GG_OK = 0,
    GG_ERR_INVALID_ARG = 1,      /* null/misaligned pointer, bad flag or value */
    GG_ERR_UNSUPPORTED_SIZE = 2, /* N not supported by the kernels             */
    GG_ERR_OUT_OF_MEMORY = 3,    /* plan tables could not be allocated         */
    GG_ERR_HIP = 4,              /* a HIP runtime call or launch failed        */
    GG_ERR_INTERNAL = 5
} gg_status;

typedef enum { GG_F32 = 0, GG_F64 = 1 } gg_dtype;

/* Lattice: N cells per side (a power of two, 8 <= N <= 1024, or 96, 160,
 * 192), box side L in Mpc/h. */
typedef struct {
    int32_t n;
    double box;
} gg_grid;

/* Cosmology of the analytic spectrum P(k, z) = D(z)^2 A k^n_s T_BBKS(k)^2
 * (BBKS fit, Gamma = omega_m h), sigma_8 at z = 0, Einstein-de Sitter growth
 * D = 1/(1+z), flat-LCDM H(a), f = 1 (Sec. 2.1 footnote; Sec. 2.2).
 * amp > 0 uses A = amp instead of the sigma_8 normalisation.
 * lattice_offset is the Lagrangian point inside a cell, in cells, in [0, 1)
 * (0.5 puts particles at cell centres as Sec. 2.2 describes). */
typedef struct {
    double omega_m;
    double h;
    double n_s;
    double sigma8;
    double z_init;
    double amp;
    double lattice_offset;
} gg_cosmo;

/* Read-only facts about a plan. */
typedef struct {
    int32_t n;
    int32_t dtype;           /* gg_dtype */
    double box;
    double amplitude;        /* A at z = 0, from the FP64 sigma_8 integral */
    double sigma8_integral;  /* sigma^2(8 Mpc/h) of the spectrum with A = 1 */
    double growth;           /* D(z_init) */
    double velocity_factor;  /* a H(a) f at z_init, km/s per Mpc/h */
    size_t real_elems;       /* N^3 */
    size_t spectrum_elems;   /* N N (N/2+1) complex values */
    size_t workspace_bytes;  /* = gg_workspace_bytes(plan) */
    int32_t chunks;          /* launches per pass of P1-P4 in gg_make_ic (pipelining) */
    int32_t p1_lines;        /* lattice lines per work-group of the first pass */
    int32_t z_lines;         /* lattice lines per work-group of the last (particle) pass */
} gg_plan_info;

typedef struct gg_plan gg_plan;

/* Builds the device tables of a plan on the current HIP device: FP64-generated
 * twiddles rounded to the dtype, the FP64 sigma_8 integral (Sec. 2.1
 * footnote) evaluated on the GPU, and the table tau[n^2] of the filter of
 * Eq. (1)-(2).  Synchronous.  *plan is set only on GG_OK.
 * Errors: INVALID_ARG (null pointer, box <= 0, cosmology out of range),
 * UNSUPPORTED_SIZE (N), OUT_OF_MEMORY, HIP. */
gg_status gg_plan_create(gg_plan** plan, const gg_grid* grid, const gg_cosmo* cosmo, gg_dtype dtype);

/* Frees the plan's tables (after synchronising its device).  NULL is a no-op. */
gg_status gg_plan_destroy(gg_plan* plan);

gg_status gg_plan_query(const gg_plan* plan, gg_plan_info* info);

/* Bytes of device workspace that gg_make_ic and gg_fft3d need; 0 for a NULL
 * plan. */
size_t gg_workspace_bytes(const gg_plan* plan);

/* White noise (Sec. 2, step 1): w[c] = N(0,1) deviate of cell c, c < N^3,
 * in the plan's dtype.  w: R, written. */
gg_status gg_noise(const gg_plan* plan, uint64_t seed, uint32_t stream_id, void* w, void* stream);

/* 3D transform (Sec. 2.1).  dir = +1: in is R, out is H (unnormalised
 * forward); work may be NULL.  dir = -1: in is H (a Hermitian half
 * spectrum, left unmodified), out is R (normalised by 1/N^3); work must hold
 * gg_workspace_bytes(plan).  in and out must not overlap. */
gg_status gg_fft3d(const gg_plan* plan, int dir, const void* in, void* out, void* work, void* stream);

/* Eq. (1) then Eq. (2): from the forward spectrum of the noise, writes the
 * three displacement spectra psi~_j = i k_j/k^2 sqrt(P N^3/L^3) W~ into
 * psi_spec (3 consecutive H arrays, component j at j N N (N/2+1)), and, if
 * delta_spec is not NULL, delta~ = sqrt(P N^3/L^3) W~ (one H array). */
gg_status gg_filter(const gg_plan* plan, const void* spec_in, void* psi_spec, void* delta_spec, void* stream);

/* Eq. (3): from three displacement fields psi (3 consecutive R arrays),
 * writes float32 positions x_j = wrap_L(q_j + psi_j) (sum in FP64, the
 * periodic image x - L floor(x/L) in [0, L), a value rounding to L stored as
 * 0) and velocities v_j = a H f psi_j, q_j = (m_j + lattice_offset) L/N. */
gg_status gg_zeldovich(const gg_plan* plan, const void* psi, float* pos, float* vel, void* stream);

/* The whole path from a seed (stream_id 0): noise, forward transform, filter,
 * three inverse transforms and Eq. (3), as five fused passes.  pos and vel as
 * for gg_zeldovich; psi_opt, if not NULL, receives the three displacement
 * fields (3 R arrays).  work must hold gg_workspace_bytes(plan).  On large
 * lattices passes 1/2 and 3/4 are pipelined in chunks over `stream` and a
 * stream owned by the plan: the call is ordered after earlier work on
 * `stream`, and later work on `stream` starts after all of it. */
gg_status gg_make_ic(const gg_plan* plan, uint64_t seed, float* pos, float* vel, void* psi_opt, void* work,
                     void* stream);

/* gg_make_ic without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a static device array of
 * GG_NOALLOC_SCRATCH_BYTES (48 MiB) that the library holds on each device it
 * runs on until the process ends; its address is looked up once per device
 * by gg_plan_create.  Lattices whose gg_workspace_bytes exceeds it (float
 * plans above 160^3, double plans above 128^3) are rejected with
 * GG_ERR_UNSUPPORTED_SIZE.  Allocates nothing.  Every call on a device shares
 * that device's array: calls that overlap in time on one device (two host
 * threads, or two streams without ordering) race and give undefined
 * results.  No state is kept between calls: every workspace byte a call reads
 * is written earlier in the same call.  Arguments and results otherwise as
 * for gg_make_ic. */
#define GG_NOALLOC_SCRATCH_BYTES ((size_t)48 << 20)
gg_status gg_make_ic_noalloc(const gg_plan* plan, uint64_t seed, float* pos, float* vel, void* psi_opt, void* stream);

/* The same path with the white noise given instead of generated: w is R in the
 * plan's dtype.  amp_scale multiplies the displacements (amp_scale^2 scales
 * the spectrum amplitude A; 1 keeps the plan's).  pos and vel may both be NULL
 * when psi_opt is given (displacements only).  Used as the forward map of the
 * adjoint below. */
gg_status gg_make_ic_from_noise(const gg_plan* plan, const void* w, double amp_scale, float* pos, float* vel,
                                void* psi_opt, void* work, void* stream);

/* Adjoint of gg_make_ic_from_noise (differentiation, Sec. 2.1 Eq. 1-2 and
 * Sec. 2.2 Eq. 3 are linear in the noise): given the gradient of a loss with
 * respect to the displacements (g_psi: 3 R in the dtype), positions (g_pos:
 * 3 N^3 float) and velocities (g_vel: 3 N^3 float) -- any may be NULL, not all
 * -- writes d loss/d w to g_w (R in the dtype):
 *   g_w = amp_scale * sum_j L_j^T g_j,   g_j = g_psi_j + g_pos_j + aHf g_vel_j,
 * where L_j maps w to psi_j.  L_j is a convolution with a real odd kernel, so
 * L_j^T = -L_j: the adjoint runs the five passes of the forward in mirror
 * order (three r2c inputs combined in the axis-0 pass, one c2r output) and
 * recomputes the transform instead of storing intermediates.  If g_log_amp
 * (a device double) and psi (the forward's displacements, 3 R) are given, it
 * also writes d loss/d log A = (1/2) sum g psi (psi scales as sqrt(A)), summed
 * in FP64 in a fixed order.  work: gg_workspace_bytes(plan). */
gg_status gg_make_ic_adjoint(const gg_plan* plan, const void* g_psi, const float* g_pos, const float* g_vel,
                             double amp_scale, const void* psi, double* g_log_amp, void* g_w, void* work,
                             void* stream);

/* The density field of Eq. (1) alone: delta = inverse transform of
 * sqrt(P N^3/L^3) W~ (mean and Nyquist planes zero), one R array in the
 * plan's dtype.  W is the noise of `seed` (stream_id 0) or, if w_opt is not
 * NULL, the R field w_opt.  work: gg_workspace_bytes(plan); delta must not
 * overlap work or w_opt.  Five passes on `stream`. */
gg_status gg_make_density(const gg_plan* plan, uint64_t seed, const void* w_opt, void* delta, void* work,
                          void* stream);

/* Binned power spectrum of a real field (R, plan dtype; Sec. 2.1 lists the
 * density power spectrum among the outputs).  Every mode n != 0 of the field's
 * transform F with b = floor(|n|) < nbins (|n| in units of k_f = 2 pi / L)
 * falls in bin b; pk[b] = (L^3/N^6) <|F|^2>, kmean[b] = k_f <|n|>, counts[b]
 * = number of modes (both halves of the spectrum), all as device doubles
 * (nbins each, 8-byte aligned).  1 <= nbins <= 1024.  work holds the
 * transform and per-work-group partial sums (gg_workspace_bytes(plan)).
 * Sums are binary64 in a fixed order (deterministic). */
gg_status gg_power_spectrum(const gg_plan* plan, const void* field, int32_t nbins, double* pk, double* kmean,
                            double* counts, void* work, void* stream);

/* out[0..3] (device doubles) = mean, standard deviation (population),
 * minimum and maximum of the N^3 values of field (R, plan dtype), in a fixed
 * summation order.  work: gg_workspace_bytes(plan) (partial sums). */
gg_status gg_field_stats(const gg_plan* plan, const void* field, double* out, void* work, void* stream);

/* White-noise refinement (App. A): each patch of N_L^3 parent cells is
 * replaced by N_H^3 child cells whose expansion on the tensor-product basis
 * E_i E_j E_k keeps the parent's coefficients (on F_i F_j F_k) and takes
 * every other coefficient from the noise (Philox value of index
 * p N_H^3 + (i N_H + j) N_H + k for patch p, row-major over the patch grid,
 * with seed and stream_id; binary64).  variant selects the 1D bases:
 *   GG_REFINE_HR      N_L = 1, N_H = 2 (Eq. A.2-A.4)
 *   GG_REFINE_3       N_L = 2, N_H = 3 (Eq. A.7-A.9; factor 3/2)
 *   GG_REFINE_4       N_L = 2, N_H = 4 (Eq. A.10-A.13; the default basis)
 *   GG_REFINE_LINEAR  N_L = 2, N_H = 4 (Eq. A.20-A.23)
 *   GG_REFINE_SINE    N_L = 2, N_H = 4 (Eq. A.24-A.27)
 * parent: n_parent^3 values of dtype; child: (n_parent / N_L * N_H)^3 values
 * (device pointers, 256-byte aligned, not overlapping).  Runs on the current
 * device; computed in binary64 and rounded once to dtype. */
typedef enum { GG_REFINE_HR = 0, GG_REFINE_3 = 1, GG_REFINE_4 = 2, GG_REFINE_LINEAR = 3, GG_REFINE_SINE = 4 } gg_refine;
gg_status gg_refine_noise(int32_t n_parent, gg_dtype dtype, gg_refine variant, const void* parent, uint64_t seed,
                          uint32_t stream_id, void* child, void* stream);

/* The same refinement restricted to a sub-box of the parent: the parent cells
 * origin[j] + [0, count) per axis (periodic in the n_parent^3 parent); count
 * a multiple of N_L; child (count / N_L * N_H)^3.  Patches are numbered
 * row-major over the sub-box.  The noise of a zoom level (Sec. 2.4). */
gg_status gg_refine_noise_region(int32_t n_parent, const int32_t origin[3], int32_t count, gg_dtype dtype,
                                 gg_refine variant, const void* parent, uint64_t seed, uint32_t stream_id, void* child,
                                 void* stream);

/* Displacements psi (3 R arrays, plan dtype) of the noise field w (R) with
 * the filter restricted to a window of modes, for combining two resolutions
 * (Eq. 4-5): modes with n^2 < n2_min or n^2 >= n2_max are dropped (n2_max
 * <= 0: no upper bound), and, if cic_deconvolve is set, the kept modes are
 * divided by the cloud-in-cell window prod_j sinc^2(pi s_j / N).  With a
 * cutoff scale r_s, Eq. 5 (large scales, k r_s < 1) is n2_max =
 * ceil((L / (2 pi r_s))^2) and Eq. 4 (small scales) n2_min = the same value.
 * work: gg_workspace_bytes(plan). */
gg_status gg_make_displacements(const gg_plan* plan, const void* w, int64_t n2_min, int64_t n2_max,
                                int32_t cic_deconvolve, void* psi, void* work, void* stream);

/* dst (3 fields of n_dst^3) += cloud-in-cell (trilinear, periodic)
 * interpolation of src (3 fields of n_src^3) to the points m L / n_dst,
 * 1 <= n_src <= n_dst <= 4096 (any ratio: a multiple for factor-2 refinement,
 * 3/2 for the three-cell patches of Eq. A.15); point m lies in source cell
 * floor(m n_src / n_dst) with weight ((m n_src) mod n_dst) / n_dst, both
 * exact; sums in binary64.  The large-scale half of Eq. 4-5 on the fine
 * lattice. */
gg_status gg_interpolate_add(int32_t n_src, int32_t n_dst, gg_dtype dtype, const void* src, void* dst, void* stream);

/* dst (3 fields of n_dst^3) += cloud-in-cell interpolation of the periodic
 * src (3 fields of n_src^3) at the points origin + m / ratio (in src cells,
 * m < n_dst per axis): the large-scale half of Eq. 4-5 for a zoom level whose
 * sub-box starts at src cell `origin` and refines it by `ratio`. */
gg_status gg_interpolate_add_at(int32_t n_src, int32_t ratio, const int32_t origin[3], int32_t n_dst, gg_dtype dtype,
                                const void* src, void* dst, void* stream);

/* The integer mode bound of the top hat f(k r_s) = [k r_s < 1] of Eq. 4-5 on
 * a periodic box of side `box`: with k = (2 pi / box) |n|, k r_s < 1 holds
 * exactly for the lattice modes with n^2 < ceil((box / (2 pi r_s))^2), the
 * value returned.  -1 for a box or r_s that is not positive and finite.
 * Host-only arithmetic, no device work. */
int64_t gg_cutoff_n2(double box, double r_s);

/* Full-box resolution increase (Sec. 2.3, Eq. 4-5, with App. A):
 *   1. w_child = App. A refinement of w_parent (basis `variant`, new
 *      coefficients from (seed, stream_id), as gg_refine_noise);
 *   2. psi = the child's displacements with the filter kept to the small
 *      scales k r_s >= 1 (Eq. 4);
 *   3. the parent's displacements of w_parent kept to k r_s < 1 (Eq. 5) and
 *      divided by the cloud-in-cell window, then added to psi by CiC
 *      interpolation onto the child's lattice points (as gg_interpolate_add).
 * parent, child: plans over the same box and dtype with child n = parent n
 * N_H / N_L.  r_s: cutoff scale in Mpc/h; 0 selects two parent cells (the
 * paper's choice).  w_parent: R of the parent (read); w_child: R of the child
 * and psi: 3 R of the child (written); work: gg_workspace_bytes(child) (it
 * also holds the parent's large-scale fields and transforms).  Buffers
 * 256-byte aligned, not overlapping.  Launches on `stream` only. */
gg_status gg_increase_resolution(const gg_plan* parent, const gg_plan* child, const void* w_parent, gg_refine variant,
                                 uint64_t seed, uint32_t stream_id, double r_s, void* w_child, void* psi, void* work,
                                 void* stream);

/* Eq. 5 on a real periodic field (R, plan dtype): its transform restricted to
 * n^2 < n2_max (n2_max <= 0: no bound), divided by the cloud-in-cell window
 * if cic_deconvolve is set, transformed back into out (R; may equal field).
 * work: gg_workspace_bytes(plan). */
gg_status gg_lowpass(const gg_plan* plan, const void* field, int64_t n2_max, int32_t cic_deconvolve, void* out,
                     void* work, void* stream);

/* Resolution degrade (Sec. 2.3, last paragraph): nearest-grid-point
 * interpolation of a fine periodic field onto the plan's lattice, then a
 * translation in Fourier space.  fine: (factor n)^3 reals of the plan dtype
 * (row-major, axis 2 contiguous), factor in [1, 16]; the plan's lattice point
 * m coincides with fine point factor * m and takes its value.  That field is
 * then moved by shift[j] cells of the plan's lattice along axis j (the paper
 * moves by half a coarse cell: shift = {0.5, 0.5, 0.5}): mode n_j (signed)
 * is multiplied by exp(-2 pi i shift_j n_j / n), a Nyquist plane n_j = n/2 by
 * cos(pi shift_j) (the real band-limited interpolant).  out: n^3 reals.
 * work: gg_workspace_bytes(plan).  fine, out and work must not overlap.
 * Apply per component to degrade a displacement field. */
gg_status gg_degrade(const gg_plan* plan, const void* fine, int32_t factor, const double shift[3], void* out,
                     void* work, void* stream);

/* Eq. (3) for a lattice placed at origin (3 doubles, Mpc/h) inside a larger
 * periodic box: x_j = wrap(origin_j + (m_j + lattice_offset) L/N + psi_j) into
 * [0, wrap_box), velocities a H f psi_j.  A zoom level's particles in the base
 * box (L is the plan's sub-box side). */
gg_status gg_zeldovich_at(const gg_plan* plan, const void* psi, const double origin[3], double wrap_box, float* pos,
                          float* vel, void* stream);

/* Zoom hierarchy (Sec. 2.3-2.4): a base lattice n[0]^3 over the periodic box
 * L_0 and levels l = 1 .. levels-1 of n[l]^3 cells, each halving its parent's
 * cell over a sub-box of n[l]/2 parent cells starting at parent cell
 * origin[l] (level 1 may wrap around the base box; deeper levels must lie
 * inside their parent sub-box).  Per level: noise = App. A refinement of the
 * parent's sub-box noise (basis `variant`, stream_id = l; the base level is
 * the noise of `seed`, stream 0); psi = Eq. 4 on the level's periodic sub-box
 * (r_s = 2 parent cells) + the CiC interpolation of Eq. 5 applied to the
 * parent's psi (with deconvolution); particles at the level's lattice inside
 * the base box (Eq. 3, positions wrapped into [0, L_0)). */
#define GG_ZOOM_MAX_LEVELS 8
typedef struct {
    int32_t levels;
    int32_t n[GG_ZOOM_MAX_LEVELS];
    int32_t origin[GG_ZOOM_MAX_LEVELS][3];  /* entry 0 unused */
    double box;                              /* L_0 */
    int32_t variant;                         /* gg_refine with N_H = 2 N_L */
} gg_zoom_desc;

typedef struct gg_zoom gg_zoom;

/* Creates one plan per level (sub-box side n[l] L_0 / (n[0] 2^l)); synchronous. */
gg_status gg_zoom_create(gg_zoom** zoom, const gg_zoom_desc* desc, const gg_cosmo* cosmo, gg_dtype dtype);
gg_status gg_zoom_destroy(gg_zoom* zoom);
size_t gg_zoom_workspace_bytes(const gg_zoom* zoom);
/* Level geometry: sub-box side, cell size and origin in the base box (Mpc/h). */
gg_status gg_zoom_query(const gg_zoom* zoom, int32_t level, double* box, double* cell, double origin[3]);

/* Runs the whole hierarchy.  w[l] (R of level l), psi[l] (3 R), pos[l] and
 * vel[l] (3 n[l]^3 floats) are host arrays of device pointers, one per level;
 * work: gg_zoom_workspace_bytes.  The work is spread over `stream` and two
 * streams owned by the zoom object, ordered by events: the noise refinement
 * and Eq. 4 of every level (which need only the noise) run beside the chain
 * of Eq. 5 and CiC interpolations (each level's large scales need its
 * parent's final displacements), and each level's particles are made as soon
 * as its displacements are final.  The call is ordered after earlier work on
 * `stream`; later work on `stream` starts after all of it.  With use_graph
 * set, the schedule is captured into one HIP graph on the first call (stream
 * must not be NULL) and replayed as one graph launch while seed and pointers
 * stay the same (captured again otherwise).  Calls on one zoom must not
 * overlap. */
gg_status gg_zoom_run(gg_zoom* zoom, uint64_t seed, void* const* w, void* const* psi, float* const* pos,
                      float* const* vel, void* work, int32_t use_graph, void* stream);

/* Autotuner of the hierarchy: for each level in turn (the others kept), times
 * gg_zoom_run (eager; one warm-up, then reps calls, HIP events on `stream`)
 * for the tile widths of the level's first and last fused passes (the full
 * LDS row of lines or half of it, as gg_plan_set_tuning), keeps the fastest
 * (a later choice must win by more than 0.5 %) and reports every timing (up
 * to `capacity` entries; *count = number timed).  Arguments of the run as for
 * gg_zoom_run (overwritten).  A captured graph is dropped (the next graph run
 * captures the tuned launches).  Synchronous. */
typedef struct {
    int32_t level;
    int32_t p1_lines;
    int32_t z_lines;
    double ms;
} gg_zoom_tune_entry;
gg_status gg_zoom_autotune(gg_zoom* zoom, uint64_t seed, void* const* w, void* const* psi, float* const* pos,
                           float* const* vel, void* work, int32_t reps, gg_zoom_tune_entry* results, int32_t capacity,
                           int32_t* count, void* stream);

/* Launch configuration of the fused path: chunks (pipelined launches per pass,
 * 1 = none; 0 keeps the current value), lines per work-group of the first and
 * of the last pass (0 = built-in; otherwise the full LDS row of lines, 16 for
 * float / 8 for double, or half of it).  INVALID_ARG for a choice the lattice
 * does not allow.  Not safe while the plan is in use. */
gg_status gg_plan_set_tuning(gg_plan* plan, int32_t chunks, int32_t p1_lines, int32_t z_lines);

/* Autotuner: times gg_make_ic (one warm-up, then reps calls, HIP events on
 * `stream`) for every valid combination of chunks (1, 2, 4, 8) and the two
 * line counts of the first and last passes (in that order: fewer chunks and
 * full tiles first), keeps the fastest in the plan -- a later combination
 * replaces the best so far only when faster by more than 0.5 %, so that
 * timing noise does not flip near-ties -- and reports each combination (up to `capacity` entries; *count = number
 * timed).  pos, vel, work as for gg_make_ic (overwritten).  Synchronous. */
typedef struct {
    int32_t chunks;
    int32_t p1_lines;
    int32_t z_lines;
    double ms;
} gg_tune_entry;
gg_status gg_plan_autotune(gg_plan* plan, float* pos, float* vel, void* work, int32_t reps, gg_tune_entry* results,
                           int32_t capacity, int32_t* count, void* stream);

/* Per-pass timing of gg_make_ic with HIP events recorded on the call's
 * stream.  Enable before the calls to time; gg_timing_read waits for the last
 * recorded call and returns, for each of the npass passes, the summed
 * milliseconds over the recorded calls, and the number of calls; it then
 * clears the records.  While enabled the plan is not safe for concurrent
 * calls.  npass is 5 (noise + forward z; forward y; forward x + filter +
 * inverse x; inverse y; inverse z + particles).  Passes 1-4 run as
 * gg_plan_info.chunks launches each, two passes overlapping on two streams;
 * their times are summed over those launches. */
gg_status gg_timing_enable(gg_plan* plan, int on);
gg_status gg_timing_read(gg_plan* plan, double* ms_per_pass, int npass, int* ncalls);

const char* gg_status_string(gg_status status);
const char* gg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GG_H */
