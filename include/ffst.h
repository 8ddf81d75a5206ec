/*
 * ffst.h -- C ABI of the MI355X (gfx950) Fast Finite Shearlet Transform.
 *
 * The library computes the finite discrete shearlet transform of the paper
 * "Fast Finite Shearlet Transform: a tutorial" (Haeuser, Steidl):
 *
 *   forward  (eq. shearletTransform, Sec. 3.1):
 *       c_i = ifft2( Psi_i .* fft2(f) ),            i = 0 .. eta-1
 *   adjoint  (eq. inverseShearletTransform, Sec. 3.3):
 *       f   = ifft2( sum_i conj(Psi_i) .* fft2(c_i) )
 *   inverse  = adjoint, because the system is a Parseval frame
 *       (Theorem in Sec. 3.2; Sec. 3.3).
 *
 * fft2 is the unnormalised 2-D DFT with kernel exp(-2 pi i ...); ifft2 carries
 * the factor 1/(M N). Psi_i are the band-limited Meyer-type shearlet spectra
 * (low-pass, every scale j < J and shear k of both cones, and the glued seam
 * elements), evaluated on the grid of Sec. 3.5.1 and made even on the grid by
 * the Nyquist-line fix of Sec. 3.8.1, so every coefficient is real.
 *
 * Layouts (all row-major, float32, contiguous, on the plan's device):
 *   image         f       [batch][M][N]         rows carry omega_2, columns omega_1
 *   coefficients  coeffs  [batch][eta][M][N]    i ordered as in Sec. 3.5.2, i = 0
 *                                               is the low-pass (the paper counts
 *                                               from 1); eta = 2^(J+2) - 3
 *   spectra       Psi     [eta][M][N/2+1]       natural DFT order (no fftshift);
 *                                               columns 0 .. N/2 of each plane,
 *                                               the rest follows from evenness
 *
 * Supported on the GPU: M and N of the form 2^a 3^b in [4, 4096]; 1 <= J <= 10.
 *
 * Ownership: the plan owns the spectra and its tables and frees them in
 * ffst_destroy. The caller owns f, coeffs and the workspace ws (device memory
 * of at least ffst_workspace_size(plan, batch) bytes, 256-byte aligned).
 * Transform calls are asynchronous on the given HIP stream (a hipStream_t
 * passed as void*, NULL = the default stream); they never synchronise the
 * host and never allocate. f and coeffs must not overlap; ws must not overlap
 * either. Two calls that run concurrently need separate workspaces.
 *
 * Threads: transform calls do not modify the plan, so several host threads
 * may call them at once, on one plan or on several, each with its own
 * workspace (and normally its own stream). Creating, tuning and destroying a
 * plan, ffst_set_tuning and the batch calls on one batch must not run
 * concurrently with other calls on the same object. While kernel timing
 * (ffst_profile_*) is enabled, all calls must come from one thread.
 *
 * Errors: every function returns an ffst_status. Arguments are checked
 * before any device work; on failure nothing is launched and nothing is
 * written. ffst_last_error() returns a message for the last failure of the
 * calling thread. No C++ exception crosses this interface.
 */
#ifndef FFST_H
#define FFST_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffst_plan ffst_plan;

typedef enum {
    FFST_OK = 0,
    FFST_EINVAL = 1,        /* bad argument (size, pointer, batch, option) */
    FFST_EUNSUPPORTED = 2,  /* valid for the transform, not for this GPU path */
    FFST_ENOMEM = 3,        /* device allocation failed (plan creation only) */
    FFST_EDEVICE = 4,       /* a HIP call or kernel launch failed */
    FFST_EBADPLAN = 5       /* NULL or destroyed plan */
} ffst_status;

/* Which spectra to generate. */
typedef enum {
    FFST_SHEARLET_MEYER = 0,        /* psi1-hat of eq. (Psi1), cone scaling phi-hat
                                       of eq. (phi); the paper's default */
    FFST_SHEARLET_MEYER_SMOOTH = 1  /* smooth shearlets of Sec. 3.4: psi1-hat
                                       replaced by eq. (newPsi1), tensor
                                       low-pass Phi-hat of eq. (Phi) */
} ffst_shearlet;

typedef struct {
    int max_scale_min;   /* 0: X = 2^(2J-1) ('max', the default); 1: X = 2^(2J-2)
                            ('min'); option maxScale of Sec. 3.5.3 */
    int shearlet;        /* an ffst_shearlet value */
    int complex_shearlets; /* 0: real shearlets (the default). 1: complex
                            shearlets from one-sided spectra (Sec. 3.8.2):
                            Psi+_i = sqrt(2) Psi_i on the side <omega, d_i> > 0
                            of the line through 0 orthogonal to the centre
                            direction d_i of shearlet i (d = (1, -k/2^j) for the
                            h cone and the seam elements, (-k/2^j, 1) for the
                            v cone), 0 on the other side, Psi_i unchanged on
                            that line, on the low-pass, and at grid points
                            whose DFT mirror lies on the same side. The
                            coefficients are complex; such a plan is used with
                            the *_complex transform calls only. */
    int aux_order;       /* auxiliary function v behind every window (Remark on
                            the construction of v): 0 = eq. (v), the default
                            (v'(x) = -140 x^3 (x-1)^3, shearlets in C^3);
                            k in 1 .. 10: v'(x) = c x^k (x-1)^k with v(1) = 1
                            (C^k); -1: the C-infinity function
                            s(x-1) / (s(x-1) + s(x)),
                            s(x) = exp(-(1/(1+x)^2 + 1/(1-x)^2)). Every choice
                            keeps v(x) + v(1-x) = 1, so the frame stays
                            Parseval. */
} ffst_options;

/*
 * Create a plan for M x N images with J scales (J <= 0 selects the default
 * floor(1/2 log2 max(M, N)), Sec. 3.1) and generate its spectra on the
 * current HIP device (once per plan, as Sec. 3.5.1 prescribes). The
 * spectra are evaluated in float64 and stored in float32. Synchronous: on
 * return the plan is ready. *out receives the plan, or NULL on failure.
 */
int ffst_spectra(int M, int N, int J, ffst_plan** out);

/* Same with options (NULL = defaults). */
int ffst_spectra_ex(int M, int N, int J, const ffst_options* opt, ffst_plan** out);

/* Sizes of a plan. Any output pointer may be NULL. */
int ffst_plan_info(const ffst_plan* plan, int* M, int* N, int* J, int* eta);

/* Bytes of workspace a transform call with this batch needs (0 on a bad plan
 * or batch < 0). */
size_t ffst_workspace_size(const ffst_plan* plan, int batch);

/*
 * Copy the plan's float32 spectra into device memory dst (stream-ordered on
 * the default stream, then synchronised): full_plane = 0 writes
 * [eta][M][N/2+1], full_plane = 1 writes [eta][M][N] (the missing columns by
 * evenness, Psi(r, c) = Psi(-r mod M, -c mod N)).
 */
int ffst_get_spectra(const ffst_plan* plan, float* dst, int full_plane);
/* For a complex-shearlet plan only full_plane = 1 is accepted; it writes the
 * one-sided spectra Psi+_i [eta][M][N] (they are not even). */

/*
 * Number of nonzero-column windows used to skip work: writes, for each
 * spectrum i, the first and last column c in [0, N/2] where Psi_i has a
 * nonzero value (host arrays of eta ints each; -1/-1 for an all-zero plane).
 */
int ffst_plan_windows(const ffst_plan* plan, int* first_col, int* last_col);
/* For a complex-shearlet plan the windows are cyclic ranges of full-plane
 * columns c in [0, N): the columns first_col, first_col + 1, ... (mod N) up to
 * last_col, so last_col < first_col when the range wraps past N - 1. */

/*
 * Index order of the coefficient planes (Sec. 3.5.2; what the paper's toolbox
 * helper computes between the index i and scale / shear): plane 0 is the
 * low-pass; scale j (0 .. J-1) follows with 2^(j+2) planes, counter-clockwise:
 * horizontal cone k = 0, -1, .., -2^j+1, the seam element k = -2^j, vertical
 * cone k = -2^j+1 .. 2^j-1, the seam element k = 2^j, horizontal cone
 * k = 2^j-1 .. 1. The dilation and shear of plane (j, k) are a = 4^-j and
 * s = k 2^-j. Pure functions of J (1 <= J <= 10); no plan or GPU needed.
 *
 * ffst_scale_shear writes the kind, j and k of plane i (0 <= i < eta; the
 * low-pass has j = -1, k = 0). ffst_shearlet_index writes the index of
 * (kind, j, k) (for the low-pass j and k are ignored); FFST_EINVAL for a
 * combination that does not occur.
 */
typedef enum {
    FFST_KIND_LOWPASS = 0,
    FFST_KIND_HORIZONTAL = 1,
    FFST_KIND_VERTICAL = 2,
    FFST_KIND_SEAM = 3     /* glued horizontal/vertical element, k = +-2^j */
} ffst_kind;
int ffst_scale_shear(int J, int i, int* kind, int* j, int* k);
int ffst_shearlet_index(int J, int kind, int j, int k, int* i);

/*
 * Forward transform of `batch` images: coeffs[b][i] = ifft2(Psi_i .* fft2(f[b])).
 * batch = 0 is a no-op. Asynchronous on `stream`.
 */
int ffst_forward(const ffst_plan* plan, const float* f, float* coeffs, int batch,
                 void* ws, void* stream);

/*
 * Forward transform for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and kernels as ffst_forward, with the
 * workspace taken from a static device array of the library (64 MiB =
 * 67108864 bytes per GPU, held by every GPU the library runs on until the
 * process ends) instead of a caller buffer. The call allocates
 * nothing and creates no HIP objects (kernel timing is skipped). Batches whose
 * workspace (ffst_workspace_size) exceeds the limit are rejected with
 * FFST_EINVAL before anything runs. The scratch needs no initial contents
 * (every byte the kernels read is written first in the same call). All calls
 * on one GPU share that GPU's array: calls that may overlap in time on one
 * GPU (other streams, other host threads) race and must be serialised by the
 * caller. Real-shearlet plans only; layouts and errors as ffst_forward.
 */
int ffst_forward_noalloc(const ffst_plan* plan, const float* f, float* coeffs, int batch, void* stream);

/*
 * Adjoint: f[b] = ifft2( sum_i Psi_i .* fft2(coeffs[b][i]) ). Overwrites f
 * (does not accumulate). Asynchronous on `stream`.
 */
int ffst_adjoint(const ffst_plan* plan, const float* coeffs, float* f, int batch,
                 void* ws, void* stream);

/* Inverse transform; the same computation as ffst_adjoint (Parseval frame). */
int ffst_inverse(const ffst_plan* plan, const float* coeffs, float* f, int batch,
                 void* ws, void* stream);

/*
 * Adjoint of the l1 subgradient (the gradient step of an l1 penalty on the
 * coefficients, Sec. 3.3 adjoint applied to s * sign(c)): f[b] = SH*(s *
 * sign(coeffs[b])) with sign(0) = 0, computed by ffst_adjoint's kernels with
 * the sign applied as the coefficients are read (no pass over them before).
 * `scale` points to ONE float s in device memory, read when the kernels run
 * (so a gradient scale computed on the device needs no host round trip).
 * Real-shearlet plans only (FFST_EINVAL otherwise); layouts, workspace and
 * errors as ffst_adjoint.
 */
int ffst_adjoint_sign(const ffst_plan* plan, const float* coeffs, float* f, int batch, const float* scale,
                      void* ws, void* stream);

/*
 * Complex shearlets (Sec. 3.8.2), on a plan created with complex_shearlets = 1.
 * Coefficients are complex, stored as interleaved float pairs (re, im):
 * coeffs [batch][eta][M][N][2], 8-byte aligned; the images stay real.
 *
 * Forward: coeffs[b][i] = ifft2(Psi+_i .* fft2(f[b])).
 * Adjoint: f[b] = Re ifft2( sum_i Psi+_i .* fft2(coeffs[b][i]) ), the adjoint
 *   of the forward map for the real inner product on the coefficients.
 * Inverse: the same computation as the adjoint; for real images the one-
 *   sided system is again a Parseval frame, since |Psi+_i(w)|^2 +
 *   |Psi+_i(-w)|^2 = Psi_i(w)^2 + Psi_i(-w)^2 at every grid pair (w, -w).
 * The real-shearlet calls reject complex plans and these calls reject real
 * plans (FFST_EINVAL). Workspace, streams and errors as above.
 */
int ffst_forward_complex(const ffst_plan* plan, const float* f, float* coeffs, int batch,
                         void* ws, void* stream);
int ffst_adjoint_complex(const ffst_plan* plan, const float* coeffs, float* f, int batch,
                         void* ws, void* stream);
int ffst_inverse_complex(const ffst_plan* plan, const float* coeffs, float* f, int batch,
                         void* ws, void* stream);

/*
 * Launch tuning of a plan (runtime knobs only; no setting changes what is
 * computed beyond the order of the adjoint's floating-point sums):
 *   nparts        number of lines the spectra of one column (of one image) are
 *                 spread over in the adjoint's column pass (1 .. 8; 0 = chosen
 *                 from the batch): every line forms a partial sum, and the
 *                 partial sums are added in a fixed order
 *   blocks_per_cu persistent workgroups per compute unit of every kernel
 *                 (1 .. 32; 0 = each kernel's default)
 * The workspace size depends on nparts: query ffst_workspace_size after
 * changing it. ffst_set_tuning keeps the other settings of ffst_tuning.
 */
int ffst_set_tuning(ffst_plan* plan, int nparts, int blocks_per_cu);
int ffst_get_tuning(const ffst_plan* plan, int* nparts, int* blocks_per_cu);

/*
 * All launch settings of a plan, including the kernel shapes compiled in
 * more than one form (real-shearlet passes; the complex shearlets' own column
 * kernels always take the default col_values, and follow nparts and
 * fwd_nparts):
 *   col_values  values per lane of the column-direction FFTs: 0 = the default
 *               for the column length M (8 below 1024, 16 from 1024 on for
 *               powers of two; 12 for 3 * 2^k), or the alternative compiled for
 *               M (16 / 8 for powers of two from 64 on, 6 for 3 * 2^k from 96
 *               on); ffst_get_tuning_ex reports the value in use
 *   row_block   rows per block of the row-direction FFTs: 0 or 1 = the default
 *               height, 2 = the alternative one, twice the default for rows of
 *               up to 512 points (4 .. 16 lanes per row) and half of it for
 *               longer rows (row lengths 64 .. 4096 that are powers of two or
 *               3 * 2^k)
 *   fwd_nparts  number of lines the spectra of one column (of one image) are
 *               spread over in the forward's column pass (1 .. 8; 0 = chosen
 *               from the batch): every line repeats the column's FFT of the
 *               image spectrum and runs every fwd_nparts-th spectrum of the
 *               column; the results do not depend on it
 * Other values are rejected with FFST_EINVAL. Every setting computes the same
 * transform; only the rounding order of the FFT stages and of the adjoint's
 * sums differs.
 */
typedef struct {
    int nparts;
    int blocks_per_cu;
    int col_values;
    int row_block;
    int fwd_nparts;
} ffst_tuning;
int ffst_set_tuning_ex(ffst_plan* plan, const ffst_tuning* tuning);
int ffst_get_tuning_ex(const ffst_plan* plan, ffst_tuning* tuning);

/*
 * Autotuner: times forward + adjoint of `batch` images (f, read) for every
 * setting nparts in {1, 2, 4, 8} x blocks_per_cu in {0, 1, 2, 4, 8, 16} x the
 * compiled col_values x row_block forms (ffst_tuning) whose
 * workspace fits in ws_size bytes (the best of 3 runs after one warm-up, HIP
 * events on `stream`), keeps the fastest, then times the forward alone for
 * fwd_nparts in {1, 2, 4, 8} with it and keeps the fastest of those. coeffs (the
 * coefficient buffer for the plan's kind, as for the transform calls) and
 * out ([batch][M][N]) are scratch. Synchronous. *best_ms (may be NULL)
 * receives the time of one forward + adjoint with the settings kept (best of
 * 3 runs after a warm-up). The tuning calls change
 * the plan: no other call may use the plan while they run.
 */
int ffst_tune(ffst_plan* plan, const float* f, float* coeffs, float* out, int batch, void* ws,
              size_t ws_size, void* stream, double* best_ms);

/*
 * Uneven batches: images of different sizes in one call per direction.
 *
 * ffst_batch_create takes `count` images with sizes M[b] x N[b] and J[b]
 * scales (J[b] <= 0: the default for that size) and the options shared by all
 * of them (NULL = defaults). Images of the same (M, N, J) form a class and
 * share one plan. The batch packs every class contiguously, classes in the
 * order of their first image, each class block starting on a 256-byte
 * boundary (unused floats in between), images of a class in the given order:
 * ffst_batch_layout writes, per image b (host arrays of count entries), the
 * float offset of its image in the packed image buffer and of its
 * coefficients ([eta_b][M_b][N_b], real or complex as the options say) in the
 * packed coefficient buffer, and the two buffers' total float counts.
 *
 * A transform call runs every class on a stream of its own, forked from and
 * joined back into `stream`, and is replayed as one HIP graph: the first call
 * with a given (input, output, workspace) triple captures and instantiates
 * the graph, later calls with the same triple launch it (the graphs of the
 * eight most recently used triples per direction are kept; callers that want
 * every call to be a replay pass the same buffers each time). The workspace must
 * hold ffst_batch_workspace_size bytes (256-byte aligned); calls that run at
 * the same time need separate workspaces. ffst_batch_tune runs ffst_tune for
 * every class, keeps the new settings only if forward + adjoint of the whole
 * batch got faster with them, and drops the captured graphs; a graph captured
 * before a class
 * plan's settings were changed otherwise keeps the settings it was captured
 * with (its results are the same). ffst_batch_class returns a class's plan
 * (owned by the batch) and its image count.
 */
typedef struct ffst_batch ffst_batch;
int ffst_batch_create(int count, const int* M, const int* N, const int* J, const ffst_options* opt,
                      ffst_batch** out);
int ffst_batch_info(const ffst_batch* batch, int* count, int* classes);
int ffst_batch_class(const ffst_batch* batch, int cls, ffst_plan** plan, int* images);
int ffst_batch_layout(const ffst_batch* batch, long long* img_offset, long long* coef_offset,
                      long long* img_total, long long* coef_total);
size_t ffst_batch_workspace_size(const ffst_batch* batch);
int ffst_batch_forward(ffst_batch* batch, const float* f, float* coeffs, void* ws, void* stream);
int ffst_batch_adjoint(ffst_batch* batch, const float* coeffs, float* f, void* ws, void* stream);
int ffst_batch_inverse(ffst_batch* batch, const float* coeffs, float* f, void* ws, void* stream);
int ffst_batch_tune(ffst_batch* batch, const float* f, float* coeffs, float* out, void* ws, void* stream);
void ffst_batch_destroy(ffst_batch* batch);

/* Release a plan (NULL is ignored). Synchronises the device first. */
void ffst_destroy(ffst_plan* plan);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* ffst_last_error(void);

/*
 * Identifier of the sources this library was compiled from: a hash of the
 * kernel and host sources, this header and the compiler flags, fixed at build
 * time (a static string owned by the library). Bindings compare it with the
 * hash of the sources they ship with and refuse a library built from others.
 */
const char* ffst_build_id(void);

/*
 * Bytes of device memory currently held by the plans and batches of this
 * process (spectra, tables; workspaces belong to the caller and are not
 * counted). A leak check for error paths: plan or batch creation that fails
 * releases everything it allocated, so the count returns to its earlier
 * value. Test hook: with the environment variable FFST_FAULT_ALLOC=n (n >= 1),
 * the n-th device allocation inside one ffst_spectra / ffst_spectra_ex /
 * ffst_batch_create call fails as if the device were out of memory, and the
 * call returns FFST_ENOMEM after releasing what it had allocated.
 */
size_t ffst_device_bytes(void);

/*
 * Tracing (no calls; read from the environment once per process):
 *   FFST_LOG=1          plan and batch creation (sizes, windows, hull values,
 *                       device bytes), tuning changes and tuner results,
 *                       destruction, and every error with its status and
 *                       message, one line each on stderr
 *   FFST_LOG=2          also every transform call with its schedule (images
 *                       per unit, lines per column, adjoint form)
 *   FFST_LOG=<l>:<path> level <l> appended to the file <path>; a bare path
 *                       means level 1 into that file; unset, empty or 0: off
 * Independently, every C ABI call and every kernel launch opens a roctx
 * range named after it (ffst_forward, k_fwd_cols, ...), which rocprofv3
 * --marker-trace shows on its timeline.
 */

/*
 * Kernel timing. With profiling enabled, every launch of a kernel whose id
 * bit is set in `mask` is bracketed by two HIP events recorded on the
 * launch's own stream. ffst_profile_read synchronises on the recorded
 * events and returns, for kernel `id`, the summed duration in milliseconds
 * and the number of timed launches since the last reset. Kernel ids are
 * 0 .. ffst_num_kernels()-1; ffst_kernel_name gives the HIP kernel's name.
 * Not thread-safe; meant for benchmarks.
 */
int ffst_profile_enable(unsigned mask);
int ffst_profile_read(int id, double* total_ms, long long* launches);
int ffst_profile_reset(void);
int ffst_num_kernels(void);
const char* ffst_kernel_name(int id);

#ifdef __cplusplus
}
#endif

#endif /* FFST_H */
