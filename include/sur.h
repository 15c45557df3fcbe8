/*
 * sur.h -- C ABI of the surrogate part of libens: a small multilayer
 * perceptron that predicts the Keller--Miksis response from the drive
 * parameters, trained and evaluated on the GPU with BF16 matrix-core kernels
 * (FP32 accumulation), used to screen large (p_A, f) sweeps so that only the
 * points it flags or is unsure about are re-solved by the FP64 integrator.
 *
 * The paper (Nagy, Plavecz, Hegedus, arXiv:2011.01740) has no learned
 * component.  What the network predicts is the paper's quantity: the maximum
 * bubble radius y1max per acoustic cycle, recorded after every successful
 * step without dense output, over the converged cycles of a frequency sweep
 * (Sec. 4.2).  Architecture, loss, optimiser and screening rule are this
 * library's definitions:
 *   - network 2 -> 256 -> 256 -> 256 -> 64, linear output; parameters packed
 *     W1, b1, W2, b2, W3, b3, W4, b4, each W row-major with shape (out, in),
 *     z = a W^T + b (148,800 parameters);
 *   - layer 1 is a fixed random Fourier-feature map, a1 = sin(x W1^T + b1):
 *     W1 holds 128 frequency vectors (each twice) and b1 the phases 0 and
 *     pi/2, so a1 carries the sine and cosine of every frequency; W1 and b1
 *     come with sur_set_params and are never trained (their gradients are
 *     0 and Adam leaves them).  Without it a network of this size smooths
 *     the response's sharp resonance and bifurcation edges away (spectral
 *     bias): on the 4096 x 4096 sweep it mislabels 2.2% of the points alone,
 *     five times the 0.43% of bilinear interpolation of its training grid;
 *   - layers 2 and 3: GELU, z Phi(z) with Phi the standard normal CDF; on
 *     the GPU the normal tail comes from the rational approximation of
 *     Abramowitz and Stegun eq. 7.1.26 (|error| <= 1.5e-7) and the features'
 *     sine from the hardware sine of an FP32 argument, in training and in
 *     inference alike;
 *   - input: (p_A, ln f) mapped linearly to [-1, 1] with the bounds given to
 *     sur_set_norm; output: the 64 values ln y1max of the last 64 cycles in
 *     decreasing order (sur_fit_norm and sur_build_dataset sort each point's
 *     records; output 0 is the largest maximum, the value the screen labels
 *     by, and the order does not depend on where a periodic or chaotic
 *     response's cycle starts in the window), standardised per output with
 *     the mean / std given to sur_set_norm;
 *   - loss: weighted mean squared error sum_j w_j (out_j - t_j)^2 over batch
 *     and outputs divided by their count, output 0 weighted 32 times the
 *     others, the weights scaled to mean 1; Adam on FP32 master weights; the
 *     layer-1 product (K = 2) runs in FP32 on the vector unit, every other
 *     product takes BF16 operands (round to nearest even) with FP32
 *     accumulation;
 *   - screening: label = [max_j y1max_j >= 2] from the de-standardised
 *     prediction; a point is re-solved if |max_j ln y1max_j - ln 2| < margin,
 *     or if the predicted spread max_j - min_j exceeds `spread` while
 *     |max_j - ln 2| < flag_margin, or if the exact labels of the training
 *     nodes around it (sur_fit_label_map) contradict the network's label:
 *     all four of them, or some of them while |max_j - ln 2| < label_margin.
 *
 * Conventions are those of ens.h: functions return ENS_OK or a negative
 * ens_status; arrays tagged with `where` are host (ENS_HOST) or device
 * (ENS_DEVICE) memory on the handle's device; work is ordered on the
 * handle's stream; host outputs are complete when the call returns.
 */
#ifndef LIBENS_SUR_H_
#define LIBENS_SUR_H_

#include <stddef.h>
#include <stdint.h>

#include "ens.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sur_ctx *sur_t;

#define SUR_N_PARAMS 148800
#define SUR_IN 2
#define SUR_HIDDEN 256
#define SUR_OUT 64

/* Creates a surrogate on `device`, enqueuing on `hip_stream` (NULL: null
 * stream).  max_batch (a positive multiple of 64, <= 65536) bounds the batch
 * of sur_train_step / sur_gradients.  Parameters start at zero; call
 * sur_set_params.  Errors: ENS_E_INVAL, ENS_E_NOMEM, ENS_E_HIP. */
int sur_create(int32_t device, void *hip_stream, int64_t max_batch, sur_t *out);
int sur_destroy(sur_t s);
const char *sur_last_error(sur_t s);

/* FP32 master parameters := flat (host, SUR_N_PARAMS doubles, rounded to
 * FP32); the BF16 copies are refreshed and the Adam state and step count are
 * reset.  sur_get_params copies the FP32 master parameters out as doubles. */
int sur_set_params(sur_t s, const double *flat);
int sur_get_params(sur_t s, double *flat);

/* Input bounds (in_lo, in_hi: p_A [Pa] and ln f) and output standardisation
 * (out_mean, out_std: SUR_OUT values each, std > 0).  Host arrays. */
int sur_set_norm(sur_t s, const double *in_lo, const double *in_hi,
                 const double *out_mean, const double *out_std);

/* Training inputs from a Keller--Miksis sweep: params [2][n] (P_A1, f1), and
 * records: the last SUR_OUT cycle maxima y1max as a [SUR_OUT][n] double array
 * (consecutive record slots, in any order).  Writes x [n][2] (normalised
 * inputs) and y [n][SUR_OUT] (each point's ln y1max in decreasing order,
 * standardised) as float, all device pointers.  Uses the bounds and
 * standardisation set by sur_set_norm.  The sorted copy of the records
 * lives in handle-owned scratch (grown on first use). */
int sur_build_dataset(sur_t s, const double *params, const double *records, int64_t n,
                      float *x, float *y);

/* Output standardisation fitted on the GPU: for each of the SUR_OUT record
 * ranks of records [SUR_OUT][n] (device, double; each point's maxima taken
 * in decreasing order, as sur_build_dataset does), mean and standard
 * deviation of ln y1max over the n points; they become the handle's output
 * standardisation (input bounds as given here) and are copied to out_mean /
 * out_std (host, SUR_OUT doubles each, may be NULL). */
int sur_fit_norm(sur_t s, const double *in_lo, const double *in_hi, const double *records,
                 int64_t n, double *out_mean, double *out_std);

/* Adam hyper-parameters (defaults lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8). */
int sur_set_adam(sur_t s, double lr, double beta1, double beta2, double eps);

/* One training step on a batch: forward, loss, backward, Adam.  x [m][2],
 * target [m][SUR_OUT] float (normalised / standardised), m a positive
 * multiple of 64 <= max_batch.  If loss is not NULL it receives the batch
 * loss (a float; host or device per `where`, which also tags x and target). */
int sur_train_step(sur_t s, const float *x, const float *target, int64_t m,
                   float *loss, int32_t where);

/* One pass over rows of a device dataset x [rows][2], y [rows][SUR_OUT]:
 * perm (device int64 [n]) lists the rows to use in order (each a valid row
 * index; a shuffled training subset); consecutive batches of `batch` entries
 * (a multiple of 64 <= max_batch; the last n mod batch are skipped), one
 * sur_train_step each.  *mean_loss (host, may be NULL) receives the mean of
 * the batch losses. */
int sur_train_epoch(sur_t s, const float *x, const float *y, int64_t n, const int64_t *perm,
                    int64_t batch, float *mean_loss);

/* `epochs` passes over the training rows rows[0 .. n) (device int64, row
 * indices of the device dataset x [..][2], y [..][SUR_OUT]), batches as in
 * sur_train_epoch; epoch e uses learning rate lr[e] (host, > 0) and a seeded
 * random order of the rows: the rows sorted by the SplitMix64 output function
 * of seed + 0x9E3779B97F4A7C15 (e n + i + 1) for the i-th row (ties in row
 * order).  One epoch's launches are captured as a graph and replayed with
 * each epoch's order, learning rate and step count from device memory, with
 * no host synchronisation between epochs.  losses (host, `epochs` floats,
 * may be NULL) receives each epoch's mean batch loss.  The handle's Adam
 * betas / epsilon apply; its learning rate is not changed. */
int sur_train_epochs(sur_t s, const float *x, const float *y, const int64_t *rows, int64_t n,
                     int64_t batch, int64_t epochs, const double *lr, uint64_t seed,
                     float *losses);

/* Loss and gradients of one batch without an update (for checking): grads
 * receives SUR_N_PARAMS floats in the parameter packing. */
int sur_gradients(sur_t s, const float *x, const float *target, int64_t m, float *grads,
                  float *loss, int32_t where);

/* Network output (standardised) for m inputs x [m][2] -> out [m][SUR_OUT].
 * One launch of the fused inference kernel (every layer, 32 points per
 * wave) for device arrays; host arrays pass through the handle's staging
 * buffers 65,536 rows at a time.  m may be any size >= 0. */
int sur_forward(sur_t s, const float *x, int64_t m, float *out, int32_t where);

typedef struct {
  double margin;       /* unsure band on max_j ln y1max around ln 2          */
  double spread;       /* flag: predicted max_j - min_j above this ...       */
  double flag_margin;  /* ... and |max_j ln y1max - ln 2| below this         */
  double label_margin; /* flag from the training grid's exact labels (needs
                          sur_fit_label_map; < 0: off): with k of the four
                          training nodes around the point carrying a label
                          other than the network's, flag if k = 4, or if
                          k >= 1 and |max_j ln y1max - ln 2| is below this   */
} sur_screen_opts;

/* Exact labels of a G x G training grid (km-grid order, the axes of
 * sur_set_norm) from its records [SUR_OUT][G*G] (device, double): node label
 * [max_j y1max_j >= 2], or -1 where a record is NaN.  The map stays in the
 * handle for sur_screen's label flag (the four nodes of the grid cell around
 * each screened point are looked up) and is copied to map_out (device int8
 * [G*G], may be NULL). */
int sur_fit_label_map(sur_t s, const double *records, int32_t G, int8_t *map_out);

/* Sizes the handle's compaction scratch for screens of up to n_screen
 * points, so that those sur_screen calls allocate nothing (sur_screen grows
 * it on demand otherwise).  For callers that time or capture the screen. */
int sur_reserve(sur_t s, int64_t n_screen);

/* Screens n sweep points params [2][n] (P_A1, f1; double).  Device outputs:
 * label [n] int8 (1: max y1max >= 2), resolve [n] uint8, pred_max [n] float
 * (predicted max_j ln y1max), resolve_idx [n] int64 receiving the indices of
 * the points to re-solve in ascending order; *n_resolve (host) their count.
 * Any output pointer except n_resolve may be NULL.  All array pointers are
 * device memory.  The network and the screening rule run as one launch over
 * all n points (the inputs normalised in the kernel, no intermediate arrays);
 * the re-solve list is then compacted in a fixed order.  Returns when the
 * outputs are complete. */
int sur_screen(sur_t s, const double *params, int64_t n, const sur_screen_opts *opts,
               int8_t *label, uint8_t *resolve, float *pred_max, int64_t *resolve_idx,
               int64_t *n_resolve);

/* Exact labels from re-solved points: for i < k, label[idx[i]] =
 * [max_j records[j][i] >= 2] with records [SUR_OUT][k] the cycle maxima of
 * the re-solved systems (device arrays; a point whose records hold a NaN is
 * labelled -1).  With idx == NULL, label[i] is written for i < k. */
int sur_exact_labels(sur_t s, const double *records, int64_t k, const int64_t *idx,
                     int8_t *label);

#ifdef __cplusplus
}
#endif
#endif /* LIBENS_SUR_H_ */
