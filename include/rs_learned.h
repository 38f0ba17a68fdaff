/*
 * rs_learned.h -- options of the learned-CDF bucket path of librs and the
 * entry points that expose its network for gradient checks.  The network
 * is the library's own extension (the paper has none): a monotone MLP
 * 1 -> 32 -> 32 -> 1 with weights softplus(v) >= 0, tanh hidden units and a
 * sigmoid output, trained on (feature of a sampled key, mid-rank of that key
 * in the sample) with Adam.
 *
 * Parameter vector layout (MLP_NPARAM = 1153 floats, device memory):
 *   v1[32] b1[32] v2[32*32] (row-major [out][in]) b2[32] v3[32] b3[1]
 *   h1 = tanh(softplus(v1) x + b1), h2 = tanh(softplus(v2) h1 + b2),
 *   y = sigmoid(softplus(v3) . h2 + b3).
 * All pointers below are device pointers unless stated; calls are
 * asynchronous on `stream` (a hipStream_t) and return argument errors
 * synchronously.
 */
#ifndef RS_LEARNED_H
#define RS_LEARNED_H

#include "rs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t train_steps;          /* Adam steps (default 8)                         */
    float lr;                     /* Adam learning rate (default 1e-2)              */
    int32_t use_network;          /* 0: buckets from the key's feature alone       */
    int32_t bucket_cap;           /* pairs one bucket may hold in LDS (<= 6144)    */
    int32_t feature_mode;         /* -1 automatic (2), 0 linear in the key, 1 log2, */
                                  /* 2 piecewise linear between sample quantiles  */
    double fallback_frac;         /* overflowed-key share above which the whole    */
                                  /* array is sorted by the LSD rounds instead     */
    int32_t train_blocks;         /* workgroups of the training launch             */
    int32_t max_fallback_buckets; /* more overflowed buckets: whole-array LSD      */
} rs_learned_opts;

/* Process-wide options of the LEARNED path (host structs). */
rs_status rs_learned_set_opts(const rs_learned_opts* opts);
rs_status rs_learned_get_opts(rs_learned_opts* opts);

/* Number of network parameters (1153). */
size_t rs_mlp_num_params(void);

/* y[i] = f(x[i]) for i < m (float32, the forward pass the learned path uses). */
rs_status rs_mlp_forward(const float* params, const float* x, float* y, size_t m, void* stream);

/* grad[0..1152] = gradient of mean_i (f(x_i) - t_i)^2 over the m samples with
 * respect to the raw parameters (through the softplus); grad[1153] = the
 * summed squared error.  `grad` holds 1154 floats. */
rs_status rs_mlp_loss_grad(const float* params, const float* x, const float* t, size_t m,
                           float* grad, void* stream);

/* One Adam step (Kingma and Ba 2015, bias-corrected) on the 1153 raw
 * parameters, the update training applies after each gradient: with
 * c1 = 1 - beta1^(step+1) and c2 = 1 - beta2^(step+1) (step counts from 0),
 *   m1 = beta1 m1 + (1 - beta1) g,  m2 = beta2 m2 + (1 - beta2) g^2,
 *   params -= lr (m1 / c1) / (sqrt(m2 / c2) + eps),
 * in float32.  params, m1, m2 (updated) and grad (read only) are device
 * arrays of 1153 floats.  Exposed for checking the update against a
 * double-precision reference. */
rs_status rs_mlp_adam_step(float* params, float* m1, float* m2, const float* grad, int32_t step,
                           float lr, float beta1, float beta2, float eps, void* stream);

/* Test hook: the following LEARNED sorts in this process skip training and
 * use these raw parameters (HOST array of count = 1153 floats, copied
 * here); params = NULL goes back to training.  The weights stay
 * softplus(v) >= 0, so the network stays monotone.  RS_ERR_INVALID for a
 * wrong count.  Not thread-safe against concurrent sorts. */
rs_status rs_mlp_set_weights(const float* params, size_t count);

/* Test hook (fault injection) for the following LEARNED sorts in this
 * process (not thread-safe against concurrent sorts):
 *   RS_LEARNED_FAULT_NONE       no fault (the default);
 *   RS_LEARNED_FAULT_SPLITTERS  `splitters` (HOST array, count = 65535;
 *                               bucket j holds the keys in [s[j-1], s[j]))
 *                               replace the splitters derived from the
 *                               network, as given, not made non-decreasing.
 *                               The bucket search is a fixed binary decision
 *                               tree, so the key-to-bucket map stays
 *                               monotone whatever their order, and the
 *                               output stays the stable sort;
 *   RS_LEARNED_FAULT_SWAP       after the buckets are sorted, the first and
 *                               last output pairs trade places (a planted
 *                               bucket-sort error), which the final
 *                               sortedness check must catch, sending the
 *                               whole array through the LSD rounds.
 * `splitters` and `count` are read only for RS_LEARNED_FAULT_SPLITTERS.
 * RS_ERR_INVALID for an unknown kind or a wrong count. */
enum {
    RS_LEARNED_FAULT_NONE = 0,
    RS_LEARNED_FAULT_SPLITTERS = 1,
    RS_LEARNED_FAULT_SWAP = 2
};
rs_status rs_learned_debug_fault(int kind, const uint64_t* splitters, size_t count);

/* Test hook for the following LEARNED sorts in this process (not
 * thread-safe against concurrent sorts): each sort of n keys also writes,
 * for every input key i, its bucket from evaluating the feature, the
 * network and the calibration directly to direct[i], and its bucket from
 * the splitter search (the ids the two stable rounds sort by) to
 * assigned[i].  The splitters are the smallest keys reaching each bucket,
 * so the two agree wherever the bucket map is non-decreasing in the key.
 * Both are DEVICE arrays of at least n uint16 that the caller owns; NULL
 * for both turns the hook off, one NULL alone is RS_ERR_INVALID. */
rs_status rs_learned_debug_ids(uint16_t* direct, uint16_t* assigned);

#ifdef __cplusplus
}
#endif
#endif
