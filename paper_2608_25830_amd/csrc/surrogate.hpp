// surrogate.hpp -- host-side view of the learned collision surrogate
// (kernels in surrogate.hip).
#pragma once

#include <cmath>

#include "gtmp_launch.hpp"

namespace gtmp {

// Offsets (elements) of the parameter blocks in the flat parameter arrays.
struct SurLayout {
    int W[4], b[4];  // hidden layers 1..4
    int w5, b5;      // output layer
    int total;
};
SurLayout sur_layout();

struct SurNet {
    int d;
    const float *fourier;  // [16][d]
    float *p32;            // FP32 parameters
    uint16_t *p16;         // BF16 copy
};

struct SurBox {
    float lo[GTMP_MAX_DOF], wd[GTMP_MAX_DOF];
};

size_t sur_workspace_bytes(int64_t n);
int64_t sur_rows_for(size_t bytes);  // rows per inference chunk that fit `bytes`
size_t sur_infer_bytes(int64_t n);   // inference workspace for n rows per chunk

hipError_t launch_sur_infer(const SurNet &net, int64_t n, const float *X, float *logits, void *ws, size_t ws_bytes,
                            hipStream_t s);
hipError_t launch_sur_grad(const SurNet &net, int n, const float *X, const uint8_t *y, float *grad, float *loss,
                           float *logits, void *ws, hipStream_t s);
hipError_t launch_sur_adam(const SurNet &net, const float *grad, float *m, float *v, int t, float lr, float b1,
                           float b2, float eps, hipStream_t s);
hipError_t launch_sur_refresh(const SurNet &net, hipStream_t s);
hipError_t launch_sur_label_states(const gtmp_problem &p, uint64_t seed, uint64_t stage, int64_t n, float *X,
                                   hipStream_t s);
// Pruning threshold of the surrogate (select.hip): the k-th smallest logit
// among the edges with flag 0, k = ceil(recall n_free) - 1; +inf without
// free edges.  tau is a device float.
size_t sur_threshold_bytes();
hipError_t launch_sur_threshold(const float *logits, const uint8_t *flags, int64_t E, double recall, float *tau,
                                void *workspace, hipStream_t s);
size_t sur_prune_bytes(const gtmp_problem &p);  // workspace of launch_sur_prune
hipError_t launch_sur_prune(const gtmp_problem &p, const SurNet &net, const float *q0, const float *goals,
                            const float *Q, const uint8_t *vcoll, float tau, uint8_t *prune, float *logits, void *ws,
                            hipStream_t s);

}  // namespace gtmp
