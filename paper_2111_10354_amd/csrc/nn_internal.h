// Host-side structures of the preconditioner network.
#pragma once

#include <vector>

#include "solver_internal.h"

namespace hisq {

struct NnGeom {
    int L[4];
    int V;
};

bool nn_channels_supported(int c);
size_t nn_thin_bytes(const NnGeom &G);
int nn_pack_thin(const NnGeom &G, const double *U, void *dst, hipStream_t s);
// Hidden activations: BF16, 8 channels, 96 bytes per site (tiled by 64 sites).
size_t nn_act_bytes(const NnGeom &G);
// Layer input / output modes: 0 = hidden (all sites, BF16 units); 1 = one
// channel on even sites as an FP32 public spinor.
size_t nn_amat_elems(int inm);
void nn_build_amat(const double *W, int cin, int cout, bool transposed, int inm, void *amat, hipStream_t s);
int nn_layer(const NnGeom &G, const void *thin, int inm, int outm, const void *in, void *out, const void *amat,
             hipStream_t s);
size_t nn_wgrad_partial_floats(const NnGeom &G);
int nn_wgrad(const NnGeom &G, const void *thin, int cin, int cout, int inm, int gm, const void *in, const void *grad,
             float *partial, double *gacc, hipStream_t s);
void nn_loss_grad(int vh, const float *out, const float *v, float *gout, double *part, double *scal, int batch,
                  hipStream_t s);
void nn_adam(double *w, double *m, double *v, const double *g, int n, double lr, int step, hipStream_t s);

}  // namespace hisq

struct hisq_nn_s {
    hisq_gauge_s *gauge = nullptr;
    int nlayers = 0;
    std::vector<int> ch;              // channel counts, ch[0] = ch[nlayers] = 1
    std::vector<size_t> woff;         // offset (in doubles) of each layer's weights
    size_t nweights = 0;              // doubles (2 per complex weight)
    hisq::DevBuf w, m, v, g;          // FP64 master weights, Adam moments, gradient
    hisq::DevBuf amat, amat_t;        // bf16 real-block matrices per layer (forward, adjoint)
    std::vector<size_t> aoff;         // element offsets into amat / amat_t
    hisq::DevBuf act;                 // activations of the hidden layers (BF16 units, full lattice)
    hisq::DevBuf gbuf;                // back-propagated gradients (two hidden-size buffers)
    hisq::DevBuf out, gout, partial, scal, partd;
    int step = 0;
    bool amat_valid = false;
    unsigned long long id = 0;        // unique per network created in this process
};
