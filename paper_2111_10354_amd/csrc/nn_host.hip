// Host orchestration of the preconditioner network: creation, weight I/O,
// forward application, loss and gradient over a batch of (A v, v) pairs by
// back-propagation through the adjoint layers, and Adam steps.

#include <algorithm>
#include <atomic>
#include <cstring>

#include "nn_internal.h"

namespace hisq {

static NnGeom nn_geom(const hisq_gauge_s *g) {
    NnGeom G;
    for (int i = 0; i < 4; ++i) G.L[i] = g->dims[i];
    G.V = 2 * g->geom.vh;
    return G;
}

// layer input modes: the first layer (and the adjoint of the last) reads the
// one-channel even-site spinor, every other layer a hidden activation
enum { MODE_HIDDEN = 0, MODE_EVEN = 1 };

int nn_create(hisq_nn_s **out, hisq_gauge_s *g, int nlayers, const int *ch, const double *weights, hipStream_t s) {
    static std::atomic<unsigned long long> next_id{1};
    hisq_nn_s *n = new (std::nothrow) hisq_nn_s();
    if (!n) {
        set_error("network: host allocation failed");
        return HISQ_ERR_OOM;
    }
    n->id = next_id++;
    n->gauge = g;
    n->nlayers = nlayers;
    n->ch.assign(ch, ch + nlayers + 1);
    const NnGeom G = nn_geom(g);
    size_t off = 0, aoff = 0, aoff_t = 0;
    std::vector<size_t> aoff_tv;
    for (int l = 0; l < nlayers; ++l) {
        n->woff.push_back(off);
        off += 2 * 9 * (size_t)ch[l] * ch[l + 1];
        n->aoff.push_back(aoff);
        aoff += nn_amat_elems(l == 0 ? MODE_EVEN : MODE_HIDDEN);
        aoff_tv.push_back(aoff_t);
        aoff_t += nn_amat_elems(l == nlayers - 1 ? MODE_EVEN : MODE_HIDDEN);
    }
    const size_t act = (size_t)(nlayers - 1) * nn_act_bytes(G);
    const size_t part = nn_wgrad_partial_floats(G);
    n->aoff.insert(n->aoff.end(), aoff_tv.begin(), aoff_tv.end());  // [fwd offsets..., adjoint offsets...]
    n->nweights = off;
    int rc;
    if ((rc = n->w.alloc(off * 8)) || (rc = n->m.alloc(off * 8)) || (rc = n->v.alloc(off * 8)) ||
        (rc = n->g.alloc(off * 8)) || (rc = n->amat.alloc(aoff * 2)) || (rc = n->amat_t.alloc(aoff_t * 2)) ||
        (rc = n->act.alloc(std::max<size_t>(act, 16))) || (rc = n->gbuf.alloc(2 * nn_act_bytes(G))) ||
        (rc = n->out.alloc(spinor_bytes(F32, G.V / 2))) || (rc = n->gout.alloc(spinor_bytes(F32, G.V / 2))) ||
        (rc = n->partial.alloc(part * 4)) || (rc = n->scal.alloc(8 * sizeof(double))) ||
        (rc = n->partd.alloc(sizeof(double) * ((G.V / 2 + 255) / 256 + 1)))) {
        delete n;
        return rc;
    }
    std::vector<double> zero(off, 0.0);
    HISQ_HIP_CHECK(hipMemcpyAsync(n->m.p, zero.data(), off * 8, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(n->v.p, zero.data(), off * 8, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipMemcpyAsync(n->w.p, weights ? weights : zero.data(), off * 8, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    *out = n;
    return HISQ_OK;
}

static void build_amats(hisq_nn_s *n, hipStream_t s) {
    const int L = n->nlayers;
    for (int l = 0; l < L; ++l) {
        const double *W = (const double *)n->w.p + n->woff[l];
        nn_build_amat(W, n->ch[l], n->ch[l + 1], false, l == 0 ? MODE_EVEN : MODE_HIDDEN,
                      (__bf16 *)n->amat.p + n->aoff[l], s);
        nn_build_amat(W, n->ch[l], n->ch[l + 1], true, l == L - 1 ? MODE_EVEN : MODE_HIDDEN,
                      (__bf16 *)n->amat_t.p + n->aoff[L + l], s);
    }
    n->amat_valid = true;
}

static void *act_of(hisq_nn_s *n, int l) {  // output of layer l-1 = input of layer l (l >= 1)
    return (char *)n->act.p + (size_t)(l - 1) * nn_act_bytes(nn_geom(n->gauge));
}

// z = N(r): r and z even FP32 spinors (public layout)
int nn_forward(hisq_nn_s *n, const float *in, float *out, hipStream_t s) {
    hisq_gauge_s *g = n->gauge;
    if (!g->thin.p) {
        set_error("the gauge handle has no thin links (hisq_gauge_set_thin)");
        return HISQ_ERR_UNSUPPORTED;
    }
    if (!n->amat_valid) build_amats(n, s);
    const NnGeom G = nn_geom(g);
    const int L = n->nlayers;
    int rc;
    for (int l = 0; l < L; ++l) {
        const void *src = l == 0 ? (const void *)in : act_of(n, l);
        void *dst = l == L - 1 ? (void *)out : act_of(n, l + 1);
        const int inm = l == 0 ? MODE_EVEN : MODE_HIDDEN, outm = l == L - 1 ? MODE_EVEN : MODE_HIDDEN;
        if ((rc = nn_layer(G, g->thin.p, inm, outm, src, dst, (const __bf16 *)n->amat.p + n->aoff[l], s))) return rc;
    }
    return HISQ_OK;
}

// Loss over a batch and its gradient, accumulated into n->g (overwritten);
// the loss ends in scal[3].
int nn_loss_grad_batch(hisq_nn_s *n, int batch, const float *av, const float *v, hipStream_t s) {
    hisq_gauge_s *g = n->gauge;
    const NnGeom G = nn_geom(g);
    const int vh = G.V / 2, L = n->nlayers;
    const size_t sb = spinor_bytes(F32, vh);
    int rc;
    HISQ_HIP_CHECK(hipMemsetAsync(n->g.p, 0, n->nweights * 8, s));
    HISQ_HIP_CHECK(hipMemsetAsync(n->scal.p, 0, 8 * sizeof(double), s));
    void *gb[2] = {n->gbuf.p, (char *)n->gbuf.p + nn_act_bytes(G)};
    for (int i = 0; i < batch; ++i) {
        const float *avi = (const float *)((const char *)av + sb * i);
        const float *vi = (const float *)((const char *)v + sb * i);
        if ((rc = nn_forward(n, avi, (float *)n->out.p, s))) return rc;
        nn_loss_grad(vh, (const float *)n->out.p, vi, (float *)n->gout.p, (double *)n->partd.p, (double *)n->scal.p,
                     batch, s);
        const void *gcur = n->gout.p;
        int gmode = MODE_EVEN;
        for (int l = L - 1; l >= 0; --l) {
            const void *inl = l == 0 ? (const void *)avi : act_of(n, l);
            const int inm = l == 0 ? MODE_EVEN : MODE_HIDDEN;
            if ((rc = nn_wgrad(G, g->thin.p, n->ch[l], n->ch[l + 1], inm, gmode, inl, gcur, (float *)n->partial.p,
                               (double *)n->g.p + n->woff[l], s)))
                return rc;
            if (l > 0) {
                void *gn = gb[l & 1];
                if ((rc = nn_layer(G, g->thin.p, gmode, MODE_HIDDEN, gcur, gn,
                                   (const __bf16 *)n->amat_t.p + n->aoff[L + l], s)))
                    return rc;
                gcur = gn;
                gmode = MODE_HIDDEN;
            }
        }
    }
    return HISQ_OK;
}

}  // namespace hisq

using namespace hisq;

static int nfail(int code, const char *msg) {
    set_error(msg);
    return code;
}

extern "C" {

int hisq_gauge_set_thin(hisq_gauge_t g, const double *thin, void *stream) {
    if (!g || !thin) return nfail(HISQ_ERR_INVALID, "gauge and thin links are required");
    std::lock_guard<std::mutex> lk(g->mu);
    const NnGeom G = nn_geom(g);
    int rc = g->thin.alloc(nn_thin_bytes(G));
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if ((rc = nn_pack_thin(G, thin, g->thin.p, s))) return rc;
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    return HISQ_OK;
}

int hisq_nn_create(hisq_nn_t *out, hisq_gauge_t g, int nlayers, const int *channels, const double *weights,
                   void *stream) {
    if (!out || !g || !channels) return nfail(HISQ_ERR_INVALID, "out, gauge and channels are required");
    *out = nullptr;
    if (nlayers < 1 || nlayers > 8) return nfail(HISQ_ERR_INVALID, "1 <= nlayers <= 8");
    if (channels[0] != 1 || channels[nlayers] != 1)
        return nfail(HISQ_ERR_INVALID, "the first and last channel counts must be 1");
    for (int l = 0; l <= nlayers; ++l)
        if (!nn_channels_supported(channels[l])) return nfail(HISQ_ERR_UNSUPPORTED, "channel counts must be in 1..8");
    std::lock_guard<std::mutex> lk(g->mu);
    return nn_create(out, g, nlayers, channels, weights, (hipStream_t)stream);
}

int hisq_nn_destroy(hisq_nn_t net) {
    if (!net) return HISQ_OK;
    (void)hipDeviceSynchronize();
    delete net;
    return HISQ_OK;
}

int hisq_nn_num_weights(hisq_nn_t net, size_t *n_complex) {
    if (!net || !n_complex) return nfail(HISQ_ERR_INVALID, "net and n_complex are required");
    *n_complex = net->nweights / 2;
    return HISQ_OK;
}

int hisq_nn_get_weights(hisq_nn_t net, double *weights, void *stream) {
    if (!net || !weights) return nfail(HISQ_ERR_INVALID, "net and weights are required");
    hipStream_t s = (hipStream_t)stream;
    HISQ_HIP_CHECK(hipMemcpyAsync(weights, net->w.p, net->nweights * 8, hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    return HISQ_OK;
}

int hisq_nn_set_weights(hisq_nn_t net, const double *weights, void *stream) {
    if (!net || !weights) return nfail(HISQ_ERR_INVALID, "net and weights are required");
    hipStream_t s = (hipStream_t)stream;
    HISQ_HIP_CHECK(hipMemcpyAsync(net->w.p, weights, net->nweights * 8, hipMemcpyHostToDevice, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    net->amat_valid = false;
    return HISQ_OK;
}

int hisq_nn_loss_grad(hisq_nn_t net, int batch, const void *av, const void *v, double *loss, double *grad,
                      void *stream) {
    TraceRange tr_("hisq_nn_loss_grad");
    if (!net || !av || !v || batch < 1) return nfail(HISQ_ERR_INVALID, "net, av, v and batch >= 1 are required");
    if (!net->gauge->thin.p) return nfail(HISQ_ERR_UNSUPPORTED, "the gauge handle has no thin links");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(net->gauge->mu);
    int rc = nn_loss_grad_batch(net, batch, (const float *)av, (const float *)v, s);
    if (rc) return rc;
    double sc[8];
    HISQ_HIP_CHECK(hipMemcpyAsync(sc, net->scal.p, sizeof(sc), hipMemcpyDeviceToHost, s));
    if (grad) HISQ_HIP_CHECK(hipMemcpyAsync(grad, net->g.p, net->nweights * 8, hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    if (loss) *loss = sc[3];
    return HISQ_OK;
}

int hisq_nn_train_step(hisq_nn_t net, int batch, const void *av, const void *v, double lr, double *loss,
                       void *stream) {
    TraceRange tr_("hisq_nn_train_step");
    if (!net || !av || !v || batch < 1 || !(lr > 0.0))
        return nfail(HISQ_ERR_INVALID, "net, av, v, batch >= 1 and lr > 0 are required");
    if (!net->gauge->thin.p) return nfail(HISQ_ERR_UNSUPPORTED, "the gauge handle has no thin links");
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(net->gauge->mu);
    int rc = nn_loss_grad_batch(net, batch, (const float *)av, (const float *)v, s);
    if (rc) return rc;
    net->step += 1;
    nn_adam((double *)net->w.p, (double *)net->m.p, (double *)net->v.p, (const double *)net->g.p,
            (int)net->nweights, lr, net->step, s);
    net->amat_valid = false;
    double sc[8];
    HISQ_HIP_CHECK(hipMemcpyAsync(sc, net->scal.p, sizeof(sc), hipMemcpyDeviceToHost, s));
    HISQ_HIP_CHECK(hipStreamSynchronize(s));
    if (loss) *loss = sc[3];
    return HISQ_OK;
}

int hisq_precond_apply(hisq_gauge_t g, hisq_nn_t net, const void *in, void *out, void *stream) {
    if (!g) return nfail(HISQ_ERR_INVALID, "gauge handle is NULL");
    if (!net || !in || !out) return nfail(HISQ_ERR_INVALID, "net, in and out are required");
    if (net->gauge != g) return nfail(HISQ_ERR_INVALID, "the network belongs to another gauge handle");
    if (in == out) return nfail(HISQ_ERR_INVALID, "in and out must not overlap");
    if (((uintptr_t)in & 15) || ((uintptr_t)out & 15)) return nfail(HISQ_ERR_INVALID, "buffers must be 16-byte aligned");
    std::lock_guard<std::mutex> lk(g->mu);
    return nn_forward(net, (const float *)in, (float *)out, (hipStream_t)stream);
}

}  // extern "C"
