// C ABI of the perception residual network (paper Sec. 3.3): the network
// object (parameters, AdamW state, operand packings, activation workspace),
// its forward and training step, and single-layer calls.  Host code only
// orders kernel launches; every step runs in prnet.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ctx.h"

using namespace me;

namespace {

enum { kDw = 0, kPw = 1 };

struct Layer {
    int kind, ci, co, s, relu6;
    int64_t off_w, off_b;     // in the flat parameter vector
    size_t fwd, bwd;          // offsets (bfloat16 elements) of the packed operands
    int MT, KS, MTb, KSb, c0b, crb;
};

inline int div_up(int a, int b) { return (a + b - 1) / b; }
inline int osz(int n, int s) { return (n - 1) / s + 1; }

std::vector<Layer> make_layers(const me_prnet_cfg& c)
{
    const int e = c.c_enc, h = c.c_hid, x = c.c_hid * c.expand;
    std::vector<Layer> L;
    auto add = [&](int kind, int ci, int co, int s, int r) { L.push_back(Layer{kind, ci, co, s, r}); };
    add(kDw, 4, 4, 2, 1);
    add(kPw, 4, e, 1, 1);
    add(kDw, e, e, 2, 1);
    add(kPw, e, e, 1, 1);
    add(kPw, c.c_feat + e, h, 1, 1);
    for (int b = 0; b < c.n_blocks; ++b) {
        add(kPw, h, x, 1, 1);
        add(kDw, x, x, 1, 1);
        add(kPw, x, h, 1, 0);
    }
    add(kPw, h, c.c_feat, 1, 0);
    int64_t off = 0;
    size_t pk = 0;
    for (size_t i = 0; i < L.size(); ++i) {
        Layer& l = L[i];
        l.off_w = off;
        off += (int64_t)l.co * (l.kind == kDw ? 9 : l.ci);
        l.off_b = off;
        off += l.co;
        if (l.kind == kPw) {
            l.MT = div_up(l.co, 16);
            l.KS = div_up(l.ci, 16);
            l.c0b = i == 4 ? c.c_feat : 0;          // the projection's input gradient covers the encoder part only
            l.crb = l.ci - l.c0b;
            l.MTb = div_up(l.crb, 16);
            l.KSb = div_up(l.co, 16);
            l.fwd = pk;
            pk += (size_t)l.MT * l.KS * 256;
            l.bwd = pk;
            pk += (size_t)l.MTb * l.KSb * 256;
        }
    }
    return L;
}

me_status check_cfg(const me_prnet_cfg* c)
{
    if (!c) return fail(ME_E_INVAL, "prnet: null configuration");
    if (c->c_feat < 16 || c->c_enc < 16 || c->c_hid < 16 || c->c_feat % 16 || c->c_enc % 16 || c->c_hid % 16)
        return fail(ME_E_INVAL, "prnet: channel counts must be positive multiples of 16");
    if (c->expand < 1 || c->expand > 16 || c->n_blocks < 0 || c->n_blocks > 16)
        return fail(ME_E_INVAL, "prnet: expand must be 1..16 and n_blocks 0..16");
    const int x = c->c_hid * c->expand;
    if (c->c_feat + c->c_enc > 1024 || x > 1024 || c->c_feat + c->c_enc + c->c_hid > 1024 || x + c->c_hid > 1024 ||
        c->c_feat + c->c_hid > 1024)
        return fail(ME_E_UNSUPPORTED, "prnet: layer widths beyond 1024 channels are not supported");
    return ME_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

PwTensor nhwc(const void* p, int C) { return PwTensor{p, C, 0, 0}; }
PwTensor none() { return PwTensor{nullptr, 0, 0, 0}; }

// Device buffer grown on demand; growth waits for the device so that no queued
// work still reads the old buffer.
me_status grow(void** p, size_t* cap, size_t bytes)
{
    if (bytes <= *cap) return ME_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, bytes) != hipSuccess) return fail(ME_E_NOMEM, "prnet: out of device memory (%zu bytes)", bytes);
    *cap = bytes;
    return ME_OK;
}

constexpr int kWgTarget = 512;   // workgroups of a weight-gradient reduction

size_t pw_partial_floats(int P, int cin, int cout)
{
    return (size_t)div_up(P, wgrad_chunk(P, kWgTarget)) * ((size_t)cout * cin + cout);
}

// Partial floats of a depthwise weight gradient over n images of H x W inputs.
size_t dw_partial_floats(int n, int H, int W, int S, int C)
{
    return (size_t)dw_wgrad_nwg(n, osz(H, S), osz(W, S)) * C * 10;
}

hipError_t dw_wgrad(const uint16_t* x, const uint16_t* dy, float* partial, float* gw, float* gb, int n, int H, int W,
                    int C, int S, hipStream_t st)
{
    return launch_dw_wgrad(x, dy, partial, gw, gb, n, H, W, C, S, st);
}

}  // namespace

// ------------------------------------------------------------------ net --

struct me_prnet_s {
    int device = 0;
    me_prnet_cfg cfg{};
    std::vector<Layer> L;
    int64_t np = 0;
    float* params = nullptr;
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    uint16_t* packs = nullptr;
    bool loaded = false;
    int64_t step = 0;
    void* ws = nullptr;
    size_t ws_cap = 0;
    void* partial = nullptr;
    size_t partial_cap = 0;
    // workspace views for the current call
    int n = 0, Hp = 0, Wp = 0, H1 = 0, W1 = 0, Hf = 0, Wf = 0;
    uint16_t *a0, *e1, *e2, *e3, *e4, *zl;
    std::vector<uint16_t*> h, u, v_;
    float* r;
    uint16_t *dr, *gA, *gB, *dh[2];
    int32_t* nbad;
    uint32_t* maxbits;
    float* lpart;
    uint8_t* flags;
    ~me_prnet_s()
    {
        (void)hipSetDevice(device);
        (void)hipDeviceSynchronize();
        (void)hipFree(params);
        (void)hipFree(grads);
        (void)hipFree(m);
        (void)hipFree(v);
        (void)hipFree(packs);
        (void)hipFree(ws);
        (void)hipFree(partial);
    }
};

namespace {

size_t packs_elems(const std::vector<Layer>& L)
{
    size_t n = 0;
    for (const Layer& l : L)
        if (l.kind == kPw) n = l.bwd + (size_t)l.MTb * l.KSb * 256;
    return n;
}

hipError_t repack(me_prnet net, hipStream_t st)
{
    for (const Layer& l : net->L) {
        if (l.kind != kPw) continue;
        const float* w = net->params + l.off_w;
        hipError_t e = launch_pw_pack(w, l.ci, 0, 0, l.co, l.ci, l.MT, l.KS, net->packs + l.fwd, st);
        if (e == hipSuccess) e = launch_pw_pack(w, l.ci, l.c0b, 1, l.crb, l.co, l.MTb, l.KSb, net->packs + l.bwd, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Carve the workspace for n frames of Hp x Wp packed pixels.
me_status layout(me_prnet net, int n, int Hp, int Wp, bool train)
{
    const me_prnet_cfg& c = net->cfg;
    const int H1 = osz(Hp, 2), W1 = osz(Wp, 2), Hf = osz(H1, 2), Wf = osz(W1, 2);
    const size_t P0 = (size_t)n * Hp * Wp, P1 = (size_t)n * H1 * W1, P2 = (size_t)n * Hf * Wf;
    const int X = c.c_hid * c.expand, nb = c.n_blocks;
    std::vector<size_t> sz;   // bytes, in carve order
    sz.push_back(P0 * 4 * 2);                    // a0
    sz.push_back(P1 * 4 * 2);                    // e1
    sz.push_back(P1 * c.c_enc * 2);              // e2
    sz.push_back(P2 * c.c_enc * 2);              // e3
    sz.push_back(P2 * c.c_enc * 2);              // e4
    for (int k = 0; k <= nb; ++k) sz.push_back(P2 * c.c_hid * 2);   // h
    for (int k = 0; k < nb; ++k) sz.push_back(P2 * X * 2);          // u
    for (int k = 0; k < nb; ++k) sz.push_back(P2 * X * 2);          // v
    sz.push_back(P2 * c.c_feat * 2);                                  // z_pred, channels-last bfloat16
    size_t gmax = 0;
    if (train) {
        sz.push_back(P2 * c.c_feat * 4);         // r
        sz.push_back(P2 * c.c_feat * 2);         // dr
        gmax = std::max(std::max(P1 * c.c_enc, P1 * 4), P2 * (size_t)std::max(std::max(X, c.c_hid), c.c_enc)) * 2;
        sz.push_back(gmax);                      // gA
        sz.push_back(gmax);                      // gB
        sz.push_back(P2 * c.c_hid * 2);          // dh[0]
        sz.push_back(P2 * c.c_hid * 2);          // dh[1]
        sz.push_back(16);                        // nbad, maxbits
        sz.push_back((size_t)prloss_blocks((int)P2) * 4);
        sz.push_back(P2);                        // loss flags
    }
    size_t total = 0;
    for (size_t s : sz) total += (s + 255) & ~(size_t)255;
    me_status st = grow(&net->ws, &net->ws_cap, total);
    if (st != ME_OK) return st;
    uint8_t* p = static_cast<uint8_t*>(net->ws);
    size_t i = 0;
    auto take = [&]() {
        uint8_t* q = p;
        p += (sz[i++] + 255) & ~(size_t)255;
        return q;
    };
    net->a0 = (uint16_t*)take();
    net->e1 = (uint16_t*)take();
    net->e2 = (uint16_t*)take();
    net->e3 = (uint16_t*)take();
    net->e4 = (uint16_t*)take();
    net->h.assign(nb + 1, nullptr);
    net->u.assign(nb, nullptr);
    net->v_.assign(nb, nullptr);
    for (int k = 0; k <= nb; ++k) net->h[k] = (uint16_t*)take();
    for (int k = 0; k < nb; ++k) net->u[k] = (uint16_t*)take();
    for (int k = 0; k < nb; ++k) net->v_[k] = (uint16_t*)take();
    net->zl = (uint16_t*)take();
    if (train) {
        net->r = (float*)take();
        net->dr = (uint16_t*)take();
        net->gA = (uint16_t*)take();
        net->gB = (uint16_t*)take();
        net->dh[0] = (uint16_t*)take();
        net->dh[1] = (uint16_t*)take();
        uint8_t* q = take();
        net->nbad = (int32_t*)q;
        net->maxbits = (uint32_t*)(q + 4);
        net->lpart = (float*)take();
        net->flags = (uint8_t*)take();
        size_t pf = 0;
        // partials: the largest layer reduction
        pf = std::max(pf, dw_partial_floats(n, Hp, Wp, 2, 4));
        pf = std::max(pf, pw_partial_floats((int)P1, 4, c.c_enc));
        pf = std::max(pf, dw_partial_floats(n, H1, W1, 2, c.c_enc));
        pf = std::max(pf, pw_partial_floats((int)P2, c.c_enc, c.c_enc));
        pf = std::max(pf, pw_partial_floats((int)P2, c.c_feat + c.c_enc, c.c_hid));
        pf = std::max(pf, pw_partial_floats((int)P2, c.c_hid, X));
        pf = std::max(pf, dw_partial_floats(n, Hf, Wf, 1, X));
        pf = std::max(pf, pw_partial_floats((int)P2, X, c.c_hid));
        pf = std::max(pf, pw_partial_floats((int)P2, c.c_hid, c.c_feat));
        st = grow(&net->partial, &net->partial_cap, pf * 4);
        if (st != ME_OK) return st;
    }
    net->n = n;
    net->Hp = Hp;
    net->Wp = Wp;
    net->H1 = H1;
    net->W1 = W1;
    net->Hf = Hf;
    net->Wf = Wf;
    return ME_OK;
}

PwArgs pw_args(me_prnet net, const Layer& l, PwTensor x, PwTensor x2, int HW, int P, void* out)
{
    PwArgs a{};
    a.x = x;
    a.x2 = x2;
    a.HW = HW;
    a.P = P;
    a.w = net->packs + l.fwd;
    a.M = l.co;
    a.KS = l.KS;
    a.bias = net->params + l.off_b;
    a.relu6 = l.relu6;
    a.add = none();
    a.mask = nullptr;
    a.out = out;
    return a;
}

// Forward through every layer.  Inference (r_out == nullptr): the head adds z_pred
// and writes z_out ([n][c_feat][Hf][Wf], dtype of z_pred).  Training: the head
// writes the residual as float32 into net->r.
hipError_t run_forward(me_prnet net, const me_frame* cur, int64_t frame_stride, const void* zp, int z_bf16, void* z_out,
                       bool train, hipStream_t st)
{
    const me_prnet_cfg& c = net->cfg;
    const int n = net->n, HW1 = net->H1 * net->W1, HW2 = net->Hf * net->Wf;
    const int P1 = n * HW1, P2 = n * HW2;
    const std::vector<Layer>& L = net->L;
    hipError_t e = hipSuccess;
    if (!train && enc_fused_ok(c.c_enc)) {
        // inference: the whole encoder in one pass (its intermediates are not kept)
        EncArgs ea{};
        ea.mosaic = cur->data;
        ea.pitch = cur->pitch;
        ea.img_stride = frame_stride;
        ea.n = n;
        ea.Hp = net->Hp;
        ea.Wp = net->Wp;
        ea.H1 = net->H1;
        ea.W1 = net->W1;
        ea.Hf = net->Hf;
        ea.Wf = net->Wf;
        ea.ce = c.c_enc;
        ea.w0 = net->params + L[0].off_w;
        ea.b0 = net->params + L[0].off_b;
        ea.w1 = net->params + L[1].off_w;
        ea.b1 = net->params + L[1].off_b;
        ea.w2 = net->params + L[2].off_w;
        ea.b2 = net->params + L[2].off_b;
        ea.w3p = net->packs + L[3].fwd;
        ea.b3 = net->params + L[3].off_b;
        ea.out = net->e4;
        e = launch_encoder(ea, st);
    } else {
        e = launch_planes(cur->data, cur->pitch, frame_stride, n, net->Hp, net->Wp, net->a0, st);
        if (e == hipSuccess)
            e = launch_dw_fwd(net->a0, net->params + L[0].off_w, net->params + L[0].off_b, net->e1, n, net->Hp,
                              net->Wp, 4, 2, 1, st);
        if (e == hipSuccess) e = launch_pw(pw_args(net, L[1], nhwc(net->e1, 4), none(), HW1, P1, net->e2), st);
        if (e == hipSuccess)
            e = launch_dw_fwd(net->e2, net->params + L[2].off_w, net->params + L[2].off_b, net->e3, n, net->H1,
                              net->W1, c.c_enc, 2, 1, st);
        if (e == hipSuccess) e = launch_pw(pw_args(net, L[3], nhwc(net->e3, c.c_enc), none(), HW2, P2, net->e4), st);
    }
    const PwTensor z{zp, c.c_feat, 1, z_bf16 ? 0 : 1};
    if (train || (HW2 & 3)) {
        // channels-last copy of z_pred (kept for the projection's weight gradient)
        if (e == hipSuccess) e = launch_to_nhwc(zp, z_bf16 ? 0 : 1, n, c.c_feat, HW2, net->zl, st);
        if (e == hipSuccess)
            e = launch_pw(pw_args(net, L[4], nhwc(net->zl, c.c_feat), nhwc(net->e4, c.c_enc), HW2, P2, net->h[0]), st);
    } else if (e == hipSuccess) {
        // inference: the projection stages z_pred straight from its channels-first layout
        e = launch_pw(pw_args(net, L[4], z, nhwc(net->e4, c.c_enc), HW2, P2, net->h[0]), st);
    }
    const int X = c.c_hid * c.expand;
    const bool fused = !train && ir_fused_ok(c.c_hid, X);   // training keeps u and v for the backward pass
    for (int k = 0; k < c.n_blocks && e == hipSuccess; ++k) {
        const Layer &le = L[5 + 3 * k], &ld = L[6 + 3 * k], &lc = L[7 + 3 * k];
        if (fused) {
            IrArgs ia{};
            ia.h_in = net->h[k];
            ia.h_out = net->h[k + 1];
            ia.we = net->packs + le.fwd;
            ia.be = net->params + le.off_b;
            ia.wd = net->params + ld.off_w;
            ia.bd = net->params + ld.off_b;
            ia.wc = net->packs + lc.fwd;
            ia.bc = net->params + lc.off_b;
            ia.n = n;
            ia.Hf = net->Hf;
            ia.Wf = net->Wf;
            ia.ch = c.c_hid;
            ia.x = X;
            e = launch_ir_block(ia, st);
            continue;
        }
        e = launch_pw(pw_args(net, le, nhwc(net->h[k], c.c_hid), none(), HW2, P2, net->u[k]), st);
        if (e == hipSuccess)
            e = launch_dw_fwd(net->u[k], net->params + ld.off_w, net->params + ld.off_b, net->v_[k], n, net->Hf,
                              net->Wf, X, 1, 1, st);
        if (e == hipSuccess) {
            PwArgs a = pw_args(net, lc, nhwc(net->v_[k], X), none(), HW2, P2, net->h[k + 1]);
            a.add = nhwc(net->h[k], c.c_hid);
            e = launch_pw(a, st);
        }
    }
    if (e != hipSuccess) return e;
    PwArgs a = pw_args(net, L.back(), nhwc(net->h[c.n_blocks], c.c_hid), none(), HW2, P2, train ? (void*)net->r : z_out);
    a.out_chw = 1;
    if (train) {
        a.out_f32 = 1;
    } else {
        a.out_f32 = z_bf16 ? 0 : 1;
        a.add = z;
    }
    return launch_pw(a, st);
}

hipError_t pw_grad(me_prnet net, const Layer& l, PwTensor x, PwTensor x2, PwTensor dy, int HW, int P, hipStream_t st)
{
    PwGradArgs g{};
    g.x = x;
    g.x2 = x2;
    g.dy = dy;
    g.HW = HW;
    g.P = P;
    g.cin = l.ci;
    g.cout = l.co;
    g.chunk = wgrad_chunk(P, kWgTarget);
    g.partial = static_cast<float*>(net->partial);
    return launch_pw_wgrad(g, net->grads + l.off_w, net->grads + l.off_b, st);
}

hipError_t pw_dgrad(me_prnet net, const Layer& l, PwTensor dy, int HW, int P, const uint16_t* add, const uint16_t* mask,
                    uint16_t* dx, hipStream_t st)
{
    PwArgs a{};
    a.x = dy;
    a.x2 = none();
    a.HW = HW;
    a.P = P;
    a.w = net->packs + l.bwd;
    a.M = l.crb;
    a.KS = l.KSb;
    a.bias = nullptr;
    a.relu6 = 0;
    a.add = add ? nhwc(add, l.crb) : none();
    a.mask = mask;
    a.out = dx;
    return launch_pw(a, st);
}

// The projection's weight gradient reads z_pred as the forward pass left it
// (channels-last bfloat16 in net->zl).
hipError_t run_backward(me_prnet net, hipStream_t st)
{
    const me_prnet_cfg& c = net->cfg;
    const std::vector<Layer>& L = net->L;
    const int n = net->n, HW1 = net->H1 * net->W1, HW2 = net->Hf * net->Wf;
    const int P1 = n * HW1, P2 = n * HW2, X = c.c_hid * c.expand, nb = c.n_blocks;
    float* part = static_cast<float*>(net->partial);
    const PwTensor dr{net->dr, c.c_feat, 1, 0};
    // head
    const Layer& lh = L.back();
    hipError_t e = pw_grad(net, lh, nhwc(net->h[nb], c.c_hid), none(), dr, HW2, P2, st);
    int cur = 0;
    if (e == hipSuccess) e = pw_dgrad(net, lh, dr, HW2, P2, nullptr, nb == 0 ? net->h[0] : nullptr, net->dh[cur], st);
    for (int k = nb - 1; k >= 0 && e == hipSuccess; --k) {
        const Layer &le = L[5 + 3 * k], &ld = L[6 + 3 * k], &lc = L[7 + 3 * k];
        const PwTensor dh = nhwc(net->dh[cur], c.c_hid);
        e = pw_grad(net, lc, nhwc(net->v_[k], X), none(), dh, HW2, P2, st);
        if (e == hipSuccess) e = pw_dgrad(net, lc, dh, HW2, P2, nullptr, net->v_[k], net->gA, st);   // dv
        if (e == hipSuccess)
            e = dw_wgrad(net->u[k], net->gA, part, net->grads + ld.off_w, net->grads + ld.off_b, n, net->Hf, net->Wf, X,
                         1, st);
        if (e == hipSuccess)
            e = launch_dw_dgrad(net->gA, net->params + ld.off_w, net->u[k], net->gB, n, net->Hf, net->Wf, X, 1, st);  // du
        if (e == hipSuccess) e = pw_grad(net, le, nhwc(net->h[k], c.c_hid), none(), nhwc(net->gB, X), HW2, P2, st);
        if (e == hipSuccess)
            e = pw_dgrad(net, le, nhwc(net->gB, X), HW2, P2, net->dh[cur], k == 0 ? net->h[0] : nullptr,
                         net->dh[cur ^ 1], st);
        cur ^= 1;
    }
    if (e != hipSuccess) return e;
    // projection: input [z_pred, e4]; its gradient reaches e4 only
    const PwTensor dp = nhwc(net->dh[cur], c.c_hid);
    e = pw_grad(net, L[4], nhwc(net->zl, c.c_feat), nhwc(net->e4, c.c_enc), dp, HW2, P2, st);
    if (e == hipSuccess) e = pw_dgrad(net, L[4], dp, HW2, P2, nullptr, net->e4, net->gA, st);              // de4
    if (e == hipSuccess) e = pw_grad(net, L[3], nhwc(net->e3, c.c_enc), none(), nhwc(net->gA, c.c_enc), HW2, P2, st);
    if (e == hipSuccess) e = pw_dgrad(net, L[3], nhwc(net->gA, c.c_enc), HW2, P2, nullptr, net->e3, net->gB, st);  // de3
    if (e == hipSuccess)
        e = dw_wgrad(net->e2, net->gB, part, net->grads + L[2].off_w, net->grads + L[2].off_b, n, net->H1, net->W1,
                     c.c_enc, 2, st);
    if (e == hipSuccess)
        e = launch_dw_dgrad(net->gB, net->params + L[2].off_w, net->e2, net->gA, n, net->H1, net->W1, c.c_enc, 2, st);
    if (e == hipSuccess) e = pw_grad(net, L[1], nhwc(net->e1, 4), none(), nhwc(net->gA, c.c_enc), HW1, P1, st);
    if (e == hipSuccess) e = pw_dgrad(net, L[1], nhwc(net->gA, c.c_enc), HW1, P1, nullptr, net->e1, net->gB, st);  // de1
    if (e == hipSuccess)
        e = dw_wgrad(net->a0, net->gB, part, net->grads + L[0].off_w, net->grads + L[0].off_b, n, net->Hp, net->Wp, 4,
                     2, st);
    return e;
}

me_status check_input(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride, const char* who)
{
    if (!net) return fail(ME_E_INVAL, "%s: null network", who);
    if (!net->loaded) return fail(ME_E_STATE, "%s: no parameters set", who);
    me_status s = check_frame(cur, who);
    if (s != ME_OK) return s;
    if (n < 1 || n > 4096) return fail(ME_E_INVAL, "%s: n must be 1..4096", who);
    if (n > 1 && frame_stride < (int64_t)cur->height * cur->pitch)
        return fail(ME_E_INVAL, "%s: frame_stride must be >= height * pitch", who);
    const int64_t Hp = cur->height / 2, Wp = cur->width / 2;
    const int64_t big = n * Hp * Wp * (int64_t)std::max(net->cfg.c_hid * net->cfg.expand, net->cfg.c_feat);
    if (big >= ((int64_t)1 << 31)) return fail(ME_E_UNSUPPORTED, "%s: batch too large for 32-bit element indices", who);
    return ME_OK;
}

}  // namespace

extern "C" {

int64_t me_prnet_num_params(const me_prnet_cfg* cfg)
{
    if (check_cfg(cfg) != ME_OK) return -1;
    int64_t n = 0;
    for (const Layer& l : make_layers(*cfg)) n += (int64_t)l.co * (l.kind == kDw ? 9 : l.ci) + l.co;
    return n;
}

me_status me_prnet_create(me_ctx ctx, const me_prnet_cfg* cfg, me_prnet* out)
{
    if (!ctx || !out) return fail(ME_E_INVAL, "me_prnet_create: null argument");
    me_status s = check_cfg(cfg);
    if (s != ME_OK) return s;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_create: hipSetDevice");
    me_prnet net = new me_prnet_s();
    net->device = ctx->device;
    net->cfg = *cfg;
    net->L = make_layers(*cfg);
    net->np = me_prnet_num_params(cfg);
    const size_t pb = (size_t)net->np * 4;
    if (hipMalloc(&net->params, pb) != hipSuccess || hipMalloc(&net->grads, pb) != hipSuccess ||
        hipMalloc(&net->m, pb) != hipSuccess || hipMalloc(&net->v, pb) != hipSuccess ||
        hipMalloc(&net->packs, packs_elems(net->L) * 2) != hipSuccess) {
        delete net;
        return fail(ME_E_NOMEM, "me_prnet_create: out of device memory");
    }
    *out = net;
    return ME_OK;
}

me_status me_prnet_destroy(me_prnet net)
{
    delete net;
    return ME_OK;
}

me_status me_prnet_set_params(me_prnet net, const float* params, int64_t count)
{
    if (!net || !params) return fail(ME_E_INVAL, "me_prnet_set_params: null argument");
    if (count != net->np) return fail(ME_E_INVAL, "me_prnet_set_params: expected %lld parameters", (long long)net->np);
    hipError_t e = hipSetDevice(net->device);
    if (e == hipSuccess) e = hipMemcpy(net->params, params, net->np * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(net->m, 0, net->np * 4);
    if (e == hipSuccess) e = hipMemset(net->v, 0, net->np * 4);
    if (e == hipSuccess) e = hipMemset(net->grads, 0, net->np * 4);
    if (e == hipSuccess) e = repack(net, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "me_prnet_set_params");
    net->step = 0;
    net->loaded = true;
    return ME_OK;
}

me_status me_prnet_get_params(me_prnet net, float* params, int64_t count)
{
    if (!net || !params) return fail(ME_E_INVAL, "me_prnet_get_params: null argument");
    if (count != net->np) return fail(ME_E_INVAL, "me_prnet_get_params: expected %lld parameters", (long long)net->np);
    if (!net->loaded) return fail(ME_E_STATE, "me_prnet_get_params: no parameters set");
    hipError_t e = hipSetDevice(net->device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(params, net->params, net->np * 4, hipMemcpyDeviceToHost);
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_get_params");
}

me_status me_prnet_forward(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride, const void* z_pred,
                           void* z_out, int32_t dtype, void* stream)
{
    me_status s = check_input(net, cur, n, frame_stride, "me_prnet_forward");
    if (s != ME_OK) return s;
    if (!z_pred || !z_out) return fail(ME_E_INVAL, "me_prnet_forward: null feature pointer");
    if (dtype != ME_F32 && dtype != ME_BF16) return fail(ME_E_INVAL, "me_prnet_forward: bad dtype");
    hipError_t e = hipSetDevice(net->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_forward: hipSetDevice");
    s = layout(net, n, cur->height / 2, cur->width / 2, false);
    if (s != ME_OK) return s;
    e = run_forward(net, cur, frame_stride, z_pred, dtype == ME_BF16, z_out, false, as_stream(stream));
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_forward");
}

me_status me_prnet_forward_acts(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride,
                                const void* z_pred, void* z_out, int32_t dtype, uint16_t* enc, uint16_t* hid,
                                void* stream)
{
    me_status s = me_prnet_forward(net, cur, n, frame_stride, z_pred, z_out, dtype, stream);
    if (s != ME_OK) return s;
    hipStream_t st = as_stream(stream);
    const size_t P2 = (size_t)net->n * net->Hf * net->Wf;
    hipError_t e = hipSuccess;
    if (enc) e = hipMemcpyAsync(enc, net->e4, P2 * net->cfg.c_enc * 2, hipMemcpyDeviceToDevice, st);
    for (int k = 0; hid && k <= net->cfg.n_blocks && e == hipSuccess; ++k)
        e = hipMemcpyAsync(hid + (size_t)k * P2 * net->cfg.c_hid, net->h[k], P2 * net->cfg.c_hid * 2,
                           hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_forward_acts: copies");
}

me_status me_prnet_train_step(me_prnet net, const me_frame* cur, int32_t n, int64_t frame_stride, const float* z_pred,
                              const float* z_target, float tau, float lr, int32_t update, float* grads, float* loss,
                              void* stream)
{
    me_status s = check_input(net, cur, n, frame_stride, "me_prnet_train_step");
    if (s != ME_OK) return s;
    if (!z_pred || !z_target || !loss) return fail(ME_E_INVAL, "me_prnet_train_step: null pointer");
    if (!(tau == tau)) return fail(ME_E_INVAL, "me_prnet_train_step: tau is NaN");
    if (update && !(lr >= 0.0f && lr < 1.0f)) return fail(ME_E_INVAL, "me_prnet_train_step: bad learning rate");
    hipError_t e = hipSetDevice(net->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_train_step: hipSetDevice");
    s = layout(net, n, cur->height / 2, cur->width / 2, true);
    if (s != ME_OK) return s;
    hipStream_t st = as_stream(stream);
    const int HW2 = net->Hf * net->Wf;
    e = run_forward(net, cur, frame_stride, z_pred, 0, nullptr, true, st);
    if (e == hipSuccess)
        e = launch_prloss(net->r, z_pred, z_target, n, net->cfg.c_feat, HW2, tau, net->nbad, net->maxbits, net->flags,
                          net->dr, net->lpart, loss, st);
    if (e == hipSuccess) e = run_backward(net, st);
    if (e == hipSuccess && grads) e = hipMemcpyAsync(grads, net->grads, net->np * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && update) {
        net->step += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 / (1.0 - pow(b1, (double)net->step)));
        const float c2 = (float)(1.0 / (1.0 - pow(b2, (double)net->step)));
        e = launch_adamw(net->params, net->grads, net->m, net->v, (int)net->np, lr, (float)b1, (float)b2, 1e-8f, 0.01f,
                         c1, c2, st);
        if (e == hipSuccess) e = repack(net, st);
    }
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_train_step");
}

// ----------------------------------------------------------- layer calls --

static me_status tensor_ok(const me_tensor* t, const char* who, bool want_bf16_nhwc)
{
    if (!t || !t->data) return fail(ME_E_INVAL, "%s: null tensor", who);
    if (t->channels < 4 || t->channels % 4 || t->channels > 1024)
        return fail(ME_E_INVAL, "%s: channels must be a multiple of 4 in 4..1024", who);
    if (t->layout != ME_NHWC && t->layout != ME_NCHW) return fail(ME_E_INVAL, "%s: bad layout", who);
    if (t->dtype != ME_F32 && t->dtype != ME_BF16) return fail(ME_E_INVAL, "%s: bad dtype", who);
    if (want_bf16_nhwc && (t->layout != ME_NHWC || t->dtype != ME_BF16))
        return fail(ME_E_INVAL, "%s: tensor must be bfloat16 channels-last", who);
    return ME_OK;
}

static PwTensor view(const me_tensor* t)
{
    return t && t->data ? PwTensor{t->data, t->channels, t->layout == ME_NCHW, t->dtype == ME_F32} : none();
}

static me_status ctx_scratch(me_ctx ctx, size_t bytes, void** p)
{
    me_status s = grow(&ctx->prn_scratch, &ctx->prn_scratch_cap, bytes);
    *p = ctx->prn_scratch;
    return s;
}

me_status me_prnet_dw_forward(me_ctx ctx, const uint16_t* x, const float* w, const float* b, int32_t n, int32_t H,
                              int32_t W, int32_t C, int32_t stride, int32_t relu6, uint16_t* y, void* stream)
{
    if (!ctx || !x || !w || !b || !y) return fail(ME_E_INVAL, "me_prnet_dw_forward: null argument");
    if (n < 1 || H < 1 || W < 1 || C < 4 || C % 4 || C > 1024 || (stride != 1 && stride != 2))
        return fail(ME_E_INVAL, "me_prnet_dw_forward: bad shape");
    if ((int64_t)n * H * W * C >= ((int64_t)1 << 31)) return fail(ME_E_UNSUPPORTED, "me_prnet_dw_forward: too large");
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = launch_dw_fwd(x, w, b, y, n, H, W, C, stride, relu6 ? 1 : 0, as_stream(stream));
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_dw_forward");
}

me_status me_prnet_dw_backward(me_ctx ctx, const uint16_t* x, const float* w, const uint16_t* dy, const uint16_t* mask,
                               int32_t n, int32_t H, int32_t W, int32_t C, int32_t stride, uint16_t* dx, float* grads,
                               void* stream)
{
    if (!ctx || !dy || (dx && !w) || (grads && !x)) return fail(ME_E_INVAL, "me_prnet_dw_backward: null argument");
    if (n < 1 || H < 1 || W < 1 || C < 4 || C % 4 || C > 1024 || (stride != 1 && stride != 2))
        return fail(ME_E_INVAL, "me_prnet_dw_backward: bad shape");
    if ((int64_t)n * H * W * C >= ((int64_t)1 << 31)) return fail(ME_E_UNSUPPORTED, "me_prnet_dw_backward: too large");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_dw_backward: hipSetDevice");
    hipStream_t st = as_stream(stream);
    if (grads) {
        void* part = nullptr;
        me_status s = ctx_scratch(ctx, std::max<size_t>(dw_partial_floats(n, H, W, stride, C), 1) * 4, &part);
        if (s != ME_OK) return s;
        e = dw_wgrad(x, dy, static_cast<float*>(part), grads, grads + (size_t)C * 9, n, H, W, C, stride, st);
    }
    if (e == hipSuccess && dx) e = launch_dw_dgrad(dy, w, mask, dx, n, H, W, C, stride, st);
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_dw_backward");
}

me_status me_prnet_pw_forward(me_ctx ctx, const me_tensor* x, const me_tensor* x2, int32_t n, int32_t HW,
                              const float* w, const float* b, int32_t cout, int32_t relu6, const me_tensor* add,
                              const uint16_t* mask, const me_tensor* out, void* stream)
{
    const char* who = "me_prnet_pw_forward";
    if (!ctx || !w) return fail(ME_E_INVAL, "%s: null argument", who);
    me_status s = tensor_ok(x, who, false);
    if (s == ME_OK && x2 && x2->data) s = tensor_ok(x2, who, false);
    if (s == ME_OK && add && add->data) s = tensor_ok(add, who, false);
    if (s == ME_OK) s = tensor_ok(out, who, false);
    if (s != ME_OK) return s;
    const int cin = x->channels + (x2 && x2->data ? x2->channels : 0);
    if (n < 1 || HW < 1 || cout < 4 || cout % 4 || cout > 1024 || cin > 1024 || out->channels != cout ||
        (add && add->data && add->channels != cout))
        return fail(ME_E_INVAL, "%s: bad shape", who);
    if ((int64_t)n * HW * std::max(cin, cout) >= ((int64_t)1 << 31)) return fail(ME_E_UNSUPPORTED, "%s: too large", who);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_pw_forward: hipSetDevice");
    const int MT = div_up(cout, 16), KS = div_up(cin, 16);
    void* pk = nullptr;
    s = ctx_scratch(ctx, (size_t)MT * KS * 256 * 2, &pk);
    if (s != ME_OK) return s;
    hipStream_t st = as_stream(stream);
    e = launch_pw_pack(w, cin, 0, 0, cout, cin, MT, KS, static_cast<uint16_t*>(pk), st);
    PwArgs a{};
    a.x = view(x);
    a.x2 = view(x2);
    a.HW = HW;
    a.P = n * HW;
    a.w = static_cast<uint16_t*>(pk);
    a.M = cout;
    a.KS = KS;
    a.bias = b;
    a.relu6 = relu6 ? 1 : 0;
    a.add = view(add);
    a.mask = mask;
    a.out = const_cast<void*>(out->data);
    a.out_chw = out->layout == ME_NCHW;
    a.out_f32 = out->dtype == ME_F32;
    if (e == hipSuccess) e = launch_pw(a, st);
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_pw_forward");
}

me_status me_prnet_pw_backward(me_ctx ctx, const me_tensor* x, const me_tensor* x2, const me_tensor* dy, int32_t n,
                               int32_t HW, const float* w, int32_t cout, int32_t dx_c0, int32_t dx_count,
                               const uint16_t* add, const uint16_t* mask, uint16_t* dx, float* grads, void* stream)
{
    const char* who = "me_prnet_pw_backward";
    if (!ctx) return fail(ME_E_INVAL, "%s: null context", who);
    me_status s = tensor_ok(x, who, false);
    if (s == ME_OK && x2 && x2->data) s = tensor_ok(x2, who, false);
    if (s == ME_OK) s = tensor_ok(dy, who, false);
    if (s != ME_OK) return s;
    const int cin = x->channels + (x2 && x2->data ? x2->channels : 0);
    if (n < 1 || HW < 1 || cout < 4 || cout % 4 || cout > 1024 || cin > 1024 || dy->channels != cout)
        return fail(ME_E_INVAL, "%s: bad shape", who);
    if (dx && (!w || dx_c0 < 0 || dx_count < 4 || dx_count % 4 || dx_c0 % 4 || dx_c0 + dx_count > cin))
        return fail(ME_E_INVAL, "%s: bad input-gradient range", who);
    if ((int64_t)n * HW * std::max(cin, cout) >= ((int64_t)1 << 31)) return fail(ME_E_UNSUPPORTED, "%s: too large", who);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_pw_backward: hipSetDevice");
    hipStream_t st = as_stream(stream);
    const int P = n * HW;
    const size_t part_b = pw_partial_floats(P, cin, cout) * 4;
    const int MT = div_up(dx_count, 16), KS = div_up(cout, 16);
    const size_t pack_b = dx ? ((size_t)MT * KS * 256 * 2 + 255) & ~(size_t)255 : 0;
    void* scr = nullptr;
    s = ctx_scratch(ctx, pack_b + (grads ? part_b : 0), &scr);
    if (s != ME_OK) return s;
    if (grads) {
        PwGradArgs g{};
        g.x = view(x);
        g.x2 = view(x2);
        g.dy = view(dy);
        g.HW = HW;
        g.P = P;
        g.cin = cin;
        g.cout = cout;
        g.chunk = wgrad_chunk(P, kWgTarget);
        g.partial = reinterpret_cast<float*>(static_cast<uint8_t*>(scr) + pack_b);
        e = launch_pw_wgrad(g, grads, grads + (size_t)cout * cin, st);
    }
    if (e == hipSuccess && dx) {
        uint16_t* pk = static_cast<uint16_t*>(scr);
        e = launch_pw_pack(w, cin, dx_c0, 1, dx_count, cout, MT, KS, pk, st);
        PwArgs a{};
        a.x = view(dy);
        a.x2 = none();
        a.HW = HW;
        a.P = P;
        a.w = pk;
        a.M = dx_count;
        a.KS = KS;
        a.add = add ? nhwc(add, dx_count) : none();
        a.mask = mask;
        a.out = dx;
        if (e == hipSuccess) e = launch_pw(a, st);
    }
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_pw_backward");
}

me_status me_prnet_loss(me_ctx ctx, const float* r, const float* z_pred, const float* z_target, int32_t n, int32_t C,
                        int32_t Hf, int32_t Wf, float tau, uint16_t* dr, float* loss, void* stream)
{
    if (!ctx || !r || !z_pred || !z_target || !dr || !loss) return fail(ME_E_INVAL, "me_prnet_loss: null argument");
    if (n < 1 || C < 1 || Hf < 1 || Wf < 1 || !(tau == tau)) return fail(ME_E_INVAL, "me_prnet_loss: bad shape");
    if ((int64_t)n * C * Hf * Wf >= ((int64_t)1 << 31)) return fail(ME_E_UNSUPPORTED, "me_prnet_loss: too large");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "me_prnet_loss: hipSetDevice");
    const int P = n * Hf * Wf;
    void* scr = nullptr;
    const size_t pb = ((size_t)prloss_blocks(P) * 4 + 255) & ~(size_t)255;
    me_status s = ctx_scratch(ctx, 256 + pb + (size_t)P, &scr);
    if (s != ME_OK) return s;
    uint8_t* q = static_cast<uint8_t*>(scr);
    e = launch_prloss(r, z_pred, z_target, n, C, Hf * Wf, tau, reinterpret_cast<int32_t*>(q),
                      reinterpret_cast<uint32_t*>(q + 4), q + 256 + pb, dr, reinterpret_cast<float*>(q + 256), loss,
                      as_stream(stream));
    return e == hipSuccess ? ME_OK : hip_fail(e, "me_prnet_loss");
}

}  // extern "C"
