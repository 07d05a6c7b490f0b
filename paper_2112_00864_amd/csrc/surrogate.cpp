// Touching-pair surrogate: a small network that corrects a low-order quadrature of the Galerkin
// integral of 1/|x - y| over two touching cubes to the accuracy of the high-order one.
//
// A touching pair of axis-aligned cubes is brought by a rigid motion and a scaling to canonical
// form: A = [0,1]^3 (the smaller cube) and B, a cube of side rho in [1, 2], on the +x side of A
// (face contact), on the +x,+y edge (edge contact) or at the +x,+y,+z vertex (vertex contact), with
// its lower corner on the free axes at off[] in (-rho, 1). The Galerkin entry of the original pair
// is J * a^5 / (4 pi) with a the smaller side and J the canonical integral.
//
// Prediction: J = J_lo * (1 + S * y0), where J_lo is the quadrature with few points, S the RMS of
// the relative residual (J_hi - J_lo) / J_lo over the training set, and y = (y0, y1) the network
// output; y1 estimates log of |y0 - true normalised residual|. A pair is accepted when
// kappa * S * exp(y1) <= tol, else it falls back to the high-order quadrature J_hi. kappa is
// calibrated on one half of the held-out pairs after training (1.5 times the largest ratio of the
// true relative error to the estimate S exp(y1)), so that the estimate bounds the error on pairs
// like those; the other half, which the calibration never saw, reports the accepted error.
// Network: features (6) -> width -> width -> 2, SiLU, FP32; the correction is added in FP64.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "internal.hpp"
#include "mlp.hpp"
#include "quadrature.hpp"

namespace bcv {

namespace {

constexpr float kAdamB1 = 0.9f, kAdamB2 = 0.999f, kAdamEps = 1e-8f;
constexpr float kErrWeight = 0.1f, kErrEps = 1e-5f;
constexpr double kCalibrationMargin = 1.5;
constexpr uint32_t kFileMagic = 0x424D4C50u;  // "BMLP"

struct Layout {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

Layout layout(int d_in, int width)
{
    Layout l;
    l.w1 = 0;
    l.b1 = l.w1 + (int64_t)d_in * width;
    l.w2 = l.b1 + width;
    l.b2 = l.w2 + (int64_t)width * width;
    l.w3 = l.b2 + width;
    l.b3 = l.w3 + (int64_t)width * kMlpOut;
    l.total = l.b3 + kMlpOut;
    return l;
}

template <class T>
struct DevBuf {
    T *p = nullptr;
    explicit DevBuf(size_t n)
    {
        if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed");
    }
    ~DevBuf() { (void)hipFree(p); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
};

// Activations and gradients of one batch.
struct Work {
    int B, width;
    DevBuf<float> Z1, H1, Z2, H2, Y, dY, dH, dZ, terms, split;
    Work(int B_, int width_, int d_in)
        : B(B_), width(width_), Z1((size_t)B_ * width_), H1((size_t)B_ * width_), Z2((size_t)B_ * width_),
          H2((size_t)B_ * width_), Y((size_t)B_ * kMlpOut), dY((size_t)B_ * kMlpOut), dH((size_t)B_ * width_),
          dZ((size_t)B_ * width_), terms((size_t)B_ * kMlpOut),
          split((size_t)std::max<int64_t>(split_workspace(std::max(width_, d_in), width_, B_),
                                          split_workspace(1, std::max(width_, kMlpOut), B_)))
    {
    }
};

void forward(const bcv_mlp_s &net, const float *X, int B, Work &w, hipStream_t st)
{
    const Layout l = layout(net.d_in, net.width);
    const float *P = net.d_params;
    const int W = net.width;
    gemm(false, false, B, W, net.d_in, X, net.d_in, P + l.w1, W, P + l.b1, false, w.Z1.p, W, w.H1.p, st);
    gemm(false, false, B, W, W, w.H1.p, W, P + l.w2, W, P + l.b2, false, w.Z2.p, W, w.H2.p, st);
    gemm(false, false, B, kMlpOut, W, w.H2.p, W, P + l.w3, kMlpOut, P + l.b3, false, w.Y.p, kMlpOut, nullptr, st);
}

// Gradient of the batch loss with respect to every parameter, into G (layout of the parameters).
void backward(const bcv_mlp_s &net, const float *X, int B, Work &w, float *G, hipStream_t st)
{
    const Layout l = layout(net.d_in, net.width);
    const float *P = net.d_params;
    const int W = net.width;
    // layer 3: Y = H2 W3 + b3
    gemm_tn_split(W, kMlpOut, B, w.H2.p, W, w.dY.p, kMlpOut, G + l.w3, w.split.p, st);
    column_sum(B, kMlpOut, w.dY.p, G + l.b3, w.split.p, st);
    gemm(false, true, B, W, kMlpOut, w.dY.p, kMlpOut, P + l.w3, kMlpOut, nullptr, false, w.dH.p, W, nullptr, st);
    silu_backward((int64_t)B * W, w.Z2.p, w.dH.p, w.dZ.p, st);
    // layer 2: Z2 = H1 W2 + b2
    gemm_tn_split(W, W, B, w.H1.p, W, w.dZ.p, W, G + l.w2, w.split.p, st);
    column_sum(B, W, w.dZ.p, G + l.b2, w.split.p, st);
    gemm(false, true, B, W, W, w.dZ.p, W, P + l.w2, W, nullptr, false, w.dH.p, W, nullptr, st);
    silu_backward((int64_t)B * W, w.Z1.p, w.dH.p, w.dZ.p, st);
    // layer 1: Z1 = X W1 + b1
    gemm_tn_split(net.d_in, W, B, X, net.d_in, w.dZ.p, W, G + l.w1, w.split.p, st);
    column_sum(B, W, w.dZ.p, G + l.b1, w.split.p, st);
}

// Canonical geometry: A = [0,1]^3, B of side rho touching A's +x face / +x+y edge / +x+y+z vertex.
void pair_geometry(const bcv_touch_pair &t, double *g)
{
    const double rho = t.rho;
    double blo[3] = {1.0, 1.0, 1.0};
    if (t.contact == BCV_CONTACT_FACE) blo[1] = t.off[0], blo[2] = t.off[1];
    if (t.contact == BCV_CONTACT_EDGE) blo[2] = t.off[0];
    for (int i = 0; i < 3; ++i) {
        g[i] = 0.0;
        g[3 + i] = 1.0;
        g[6 + i] = blo[i];
        g[9 + i] = blo[i] + rho;
    }
}

void pair_features(const bcv_touch_pair &t, float *x)
{
    x[0] = t.contact == BCV_CONTACT_FACE ? 1.0f : 0.0f;
    x[1] = t.contact == BCV_CONTACT_EDGE ? 1.0f : 0.0f;
    x[2] = t.contact == BCV_CONTACT_VERTEX ? 1.0f : 0.0f;
    x[3] = (float)(2.0 * std::log2(t.rho) - 1.0);
    const int n_free = t.contact == BCV_CONTACT_FACE ? 2 : (t.contact == BCV_CONTACT_EDGE ? 1 : 0);
    for (int k = 0; k < 2; ++k)  // position of B's lower corner in (-rho, 1), mapped to (-1, 1)
        x[4 + k] = k < n_free ? (float)(2.0 * (t.off[k] + t.rho) / (1.0 + t.rho) - 1.0) : 0.0f;
}

void check_pair(const bcv_touch_pair &t)
{
    BCV_REQUIRE(t.contact >= BCV_CONTACT_FACE && t.contact <= BCV_CONTACT_VERTEX, BCV_EINVAL, "unknown contact type");
    BCV_REQUIRE(t.rho >= 1.0 && t.rho <= 2.0, BCV_EINVAL, "size ratio must lie in [1, 2]");
    const int n_free = t.contact == BCV_CONTACT_FACE ? 2 : (t.contact == BCV_CONTACT_EDGE ? 1 : 0);
    for (int k = 0; k < n_free; ++k)
        BCV_REQUIRE(t.off[k] > -t.rho && t.off[k] < 1.0, BCV_EINVAL, "offset outside (-rho, 1): not a touching pair");
}

// J for n canonical pairs at Gauss order n_gauss (device result array).
void quadrature(const std::vector<bcv_touch_pair> &pairs, int n_gauss, double *out_dev, hipStream_t st)
{
    std::vector<double> geom(12 * pairs.size());
    for (size_t i = 0; i < pairs.size(); ++i) pair_geometry(pairs[i], &geom[12 * i]);
    DevBuf<double> d_geom(geom.size());
    BCV_HIP(hipMemcpyAsync(d_geom.p, geom.data(), geom.size() * sizeof(double), hipMemcpyHostToDevice, st));
    box_pair_integrals_device((int64_t)pairs.size(), d_geom.p, n_gauss, out_dev, st);
    BCV_HIP(hipStreamSynchronize(st));
}

std::vector<double> download(const double *d, size_t n, hipStream_t st)
{
    std::vector<double> h(n);
    BCV_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, st));
    BCV_HIP(hipStreamSynchronize(st));
    return h;
}

// Random canonical pairs: contact face/edge/vertex 1/2, 3/10, 1/5; rho exactly 1 or 2 with
// probability 1/5 each, else uniform; each free offset aligned with A's lower or upper face with
// probability 1/4 and 1/10 (the positions a 2:1 octree produces), else uniform in (-rho, 1).
std::vector<bcv_touch_pair> sample_pairs(int64_t n, uint64_t seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::vector<bcv_touch_pair> v(n);
    for (auto &t : v) {
        const double c = U(rng);
        t.contact = c < 0.5 ? BCV_CONTACT_FACE : (c < 0.8 ? BCV_CONTACT_EDGE : BCV_CONTACT_VERTEX);
        const double r = U(rng);
        t.rho = r < 0.2 ? 1.0 : (r < 0.4 ? 2.0 : 1.0 + U(rng));
        for (int k = 0; k < 2; ++k) {
            const double a = U(rng);
            if (a < 0.25) t.off[k] = 0.0;
            else if (a < 0.35) t.off[k] = 1.0 - t.rho;
            else t.off[k] = -t.rho + (0.01 + 0.98 * U(rng)) * (1.0 + t.rho);
        }
        if (t.contact != BCV_CONTACT_FACE) t.off[1] = 0.0;
        if (t.contact == BCV_CONTACT_VERTEX) t.off[0] = 0.0;
    }
    return v;
}

}  // namespace

int64_t mlp_n_params(const bcv_mlp_s &net) { return layout(net.d_in, net.width).total; }

bcv_mlp_s *mlp_create(int width, uint64_t seed, int device)
{
    BCV_REQUIRE(width >= 2 && width <= 1024, BCV_EINVAL, "width must be 2..1024");
    auto net = std::make_unique<bcv_mlp_s>();
    net->device = device;
    net->d_in = kMlpIn;
    net->width = width;
    const Layout l = layout(net->d_in, width);
    std::vector<float> P(l.total, 0.0f);
    std::mt19937_64 rng(seed);
    auto init = [&](int64_t at, int fan_in, int64_t count) {  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in))
        std::uniform_real_distribution<float> U(-1.0f / std::sqrt((float)fan_in), 1.0f / std::sqrt((float)fan_in));
        for (int64_t i = 0; i < count; ++i) P[at + i] = U(rng);
    };
    init(l.w1, net->d_in, (int64_t)net->d_in * width);
    init(l.w2, width, (int64_t)width * width);
    init(l.w3, width, (int64_t)width * kMlpOut);
    BCV_HIP(hipSetDevice(device));
    for (float **b : {&net->d_params, &net->d_grad, &net->d_m, &net->d_v})
        if (hipMalloc(b, l.total * sizeof(float)) != hipSuccess) fail(BCV_ENOMEM, "hipMalloc failed");
    BCV_HIP(hipMemcpy(net->d_params, P.data(), l.total * sizeof(float), hipMemcpyHostToDevice));
    BCV_HIP(hipMemset(net->d_m, 0, l.total * sizeof(float)));
    BCV_HIP(hipMemset(net->d_v, 0, l.total * sizeof(float)));
    return net.release();
}

void mlp_destroy(bcv_mlp_s *net)
{
    if (!net) return;
    (void)hipSetDevice(net->device);
    for (float *b : {net->d_params, net->d_grad, net->d_m, net->d_v})
        if (b) (void)hipFree(b);
    net->magic = 0;
    delete net;
}

void mlp_get_params(const bcv_mlp_s &net, float *host)
{
    BCV_HIP(hipMemcpy(host, net.d_params, mlp_n_params(net) * sizeof(float), hipMemcpyDeviceToHost));
}

void mlp_set_params(bcv_mlp_s &net, const float *host)
{
    BCV_HIP(hipMemcpy(net.d_params, host, mlp_n_params(net) * sizeof(float), hipMemcpyHostToDevice));
}

void mlp_forward_host(const bcv_mlp_s &net, int64_t n, const float *X, float *Y)
{
    if (n == 0) return;
    BCV_REQUIRE(n <= INT32_MAX, BCV_EINVAL, "batch too large");
    DevBuf<float> dX((size_t)n * net.d_in);
    Work w((int)n, net.width, net.d_in);
    BCV_HIP(hipMemcpy(dX.p, X, (size_t)n * net.d_in * sizeof(float), hipMemcpyHostToDevice));
    forward(net, dX.p, (int)n, w, nullptr);
    BCV_HIP(hipMemcpy(Y, w.Y.p, (size_t)n * kMlpOut * sizeof(float), hipMemcpyDeviceToHost));
}

void mlp_forward_noalloc(const bcv_mlp_s &net, int64_t n, const float *X, float *Y, hipStream_t st)
{
    BCV_REQUIRE(n >= 0 && n * net.width <= kNoAllocFloats, BCV_EINVAL,
                "batch too large for the fixed workspace: rows x width must not exceed 2^20");
    if (n == 0) return;
    float *ws = noalloc_workspace(net.device);
    float *Z = ws, *H1 = ws + kNoAllocFloats, *H2 = ws + 2 * kNoAllocFloats;
    const Layout l = layout(net.d_in, net.width);
    const float *P = net.d_params;
    const int W = net.width, B = (int)n;
    // the layers of forward(), with both pre-activations in one buffer (inference never reads them)
    gemm(false, false, B, W, net.d_in, X, net.d_in, P + l.w1, W, P + l.b1, false, Z, W, H1, st);
    gemm(false, false, B, W, W, H1, W, P + l.w2, W, P + l.b2, false, Z, W, H2, st);
    gemm(false, false, B, kMlpOut, W, H2, W, P + l.w3, kMlpOut, P + l.b3, false, Y, kMlpOut, nullptr, st);
}

double mlp_loss_grad_host(const bcv_mlp_s &net, int64_t n, const float *X, const float *r, float *grad)
{
    BCV_REQUIRE(n > 0 && n <= INT32_MAX, BCV_EINVAL, "batch size must be 1..2^31-1");
    const int B = (int)n;
    DevBuf<float> dX((size_t)B * net.d_in), dr(B);
    Work w(B, net.width, net.d_in);
    BCV_HIP(hipMemcpy(dX.p, X, (size_t)B * net.d_in * sizeof(float), hipMemcpyHostToDevice));
    BCV_HIP(hipMemcpy(dr.p, r, (size_t)B * sizeof(float), hipMemcpyHostToDevice));
    forward(net, dX.p, B, w, nullptr);
    loss_grad(B, w.Y.p, dr.p, kErrWeight, kErrEps, w.dY.p, w.terms.p, nullptr);
    backward(net, dX.p, B, w, net.d_grad, nullptr);
    BCV_HIP(hipMemcpy(grad, net.d_grad, mlp_n_params(net) * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<float> terms((size_t)B * kMlpOut);
    BCV_HIP(hipMemcpy(terms.data(), w.terms.p, terms.size() * sizeof(float), hipMemcpyDeviceToHost));
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < B; ++i) s0 += terms[2 * i], s1 += terms[2 * i + 1];
    return (s0 + kErrWeight * s1) / B;
}

void mlp_train(bcv_mlp_s &net, const bcv_mlp_train_opts &o, bcv_mlp_train_report *rep)
{
    BCV_REQUIRE(o.n_train >= 1 && o.n_valid >= 1 && o.epochs >= 1 && o.batch >= 1, BCV_EINVAL, "bad training sizes");
    BCV_REQUIRE(o.n_gauss_lo >= 1 && o.n_gauss_hi > o.n_gauss_lo && o.n_gauss_hi <= kQMaxGauss, BCV_EINVAL,
                "need 1 <= n_gauss_lo < n_gauss_hi <= 16");
    BCV_HIP(hipSetDevice(net.device));
    hipStream_t st = nullptr;
    const int64_t N = o.n_train, NV = o.n_valid, NT = N + NV;
    // training data from the quadrature at both orders
    const std::vector<bcv_touch_pair> pairs = sample_pairs(NT, o.seed);
    DevBuf<double> d_hi(NT), d_lo(NT);
    quadrature(pairs, o.n_gauss_hi, d_hi.p, st);
    quadrature(pairs, o.n_gauss_lo, d_lo.p, st);
    const std::vector<double> hi = download(d_hi.p, NT, st), lo = download(d_lo.p, NT, st);
    std::vector<double> q(NT);
    double ss = 0.0;
    for (int64_t i = 0; i < NT; ++i) {
        BCV_REQUIRE(std::isfinite(hi[i]) && std::isfinite(lo[i]) && lo[i] > 0.0, BCV_ESTATE,
                    "internal: quadrature of a training pair failed");
        q[i] = (hi[i] - lo[i]) / lo[i];
        if (i < N) ss += q[i] * q[i];
    }
    net.scale = std::sqrt(ss / N);
    BCV_REQUIRE(net.scale > 0.0, BCV_ESTATE, "internal: zero residual scale");
    net.n_gauss_lo = o.n_gauss_lo;
    net.n_gauss_hi = o.n_gauss_hi;
    std::vector<float> X((size_t)NT * net.d_in), R(NT);
    for (int64_t i = 0; i < NT; ++i) {
        pair_features(pairs[i], &X[(size_t)i * net.d_in]);
        R[i] = (float)(q[i] / net.scale);
    }
    DevBuf<float> dX(X.size()), dR(NT);
    BCV_HIP(hipMemcpy(dX.p, X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice));
    BCV_HIP(hipMemcpy(dR.p, R.data(), R.size() * sizeof(float), hipMemcpyHostToDevice));
    const int B = (int)std::min<int64_t>(o.batch, N);
    Work w(B, net.width, net.d_in);
    DevBuf<float> bX((size_t)B * net.d_in), bR(B);
    DevBuf<int32_t> bIdx(B);
    const int64_t n_par = mlp_n_params(net);
    BCV_HIP(hipMemset(net.d_m, 0, n_par * sizeof(float)));
    BCV_HIP(hipMemset(net.d_v, 0, n_par * sizeof(float)));
    std::vector<int32_t> perm(N);
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    std::mt19937_64 rng(o.seed ^ 0x9E3779B97F4A7C15ull);
    const int64_t steps_per_epoch = N / B;
    const int64_t total_steps = steps_per_epoch * o.epochs;
    int64_t step = 0;
    for (int ep = 0; ep < o.epochs; ++ep) {
        std::shuffle(perm.begin(), perm.end(), rng);
        for (int64_t s = 0; s < steps_per_epoch; ++s, ++step) {
            BCV_HIP(hipMemcpyAsync(bIdx.p, perm.data() + s * B, (size_t)B * sizeof(int32_t), hipMemcpyHostToDevice, st));
            gather_rows(B, net.d_in, bIdx.p, dX.p, bX.p, st);
            gather_rows(B, 1, bIdx.p, dR.p, bR.p, st);
            forward(net, bX.p, B, w, st);
            loss_grad(B, w.Y.p, bR.p, kErrWeight, kErrEps, w.dY.p, w.terms.p, st);
            backward(net, bX.p, B, w, net.d_grad, st);
            // cosine decay of the learning rate, Adam bias correction folded in
            const double frac = (double)step / std::max<int64_t>(total_steps, 1);
            const double lr = o.lr * 0.5 * (1.0 + std::cos(M_PI * frac));
            const double t = (double)(step + 1);
            const double lr_t = lr * std::sqrt(1.0 - std::pow(kAdamB2, t)) / (1.0 - std::pow(kAdamB1, t));
            adam_step(n_par, net.d_params, net.d_grad, net.d_m, net.d_v, (float)lr_t, kAdamB1, kAdamB2, kAdamEps, st);
            // the host permutation buffer is reused next step: wait for the copy
            BCV_HIP(hipStreamSynchronize(st));
        }
    }
    // held-out pairs: the first half calibrates the error estimate, the second half (pairs the
    // calibration never saw) reports the corrected value's error and the acceptance
    std::vector<float> Y((size_t)NV * kMlpOut);
    mlp_forward_host(net, NV, X.data() + (size_t)N * net.d_in, Y.data());
    std::vector<double> err(NV), raw(NV);
    for (int64_t i = 0; i < NV; ++i) {
        const int64_t j = N + i;
        const double value = lo[j] * (1.0 + net.scale * Y[2 * i]);
        err[i] = std::fabs(value - hi[j]) / std::fabs(hi[j]);
        raw[i] = net.scale * std::exp((double)Y[2 * i + 1]);
    }
    const int64_t n_cal = std::max<int64_t>(1, NV / 2);
    double ratio = 0.0;
    for (int64_t i = 0; i < n_cal; ++i) ratio = std::max(ratio, err[i] / raw[i]);
    net.kappa = std::max(1.0, kCalibrationMargin * ratio);
    const int64_t r0 = n_cal < NV ? n_cal : 0;  // one held-out pair: it serves both
    double max_err = 0.0, sum2 = 0.0, max_err_acc = 0.0, lo_max = 0.0;
    int64_t accepted = 0;
    for (int64_t i = r0; i < NV; ++i) {
        max_err = std::max(max_err, err[i]);
        sum2 += err[i] * err[i];
        lo_max = std::max(lo_max, std::fabs(lo[N + i] - hi[N + i]) / std::fabs(hi[N + i]));
        if (net.kappa * raw[i] <= o.tol) {
            ++accepted;
            max_err_acc = std::max(max_err_acc, err[i]);
        }
    }
    if (rep) {
        rep->residual_scale = net.scale;
        rep->kappa = net.kappa;
        rep->valid_max_rel_err = max_err;
        rep->valid_rms_rel_err = std::sqrt(sum2 / (double)(NV - r0));
        rep->valid_accepted = accepted;
        rep->valid_max_rel_err_accepted = max_err_acc;
        rep->valid_max_rel_err_lo = lo_max;
        rep->valid_reported = NV - r0;
    }
    net.trained = 1;
}

void surrogate_eval(const bcv_mlp_s &net, int64_t n, const bcv_touch_pair *pairs, double tol, double *value,
                    double *est_err, int32_t *fallback, int64_t *n_fallback)
{
    BCV_REQUIRE(net.trained, BCV_ESTATE, "the network has not been trained or loaded");
    BCV_REQUIRE(tol >= 0.0, BCV_EINVAL, "negative tolerance");
    BCV_HIP(hipSetDevice(net.device));
    int64_t nf = 0;
    if (n > 0) {
        std::vector<bcv_touch_pair> v(pairs, pairs + n);
        for (const auto &t : v) check_pair(t);
        DevBuf<double> d_lo(n);
        quadrature(v, net.n_gauss_lo, d_lo.p, nullptr);
        const std::vector<double> lo = download(d_lo.p, n, nullptr);
        std::vector<float> X((size_t)n * net.d_in), Y((size_t)n * kMlpOut);
        for (int64_t i = 0; i < n; ++i) pair_features(v[i], &X[(size_t)i * net.d_in]);
        mlp_forward_host(net, n, X.data(), Y.data());
        std::vector<bcv_touch_pair> back;
        std::vector<int64_t> back_idx;
        for (int64_t i = 0; i < n; ++i) {
            const double est = net.kappa * net.scale * std::exp((double)Y[2 * i + 1]);
            est_err[i] = est;
            value[i] = lo[i] * (1.0 + net.scale * (double)Y[2 * i]);
            const bool fb = !(est <= tol) || !std::isfinite(value[i]);
            fallback[i] = fb ? 1 : 0;
            if (fb) back.push_back(v[i]), back_idx.push_back(i);
        }
        nf = (int64_t)back.size();
        if (nf > 0) {
            DevBuf<double> d_hi(nf);
            quadrature(back, net.n_gauss_hi, d_hi.p, nullptr);
            const std::vector<double> hi = download(d_hi.p, nf, nullptr);
            for (int64_t k = 0; k < nf; ++k) value[back_idx[k]] = hi[k];
        }
    }
    if (n_fallback) *n_fallback = nf;
}

void touch_pair_quadrature(int device, int64_t n, const bcv_touch_pair *pairs, int n_gauss, double *out)
{
    BCV_HIP(hipSetDevice(device));
    if (n == 0) return;
    std::vector<bcv_touch_pair> v(pairs, pairs + n);
    for (const auto &t : v) check_pair(t);
    DevBuf<double> d(n);
    quadrature(v, n_gauss, d.p, nullptr);
    const std::vector<double> h = download(d.p, n, nullptr);
    std::copy(h.begin(), h.end(), out);
}

void mlp_save(const bcv_mlp_s &net, const char *path)
{
    BCV_REQUIRE(net.trained, BCV_ESTATE, "the network has not been trained or loaded");
    std::vector<float> P(mlp_n_params(net));
    mlp_get_params(net, P.data());
    FILE *fp = std::fopen(path, "wb");
    BCV_REQUIRE(fp != nullptr, BCV_EINVAL, std::string("cannot open ") + path);
    const uint32_t head[6] = {kFileMagic, 1u, (uint32_t)net.d_in, (uint32_t)net.width, (uint32_t)net.n_gauss_lo,
                              (uint32_t)net.n_gauss_hi};
    const double sk[2] = {net.scale, net.kappa};
    bool ok = std::fwrite(head, sizeof(head), 1, fp) == 1 && std::fwrite(sk, sizeof(sk), 1, fp) == 1 &&
              std::fwrite(P.data(), sizeof(float), P.size(), fp) == P.size();
    ok = (std::fclose(fp) == 0) && ok;
    BCV_REQUIRE(ok, BCV_EINVAL, std::string("write failed: ") + path);
}

bcv_mlp_s *mlp_load(const char *path, int device)
{
    FILE *fp = std::fopen(path, "rb");
    BCV_REQUIRE(fp != nullptr, BCV_EINVAL, std::string("cannot open ") + path);
    uint32_t head[6];
    double sk[2] = {0.0, 0.0};
    bool ok = std::fread(head, sizeof(head), 1, fp) == 1 && std::fread(sk, sizeof(sk), 1, fp) == 1 &&
              head[0] == kFileMagic && head[1] == 1u && head[2] == (uint32_t)kMlpIn && head[3] >= 2 && head[3] <= 1024 &&
              head[4] >= 1 && head[5] > head[4] && head[5] <= (uint32_t)kQMaxGauss && sk[0] > 0.0 && sk[1] >= 1.0;
    if (!ok) {
        std::fclose(fp);
        fail(BCV_EINVAL, std::string("not a surrogate file: ") + path);
    }
    std::unique_ptr<bcv_mlp_s, void (*)(bcv_mlp_s *)> net(mlp_create((int)head[3], 0, device), mlp_destroy);
    std::vector<float> P(mlp_n_params(*net));
    ok = std::fread(P.data(), sizeof(float), P.size(), fp) == P.size();
    std::fclose(fp);
    BCV_REQUIRE(ok, BCV_EINVAL, std::string("truncated surrogate file: ") + path);
    mlp_set_params(*net, P.data());
    net->scale = sk[0];
    net->kappa = sk[1];
    net->n_gauss_lo = (int)head[4];
    net->n_gauss_hi = (int)head[5];
    net->trained = 1;
    return net.release();
}

}  // namespace bcv
