// C ABI of the learned warm start: POD basis and MLP (forward, backward, Adam).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <vector>

#include "device.h"
#include "runtime.h"

using namespace mtf;

namespace {

using cd = std::complex<double>;

uint64_t splitmix64(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t& st) { return (splitmix64(st) >> 11) * (1.0 / 9007199254740992.0); }

// Cyclic Jacobi for a real symmetric matrix a (n x n, row-major, destroyed): eigenvalues w,
// eigenvectors in the columns of v (row-major n x n).
void jacobi_eig(std::vector<double>& a, int n, std::vector<double>& w, std::vector<double>& v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += a[(size_t)i * n + j] * a[(size_t)i * n + j];
                if (i != j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = a[(size_t)p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - sn * akq;
                    a[(size_t)k * n + q] = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - sn * aqk;
                    a[(size_t)q * n + k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - sn * vkq;
                    v[(size_t)k * n + q] = sn * vkp + c * vkq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = a[(size_t)i * n + i];
}

// Orthonormalise the q columns of X (m x q, column-major complex, double) by modified
// Gram-Schmidt applied twice.
void orthonormalise(std::vector<cd>& X, int m, int q) {
    for (int j = 0; j < q; ++j) {
        cd* xj = &X[(size_t)j * m];
        for (int pass = 0; pass < 2; ++pass)
            for (int i = 0; i < j; ++i) {
                const cd* xi = &X[(size_t)i * m];
                cd d = 0.0;
                for (int k = 0; k < m; ++k) d += std::conj(xi[k]) * xj[k];
                for (int k = 0; k < m; ++k) xj[k] -= d * xi[k];
            }
        double nr = 0.0;
        for (int k = 0; k < m; ++k) nr += std::norm(xj[k]);
        nr = std::sqrt(nr);
        for (int k = 0; k < m; ++k) xj[k] = nr > 0 ? xj[k] / nr : 0.0;
    }
}

void upload_c128(DevBuf<double>& d, const std::vector<cd>& h, hipStream_t s) {
    d.alloc(2 * h.size());
    HIPCHK(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(cd), hipMemcpyHostToDevice, s));
}

std::vector<cd> download_c128(const double* d, size_t n, hipStream_t s) {
    std::vector<cd> h(n);
    HIPCHK(hipMemcpyAsync(h.data(), d, n * sizeof(cd), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return h;
}


}  // namespace

struct mtf_mlp_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_in = 0, width = 0, n_out = 0;
    int64_t nparams = 0;
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;
    DevBuf<float> params, grads, m1, m2;
    DevBuf<float> A1, A2, Y, dY, dA, dZ, Xb, Tb, lossp;
    DevBuf<int> idx;
    int cap = 0;
    int64_t adam_t = 0;

    void ensure(int n) {
        if (n <= cap) return;
        A1.alloc((size_t)n * width);
        A2.alloc((size_t)n * width);
        Y.alloc((size_t)n * n_out);
        dY.alloc((size_t)n * n_out);
        dA.alloc((size_t)n * width);
        dZ.alloc((size_t)n * width);
        Xb.alloc((size_t)n * n_in);
        Tb.alloc((size_t)n * n_out);
        lossp.alloc(((size_t)n * n_out + 255) / 256 + 1);
        idx.alloc(n);
        cap = n;
    }
    const float* P(int64_t o) const { return params.p + o; }
    float* G(int64_t o) { return grads.p + o; }

    void forward(int n, const float* X, float* out) {
        hipStream_t s = stream;
        launch_sgemm(n, width, n_in, X, n_in, 0, P(oW1), n_in, 1, P(ob1), 1, A1.p, width, 0, s);
        launch_sgemm(n, width, width, A1.p, width, 0, P(oW2), width, 1, P(ob2), 1, A2.p, width, 0, s);
        launch_sgemm(n, n_out, width, A2.p, width, 0, P(oW3), width, 1, P(ob3), 0, out, n_out, 0, s);
    }

    // forward + MSE + backward into grads; returns the number of loss partial sums
    int loss_backward(int n, const float* X, const float* T) {
        hipStream_t s = stream;
        forward(n, X, Y.p);
        const int64_t ny = (int64_t)n * n_out;
        const int nbl = launch_mse(Y.p, T, dY.p, ny, 1.0f / (float)ny, lossp.p, s);
        // layer 3
        launch_sgemm(n_out, width, n, dY.p, n_out, 1, A2.p, width, 0, nullptr, 0, G(oW3), width, 0, s);
        launch_colsum(dY.p, n, n_out, G(ob3), s);
        launch_sgemm(n, width, n_out, dY.p, n_out, 0, P(oW3), width, 0, nullptr, 0, dA.p, width, 0, s);
        launch_tanh_back(A2.p, dA.p, dZ.p, (int64_t)n * width, s);
        // layer 2
        launch_sgemm(width, width, n, dZ.p, width, 1, A1.p, width, 0, nullptr, 0, G(oW2), width, 0, s);
        launch_colsum(dZ.p, n, width, G(ob2), s);
        launch_sgemm(n, width, width, dZ.p, width, 0, P(oW2), width, 0, nullptr, 0, dA.p, width, 0, s);
        launch_tanh_back(A1.p, dA.p, dZ.p, (int64_t)n * width, s);
        // layer 1
        launch_sgemm(width, n_in, n, dZ.p, width, 1, X, n_in, 0, nullptr, 0, G(oW1), n_in, 0, s);
        launch_colsum(dZ.p, n, width, G(ob1), s);
        return nbl;
    }

    float read_loss(int nbl) {
        std::vector<float> h(nbl);
        HIPCHK(hipMemcpyAsync(h.data(), lossp.p, nbl * sizeof(float), hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        double l = 0;
        for (float v : h) l += v;
        return (float)l;
    }
};

namespace {

void check_mlp(mtf_mlp m) {
    if (!m) throw ArgError("mlp is NULL");
}

}  // namespace

extern "C" {

int mtf_pod_build(mtf_problem p, int32_t nsnap, const void* U_dev, int64_t ldu, int32_t r, void* Phi_dev, int64_t ldphi,
                  double* sv) {
    return guarded([&] {
        int dev;
        hipStream_t s;
        int64_t N;
        problem_info(p, &dev, &s, &N);
        if (nsnap < 1 || r < 1 || r > nsnap || r > 256 || !U_dev || !Phi_dev || !sv || ldu < N || ldphi < N)
            throw ArgError("mtf_pod_build: bad sizes or pointers");
        DeviceGuard g(dev);
        const int q = std::min<int>(nsnap, r + 16);
        const double* U = static_cast<const double*>(U_dev);
        DevBuf<double> G, X, Y, Z;
        G.alloc(2 * (size_t)nsnap * nsnap);
        launch_zgemm(nsnap, nsnap, (int)N, true, U, ldu, U, ldu, G.p, nsnap, s);   // G = U^H U
        // subspace iteration on G
        uint64_t st = 0x5EEDull + nsnap;
        std::vector<cd> Xh((size_t)nsnap * q);
        for (auto& v : Xh) v = cd(uniform01(st) - 0.5, uniform01(st) - 0.5);
        orthonormalise(Xh, nsnap, q);
        Y.alloc(2 * (size_t)nsnap * q);
        std::vector<double> prev(q, 0.0);
        for (int it = 0; it < 60; ++it) {
            upload_c128(X, Xh, s);
            launch_zgemm(nsnap, q, nsnap, false, G.p, nsnap, X.p, nsnap, Y.p, nsnap, s);
            std::vector<cd> Yh = download_c128(Y.p, (size_t)nsnap * q, s);
            // Rayleigh quotients for the convergence test
            std::vector<double> rq(q);
            for (int j = 0; j < q; ++j) {
                cd d = 0.0;
                for (int k = 0; k < nsnap; ++k) d += std::conj(Xh[(size_t)j * nsnap + k]) * Yh[(size_t)j * nsnap + k];
                rq[j] = d.real();
            }
            Xh = Yh;
            orthonormalise(Xh, nsnap, q);
            double ch = 0.0;
            for (int j = 0; j < r; ++j) ch = std::max(ch, std::fabs(rq[j] - prev[j]) / std::max(1e-300, std::fabs(rq[j])));
            prev = rq;
            if (it > 3 && ch < 1e-10) break;
        }
        // Rayleigh-Ritz: H = X^H G X (q x q Hermitian) as a real symmetric 2q x 2q matrix
        upload_c128(X, Xh, s);
        launch_zgemm(nsnap, q, nsnap, false, G.p, nsnap, X.p, nsnap, Y.p, nsnap, s);
        std::vector<cd> GX = download_c128(Y.p, (size_t)nsnap * q, s);
        std::vector<cd> H((size_t)q * q);
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                cd d = 0.0;
                for (int k = 0; k < nsnap; ++k) d += std::conj(Xh[(size_t)i * nsnap + k]) * GX[(size_t)j * nsnap + k];
                H[(size_t)i * q + j] = d;
            }
        const int n2 = 2 * q;
        std::vector<double> a((size_t)n2 * n2), w, v;
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                const cd h = 0.5 * (H[(size_t)i * q + j] + std::conj(H[(size_t)j * q + i]));
                a[(size_t)i * n2 + j] = h.real();
                a[(size_t)i * n2 + q + j] = -h.imag();
                a[(size_t)(q + i) * n2 + j] = h.imag();
                a[(size_t)(q + i) * n2 + q + j] = h.real();
            }
        jacobi_eig(a, n2, w, v);
        std::vector<int> order(n2);
        for (int i = 0; i < n2; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return w[x] > w[y]; });
        // each eigenvalue of the Hermitian matrix appears twice (vectors x+iy and i(x+iy)); keep one
        std::vector<std::vector<cd>> keep;
        std::vector<double> lam;
        for (int t = 0; t < n2 && (int)keep.size() < r; ++t) {
            const int c = order[t];
            std::vector<cd> z(q);
            for (int i = 0; i < q; ++i) z[i] = cd(v[(size_t)i * n2 + c], v[(size_t)(q + i) * n2 + c]);
            for (auto& u : keep) {
                cd d = 0.0;
                for (int i = 0; i < q; ++i) d += std::conj(u[i]) * z[i];
                for (int i = 0; i < q; ++i) z[i] -= d * u[i];
            }
            double nr = 0.0;
            for (auto& e : z) nr += std::norm(e);
            nr = std::sqrt(nr);
            if (nr < 0.5) continue;
            for (auto& e : z) e /= nr;
            keep.push_back(z);
            lam.push_back(w[c]);
        }
        if ((int)keep.size() < r) throw NonFiniteError("POD: Rayleigh-Ritz produced fewer modes than requested");
        // Z = X W Lambda^{-1/2} (nsnap x r);  Phi = U Z
        std::vector<cd> Zh((size_t)nsnap * r, 0.0);
        for (int j = 0; j < r; ++j) {
            if (!(lam[j] > 0.0)) throw NonFiniteError("POD: non-positive Gram eigenvalue (rank-deficient snapshots)");
            const double sc = 1.0 / std::sqrt(lam[j]);
            for (int i = 0; i < q; ++i)
                for (int k = 0; k < nsnap; ++k) Zh[(size_t)j * nsnap + k] += Xh[(size_t)i * nsnap + k] * keep[j][i] * sc;
            sv[j] = std::sqrt(lam[j]);
        }
        upload_c128(Z, Zh, s);
        launch_zgemm((int)N, r, nsnap, false, U, ldu, Z.p, nsnap, static_cast<double*>(Phi_dev), ldphi, s);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        return MTF_OK;
    });
}

int mtf_pod_project(mtf_problem p, int32_t r, const void* Phi_dev, int64_t ldphi, int32_t n, const void* X_dev,
                    int64_t ldx, void* C_dev) {
    return guarded([&] {
        int dev;
        hipStream_t s;
        int64_t N;
        problem_info(p, &dev, &s, &N);
        if (r < 1 || n < 1 || !Phi_dev || !X_dev || !C_dev || ldphi < N || ldx < N) throw ArgError("mtf_pod_project: bad arguments");
        DeviceGuard g(dev);
        launch_zgemm(r, n, (int)N, true, static_cast<const double*>(Phi_dev), ldphi, static_cast<const double*>(X_dev),
                     ldx, static_cast<double*>(C_dev), r, s);     // C = Phi^H X
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        return MTF_OK;
    });
}

int mtf_pod_expand(mtf_problem p, int32_t r, const void* Phi_dev, int64_t ldphi, int32_t n, const void* C_dev,
                   void* X_dev, int64_t ldx) {
    return guarded([&] {
        int dev;
        hipStream_t s;
        int64_t N;
        problem_info(p, &dev, &s, &N);
        if (r < 1 || n < 1 || !Phi_dev || !X_dev || !C_dev || ldphi < N || ldx < N) throw ArgError("mtf_pod_expand: bad arguments");
        DeviceGuard g(dev);
        launch_zgemm((int)N, n, r, false, static_cast<const double*>(Phi_dev), ldphi, static_cast<const double*>(C_dev),
                     r, static_cast<double*>(X_dev), ldx, s);     // X = Phi C
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        return MTF_OK;
    });
}

int mtf_mlp_create(mtf_mlp* out, int device, void* stream, int32_t n_in, int32_t width, int32_t n_out, uint64_t seed) {
    return guarded([&] {
        if (!out) throw ArgError("out is NULL");
        *out = nullptr;
        if (n_in < 1 || width < 1 || n_out < 1 || n_in > 4096 || width > 4096 || n_out > 4096)
            throw ArgError("mlp sizes out of range");
        int nd = 0;
        HIPCHK(hipGetDeviceCount(&nd));
        if (device < 0 || device >= nd) throw ArgError("device index out of range");
        DeviceGuard g(device);
        auto m = std::make_unique<mtf_mlp_s>();
        m->device = device;
        m->stream = static_cast<hipStream_t>(stream);
        m->n_in = n_in; m->width = width; m->n_out = n_out;
        int64_t o = 0;
        m->oW1 = o; o += (int64_t)width * n_in;
        m->ob1 = o; o += width;
        m->oW2 = o; o += (int64_t)width * width;
        m->ob2 = o; o += width;
        m->oW3 = o; o += (int64_t)n_out * width;
        m->ob3 = o; o += n_out;
        m->nparams = o;
        std::vector<float> init(o, 0.f);
        uint64_t st = seed;
        auto fill = [&](int64_t off, int fan_out, int fan_in) {
            const double a = std::sqrt(6.0 / (fan_in + fan_out));
            for (int64_t k = 0; k < (int64_t)fan_out * fan_in; ++k) init[off + k] = (float)((2.0 * uniform01(st) - 1.0) * a);
        };
        fill(m->oW1, width, n_in);
        fill(m->oW2, width, width);
        fill(m->oW3, n_out, width);
        m->params.upload(init, m->stream);
        m->grads.alloc(o);
        std::vector<float> zeros(o, 0.f);
        m->m1.upload(zeros, m->stream);
        m->m2.upload(zeros, m->stream);
        HIPCHK(hipStreamSynchronize(m->stream));
        *out = m.release();
        return MTF_OK;
    });
}

int mtf_mlp_destroy(mtf_mlp m) {
    if (!m) return MTF_OK;
    return guarded([&] {
        DeviceGuard g(m->device);
        (void)hipStreamSynchronize(m->stream);
        delete m;
        return MTF_OK;
    });
}

int mtf_mlp_num_params(mtf_mlp m, int64_t* n) {
    return guarded([&] {
        check_mlp(m);
        if (!n) throw ArgError("n is NULL");
        *n = m->nparams;
        return MTF_OK;
    });
}

int mtf_mlp_get_params(mtf_mlp m, float* host) {
    return guarded([&] {
        check_mlp(m);
        if (!host) throw ArgError("host is NULL");
        DeviceGuard g(m->device);
        HIPCHK(hipMemcpyAsync(host, m->params.p, m->nparams * sizeof(float), hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        return MTF_OK;
    });
}

int mtf_mlp_set_params(mtf_mlp m, const float* host) {
    return guarded([&] {
        check_mlp(m);
        if (!host) throw ArgError("host is NULL");
        for (int64_t i = 0; i < m->nparams; ++i)
            if (!std::isfinite(host[i])) throw ArgError("non-finite parameter");
        DeviceGuard g(m->device);
        HIPCHK(hipMemcpyAsync(m->params.p, host, m->nparams * sizeof(float), hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        m->adam_t = 0;
        return MTF_OK;
    });
}

int mtf_mlp_forward(mtf_mlp m, int32_t n, const float* X_dev, float* Y_dev) {
    return guarded([&] {
        check_mlp(m);
        if (n < 1 || !X_dev || !Y_dev) throw ArgError("bad arguments");
        DeviceGuard g(m->device);
        m->ensure(n);
        m->forward(n, X_dev, Y_dev);
        HIPCHK(hipGetLastError());
        return MTF_OK;
    });
}

int mtf_mlp_loss_grad(mtf_mlp m, int32_t n, const float* X_dev, const float* T_dev, float* loss, float* grad_host) {
    return guarded([&] {
        check_mlp(m);
        if (n < 1 || !X_dev || !T_dev || !loss) throw ArgError("bad arguments");
        DeviceGuard g(m->device);
        m->ensure(n);
        const int nbl = m->loss_backward(n, X_dev, T_dev);
        HIPCHK(hipGetLastError());
        *loss = m->read_loss(nbl);
        if (grad_host) {
            HIPCHK(hipMemcpyAsync(grad_host, m->grads.p, m->nparams * sizeof(float), hipMemcpyDeviceToHost, m->stream));
            HIPCHK(hipStreamSynchronize(m->stream));
        }
        return MTF_OK;
    });
}

int mtf_mlp_train(mtf_mlp m, int32_t n, const float* X_dev, const float* T_dev, const mtf_train_opts* o,
                  float* loss_hist) {
    return guarded([&] {
        check_mlp(m);
        if (!o || o->struct_size < (int)sizeof(mtf_train_opts)) throw ArgError("bad mtf_train_opts");
        if (n < 1 || !X_dev || !T_dev || o->epochs < 1 || o->batch < 1) throw ArgError("bad arguments");
        if (!(o->lr > 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f) || !(o->eps > 0.f))
            throw ArgError("bad Adam hyper-parameters");
        DeviceGuard g(m->device);
        hipStream_t s = m->stream;
        const int B = std::min<int>(o->batch, n);
        m->ensure(std::max(n, B));
        DevBuf<int> perm;
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        uint64_t st = o->seed;
        for (int ep = 0; ep < o->epochs; ++ep) {
            for (int i = n - 1; i > 0; --i) {
                const int j = (int)(splitmix64(st) % (uint64_t)(i + 1));
                std::swap(order[i], order[j]);
            }
            perm.upload(order, s);
            for (int b0 = 0; b0 + B <= n; b0 += B) {
                launch_gather_rows(X_dev, perm.p + b0, B, m->n_in, m->Xb.p, s);
                launch_gather_rows(T_dev, perm.p + b0, B, m->n_out, m->Tb.p, s);
                m->loss_backward(B, m->Xb.p, m->Tb.p);
                ++m->adam_t;
                const double bc1 = 1.0 - std::pow((double)o->beta1, (double)m->adam_t);
                const double bc2 = 1.0 - std::pow((double)o->beta2, (double)m->adam_t);
                const float lr_t = (float)(o->lr * std::sqrt(bc2) / bc1);
                launch_adam(m->params.p, m->grads.p, m->m1.p, m->m2.p, m->nparams, lr_t, o->beta1, o->beta2, o->eps, s);
            }
            HIPCHK(hipGetLastError());
            if (loss_hist) {
                m->forward(n, X_dev, m->Y.p);
                const int64_t ny = (int64_t)n * m->n_out;
                const int nbl = launch_mse(m->Y.p, T_dev, m->dY.p, ny, 1.0f / (float)ny, m->lossp.p, s);
                loss_hist[ep] = m->read_loss(nbl);
            } else {
                HIPCHK(hipStreamSynchronize(s));
            }
        }
        return MTF_OK;
    });
}

}  // extern "C"
