// plan_driver.cpp -- drives the batched entry points (sweep_eval_batched,
// sweep_backward_ex) of the plan code built against the CPU stand-in of the
// HIP runtime.
//
//   plan_driver selftest   plants the hazards the stand-in must report (a
//                          graph executable destroyed and memory freed while
//                          a launch is in flight); prints the report.
//   plan_driver plans      the four-sweep rational batch of degrees 2 to 4,
//                          then more batch shapes than the plan cache holds
//                          (so plans are evicted), launched on two streams
//                          with no synchronisation between calls, output
//                          buffers changing between calls (graph parameter
//                          updates), adjoint calls with weight gradients in
//                          between, and the first batch again after its plan
//                          was evicted.  Prints the report; exit status 0
//                          only without violations.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/sweep.h"
#include "../../paper_1110_5450_amd/csrc/kernels.hpp"
#include "stub_kernels.hpp"

namespace {

struct HostBatch {
    std::vector<int32_t> path_n, path_deg, prof_n, prof_deg, prof_closed, n_u, n_v;
    double* path_ctrl = nullptr;
    double* prof_ctrl = nullptr;
    double* path_w = nullptr;
    double* prof_w = nullptr;
    sweep_batch b{};
};

void* dev_alloc(size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        std::fprintf(stderr, "stub hipMalloc failed\n");
        std::exit(2);
    }
    std::memset(p, 0, bytes);
    return p;
}

void make_batch(HostBatch& h, const std::vector<int>& deg, const std::vector<int>& nu, const std::vector<int>& nv,
                bool rational, std::mt19937& rng)
{
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const int n = (int)deg.size();
    long long np = 0, nq = 0;
    for (int k = 0; k < n; ++k) {
        h.path_n.push_back(deg[k] + 5 + k % 3);
        h.path_deg.push_back(deg[k]);
        h.prof_n.push_back(6 + k % 4);
        h.prof_deg.push_back(2 + k % 2);
        h.prof_closed.push_back(1);
        h.n_u.push_back(nu[k]);
        h.n_v.push_back(nv[k]);
        np += h.path_n.back();
        nq += h.prof_n.back();
    }
    h.path_ctrl = (double*)dev_alloc(sizeof(double) * 3 * np);
    h.prof_ctrl = (double*)dev_alloc(sizeof(double) * 3 * nq);
    for (long long i = 0; i < 3 * np; ++i) h.path_ctrl[i] = U(rng);
    for (long long i = 0; i < 3 * nq; ++i) h.prof_ctrl[i] = U(rng);
    if (rational) {
        h.path_w = (double*)dev_alloc(sizeof(double) * np);
        h.prof_w = (double*)dev_alloc(sizeof(double) * nq);
        for (long long i = 0; i < np; ++i) h.path_w[i] = 1.0 + 0.5 * U(rng);
        for (long long i = 0; i < nq; ++i) h.prof_w[i] = 1.0 + 0.5 * U(rng);
    }
    sweep_batch& b = h.b;
    b.n_sweeps = n;
    b.path_n = h.path_n.data();
    b.path_degree = h.path_deg.data();
    b.prof_n = h.prof_n.data();
    b.prof_degree = h.prof_deg.data();
    b.prof_closed = h.prof_closed.data();
    b.n_u = h.n_u.data();
    b.n_v = h.n_v.data();
    b.path_ctrl = h.path_ctrl;
    b.prof_ctrl = h.prof_ctrl;
    b.path_weights = h.path_w;
    b.prof_weights = h.prof_w;
}

struct Buffers {
    float* pos = nullptr;
    float* nrm = nullptr;
    void* ws = nullptr;
    size_t ws_bytes = 0;
};

int check(sweep_status st, const char* what)
{
    if (st != SWEEP_OK) {
        std::fprintf(stderr, "%s failed: %d %s\n", what, st, sweep_last_error());
        return 1;
    }
    return 0;
}

int selftest()
{
    hipStream_t s = (hipStream_t)0x1;
    void* a = dev_alloc(4096);
    void* b = dev_alloc(4096);
    hipGraph_t g;
    hipGraphCreate(&g, 0);
    sweep::BatchedKernels K = sweep::batched_kernels(true, false, true, true, 1024, false, false, false, false);
    void *descs = a, *vch = a, *qc = a, *qw = nullptr, *kn = nullptr, *ptab = b;
    void* params[6] = {&descs, &vch, &qc, &qw, &kn, &ptab};
    hipKernelNodeParams prm{};
    prm.func = const_cast<void*>(K.profile);
    prm.gridDim = dim3(1);
    prm.blockDim = dim3(256);
    prm.kernelParams = params;
    hipGraphNode_t node;
    hipGraphAddKernelNode(&node, g, nullptr, 0, &prm);
    hipGraphExec_t ex;
    hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphLaunch(ex, s);
    hipGraphExecKernelNodeSetParams(ex, node, &prm);   // in flight: reported
    hipGraphExecDestroy(ex);                           // in flight: reported
    hipFree(b);                                        // in use: reported
    hipStreamSynchronize(s);
    hipGraphDestroy(g);
    hipFree(a);
    return stub::report(true);
}

int plans()
{
    std::mt19937 rng(20261203);
    hipStream_t streams[2] = {(hipStream_t)0x1, (hipStream_t)0x2};
    sweep_options opt;
    sweep_default_options(&opt);
    int bad = 0;

    // the four-sweep rational batch of degrees 2 to 4
    HostBatch first;
    make_batch(first, {3, 2, 3, 4}, {200, 999, 64, 1500}, {40, 17, 256, 9}, true, rng);
    std::vector<HostBatch> shapes(40);
    for (int i = 0; i < 40; ++i) {
        std::vector<int> deg, nu, nv;
        const int n = 1 + i % 5;
        for (int k = 0; k < n; ++k) {
            deg.push_back(1 + (i + k) % 7);
            // some sweeps longer than one frame chunk (the chunk-walking frame kernel)
            nu.push_back(16 + 37 * i + 101 * k + (i % 7 == 3 && k == 0 ? 4500 : 0));
            nv.push_back(8 + (i * 13 + k * 7) % 200);
        }
        make_batch(shapes[i], deg, nu, nv, i % 2 == 0, rng);
    }
    std::vector<HostBatch*> order{&first};
    for (auto& h : shapes) order.push_back(&h);
    order.push_back(&first);

    std::vector<Buffers> owned;
    int call = 0, shape = 0;
    for (HostBatch* h : order) {
        // every third shape samples its paths at equal arc length or
        // adaptively (arc plans built, updated and evicted among the others)
        sweep_options o = opt;
        if (shape % 3 == 1) {
            o.u_sampling = shape % 2 ? SWEEP_U_ARCLENGTH : SWEEP_U_ADAPTIVE;
            o.u_lambda = shape % 2 ? 0.0 : 0.5;
        }
        ++shape;
        for (int rep = 0; rep < 3; ++rep, ++call) {
            const int64_t elems = sweep_batched_output_elems(&h->b);
            Buffers B;
            B.pos = (float*)dev_alloc(sizeof(float) * elems);
            B.nrm = (float*)dev_alloc(sizeof(float) * elems);
            B.ws_bytes = sweep_batched_workspace_size(&h->b, &o);
            B.ws = dev_alloc(B.ws_bytes);
            owned.push_back(B);
            bad += check(sweep_eval_batched(&h->b, &o, B.pos, B.nrm, B.ws, B.ws_bytes, streams[call % 2]),
                         "sweep_eval_batched");
            if (call % 4 == 3 && o.u_sampling == SWEEP_U_PARAMETER) {
                const size_t wb = sweep_backward_workspace_size(&h->b, &opt);
                void* ws = dev_alloc(wb);
                long long np = 0, nq = 0;
                for (int k = 0; k < h->b.n_sweeps; ++k) { np += h->path_n[k]; nq += h->prof_n[k]; }
                double* gP = (double*)dev_alloc(sizeof(double) * 3 * np);
                double* gQ = (double*)dev_alloc(sizeof(double) * 3 * nq);
                sweep_param_grads pg{};
                if (h->path_w) {
                    pg.path_weights = (double*)dev_alloc(sizeof(double) * np);
                    pg.prof_weights = (double*)dev_alloc(sizeof(double) * nq);
                }
                bad += check(sweep_backward_ex(&h->b, &opt, B.pos, B.nrm, gP, gQ, h->path_w ? &pg : nullptr, ws, wb,
                                               streams[call % 2]),
                             "sweep_backward_ex");
                // the caller's buffers stay allocated until the end (freeing
                // them in flight would be the caller's mistake, not the plan's)
                owned.push_back(Buffers{(float*)gP, (float*)gQ, ws, wb});
                if (pg.path_weights) owned.push_back(Buffers{(float*)pg.path_weights, (float*)pg.prof_weights, nullptr, 0});
            }
        }
    }
    hipDeviceSynchronize();
    sweep_release_caches();
    for (auto& B : owned) {
        hipFree(B.pos);
        hipFree(B.nrm);
        if (B.ws) hipFree(B.ws);
    }
    const int v = stub::report(true);
    std::printf("calls %d, failed calls %d\n", call, bad);
    return v + bad;
}

// The batched autotuner on the four-sweep rational batch: plans for every
// candidate configuration, timed replays, then the automatic plan dropped and
// rebuilt with the recorded choice.
int tune()
{
    std::mt19937 rng(11);
    HostBatch h;
    make_batch(h, {3, 2, 3, 4}, {200, 999, 64, 5000}, {40, 17, 256, 9}, true, rng);
    sweep_options opt;
    sweep_default_options(&opt);
    const int64_t elems = sweep_batched_output_elems(&h.b);
    float* pos = (float*)dev_alloc(sizeof(float) * elems);
    float* nrm = (float*)dev_alloc(sizeof(float) * elems);
    const size_t wb = sweep_batched_workspace_size(&h.b, &opt);
    void* ws = dev_alloc(wb);
    int32_t cfg = -1;
    float ms = -1.f;
    int bad = check(sweep_autotune_batched(&h.b, &opt, pos, nrm, ws, wb, (hipStream_t)0x1, &cfg, &ms),
                    "sweep_autotune_batched");
    const int auto_cfg = sweep_batched_config_for(&h.b, &opt, 1);
    bad += check(sweep_eval_batched(&h.b, &opt, pos, nrm, ws, wb, (hipStream_t)0x1), "sweep_eval_batched");
    // then more batch shapes than the plan cache holds (evictions), each
    // evaluated and differentiated, on the null stream
    std::vector<HostBatch> more(24);
    for (int i = 0; i < 24; ++i) {
        std::vector<int> deg, nu, nv;
        for (int k = 0; k < 1 + i % 4; ++k) {
            deg.push_back(1 + (i + k) % 7);
            nu.push_back(20 + 53 * i + 7 * k + (i % 5 == 1 ? 4200 : 0));
            nv.push_back(5 + (i * 11 + k) % 90);
        }
        make_batch(more[i], deg, nu, nv, i % 3 == 0, rng);
        opt.batch_stages = i % 5;   // one to four pipeline stages (0: automatic)
        const int64_t e2 = sweep_batched_output_elems(&more[i].b);
        float* p2 = (float*)dev_alloc(sizeof(float) * e2);
        float* n2 = (float*)dev_alloc(sizeof(float) * e2);
        const size_t w2 = sweep_batched_workspace_size(&more[i].b, &opt);
        void* ws2 = dev_alloc(w2);
        bad += check(sweep_eval_batched(&more[i].b, &opt, p2, n2, ws2, w2, nullptr), "sweep_eval_batched");
        if (i % 2 == 0) {
            int32_t c2 = -1;
            float m2 = 0.f;
            bad += check(sweep_autotune_batched(&more[i].b, &opt, p2, n2, ws2, w2, nullptr, &c2, &m2),
                         "sweep_autotune_batched");
        }
        const size_t wbk = sweep_backward_workspace_size(&more[i].b, &opt);
        void* wsb = dev_alloc(wbk);
        long long np = 0, nq = 0;
        for (int k = 0; k < more[i].b.n_sweeps; ++k) { np += more[i].path_n[k]; nq += more[i].prof_n[k]; }
        double* gP = (double*)dev_alloc(sizeof(double) * 3 * np);
        double* gQ = (double*)dev_alloc(sizeof(double) * 3 * nq);
        bad += check(sweep_backward(&more[i].b, &opt, p2, gP, gQ, wsb, wbk, nullptr), "sweep_backward");
    }
    {
        // a batch of 300 sweeps of mixed lengths (short and chunk-walking
        // frame nodes of two degrees, three pipeline stages), evaluated into
        // two sets of buffers (node parameter updates), then differentiated
        opt.batch_stages = 3;
        HostBatch big;
        std::vector<int> deg, nu, nv;
        for (int k = 0; k < 300; ++k) {
            deg.push_back(2 + k % 2);
            nu.push_back(16 + (k * 97) % 5000);
            nv.push_back(8 + (k * 31) % 120);
        }
        make_batch(big, deg, nu, nv, false, rng);
        const int64_t e3 = sweep_batched_output_elems(&big.b);
        const size_t w3 = sweep_batched_workspace_size(&big.b, &opt);
        for (int rep = 0; rep < 2; ++rep) {
            float* p3 = (float*)dev_alloc(sizeof(float) * e3);
            float* n3 = (float*)dev_alloc(sizeof(float) * e3);
            void* ws3 = dev_alloc(w3);
            bad += check(sweep_eval_batched(&big.b, &opt, p3, n3, ws3, w3, nullptr), "sweep_eval_batched");
            if (rep == 1) {
                const size_t wbk = sweep_backward_workspace_size(&big.b, &opt);
                void* wsb = dev_alloc(wbk);
                long long np = 0, nq = 0;
                for (int k = 0; k < big.b.n_sweeps; ++k) { np += big.path_n[k]; nq += big.prof_n[k]; }
                double* gP = (double*)dev_alloc(sizeof(double) * 3 * np);
                double* gQ = (double*)dev_alloc(sizeof(double) * 3 * nq);
                bad += check(sweep_backward(&big.b, &opt, p3, gP, gQ, wsb, wbk, nullptr), "sweep_backward");
            }
        }
    }
    {
        // Frenet frames and a sweep law with given knots (extended row
        // records): two evaluations into different buffers, the adjoint
        // refused
        HostBatch hx;
        make_batch(hx, {3, 2, 3, 1}, {200, 1500, 5000, 90}, {40, 17, 9, 12}, false, rng);
        sweep_options ox;
        sweep_default_options(&ox);
        ox.frame_mode = SWEEP_FRAME_FRENET;
        const double lk[8] = {0, 0, 0, 0.25, 0.5, 1, 1, 1};
        sweep_curve law{};
        law.n_ctrl = 5;
        law.degree = 2;
        law.ctrl = (const double*)dev_alloc(sizeof(double) * 3 * 5);
        law.knots = lk;
        ox.law = &law;
        const int64_t ex = sweep_batched_output_elems(&hx.b);
        const size_t wx = sweep_batched_workspace_size(&hx.b, &ox);
        for (int rep = 0; rep < 2; ++rep) {
            float* px = (float*)dev_alloc(sizeof(float) * ex);
            float* nx = (float*)dev_alloc(sizeof(float) * ex);
            void* wsx = dev_alloc(wx);
            bad += check(sweep_eval_batched(&hx.b, &ox, px, nx, wsx, wx, nullptr), "sweep_eval_batched (Frenet, law)");
            if (rep == 1) {
                double* gP = (double*)dev_alloc(sizeof(double) * 3 * 64);
                double* gQ = (double*)dev_alloc(sizeof(double) * 3 * 64);
                if (sweep_backward(&hx.b, &ox, px, gP, gQ, wsx, wx, nullptr) != SWEEP_ERR_UNSUPPORTED) ++bad;
                if (sweep_backward_workspace_size(&hx.b, &ox) != 0) ++bad;
            }
        }
    }
    {
        // arc-length and curvature-adaptive samples (the arc nodes of each
        // path degree before the frames; the one-wave and chunk-walking
        // frame kernels), polynomial and rational paths
        for (int rat = 0; rat < 2; ++rat)
        for (int mode = 1; mode <= 2; ++mode) {
            HostBatch ha;
            make_batch(ha, {3, 2, 5, 1, 3}, {200, 1500, 5000, 90, 33}, {40, 17, 9, 12, 8}, rat != 0, rng);
            sweep_options oa;
            sweep_default_options(&oa);
            oa.u_sampling = mode;
            oa.u_lambda = mode == 2 ? 0.5 : 0.0;
            const int64_t ea = sweep_batched_output_elems(&ha.b);
            const size_t wa = sweep_batched_workspace_size(&ha.b, &oa);
            for (int rep = 0; rep < 2; ++rep) {
                float* pa = (float*)dev_alloc(sizeof(float) * ea);
                float* na = (float*)dev_alloc(sizeof(float) * ea);
                void* wsa = dev_alloc(wa);
                bad += check(sweep_eval_batched(&ha.b, &oa, pa, na, wsa, wa, nullptr), "sweep_eval_batched (arc length)");
            }
            if (sweep_backward_workspace_size(&ha.b, &oa) != 0) ++bad;
        }
    }
    hipDeviceSynchronize();
    sweep_release_caches();
    std::printf("tuned config %d (%.3f ms), automatic config %d\n", cfg, ms, auto_cfg);
    const int v = stub::report(true);
    return v + bad + (cfg < 0 || auto_cfg != cfg ? 1 : 0);
}

void table()
{
    for (const stub::KernelSig* k : stub::all_kernels()) std::printf("%s %zu\n", k->name, k->args.size());
}

}  // namespace

int main(int argc, char** argv)
{
    const char* mode = argc > 1 ? argv[1] : "plans";
    if (!std::strcmp(mode, "selftest")) {
        selftest();
        return 0;
    }
    if (!std::strcmp(mode, "table")) {
        table();
        return 0;
    }
    if (!std::strcmp(mode, "tune")) return tune() == 0 ? 0 : 1;
    return plans() == 0 ? 0 : 1;
}
