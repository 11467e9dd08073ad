// hip_stub.cpp -- a CPU stand-in of the HIP runtime calls that the batched
// plan code (batched_abi.hip, host_checks.hip) makes, for checking that code
// on the host under AddressSanitizer.  "Device" memory is host memory from
// malloc, kernels are entries of a table with their argument sizes, and
// launches are recorded, not run.  The stand-in models asynchrony: a launch
// on a stream stays in flight until that stream, an event recorded after it,
// or the device is synchronised.  It counts as a violation (stub_report()):
//   * a kernel node or launch whose function is not a known kernel;
//   * a launch whose pointer argument is neither null (where the kernel
//     allows it) nor inside a live allocation;
//   * hipFree of memory that a launch still in flight uses;
//   * destroying a graph executable, or rewriting its node parameters,
//     while a launch of it is in flight;
//   * using a destroyed graph, graph executable or event.
// Reading each kernel argument through the caller's parameter array (the
// argument sizes come from the kernel table) also lets AddressSanitizer
// catch a parameter array that is too short or points at freed memory.
// Pointer arguments are checked when a kernel or graph is launched: graph
// nodes may hold placeholders until their parameters are set.
#include <hip/hip_runtime_api.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "stub_kernels.hpp"

namespace {

struct Launch {
    long long seq;                       // per-stream sequence number
    std::vector<const void*> ptrs;       // pointer arguments it reads or writes
    const void* exec;                    // graph executable, or null
};

struct Graph {
    std::vector<hipGraphNode_t> nodes;
};

struct Node {
    Graph* graph;
    const stub::KernelSig* sig;
    std::vector<std::vector<unsigned char>> args;
    const void* fn;
    unsigned grid;
};

struct Exec {
    std::vector<Node*> nodes;            // nodes of the graph it was made from
    std::map<Node*, std::vector<std::vector<unsigned char>>> args;  // its own copy
    bool live = true;
};

struct Event {
    hipStream_t stream = nullptr;
    long long seq = -1;
    bool live = true;
};

std::mutex g_mu;
std::map<uintptr_t, size_t> g_alloc;                  // live allocations
std::map<hipStream_t, long long> g_next_seq;          // next sequence number per stream
std::map<hipStream_t, std::vector<Launch>> g_pending; // launches in flight per stream
std::set<Graph*> g_graphs;
std::set<Node*> g_nodes;
std::set<Exec*> g_execs;
std::set<Event*> g_events;
std::map<std::string, int> g_violations;
long long g_launches = 0, g_graph_launches = 0, g_updates = 0, g_frees = 0;

void violation(const std::string& what)
{
    ++g_violations[what];
    if (g_violations[what] <= 3) std::fprintf(stderr, "[hip stub] violation: %s\n", what.c_str());
}

bool in_alloc(const void* p)
{
    const uintptr_t a = (uintptr_t)p;
    auto it = g_alloc.upper_bound(a);
    if (it == g_alloc.begin()) return false;
    --it;
    return a >= it->first && a < it->first + it->second;
}

bool ptr_in_alloc_range(const void* p, uintptr_t base, size_t n)
{
    const uintptr_t a = (uintptr_t)p;
    return a >= base && a < base + n;
}

// Copies every argument of `sig` out of `params` (sizes from the table).
std::vector<std::vector<unsigned char>> capture_args(const stub::KernelSig* sig, void** params)
{
    std::vector<std::vector<unsigned char>> out;
    for (size_t i = 0; i < sig->args.size(); ++i) {
        std::vector<unsigned char> bytes(sig->args[i].size);
        std::memcpy(bytes.data(), params[i], sig->args[i].size);
        out.push_back(std::move(bytes));
    }
    return out;
}

// Pointer arguments of a launch must be inside live allocations (or null
// where the kernel allows it).  Graph nodes may hold placeholders until
// their parameters are set, so this is checked when they are launched.
void check_launch_args(const stub::KernelSig* sig, const std::vector<std::vector<unsigned char>>& args)
{
    for (size_t i = 0; i < sig->args.size(); ++i) {
        const stub::ArgSig& a = sig->args[i];
        if (a.kind == stub::kValue) continue;
        const void* p;
        std::memcpy(&p, args[i].data(), sizeof p);
        if (!p) {
            if (a.kind == stub::kDevicePtr)
                violation(std::string(sig->name) + ": launched with a null device pointer argument " + std::to_string(i));
        } else if (!in_alloc(p)) {
            violation(std::string(sig->name) + ": launched with argument " + std::to_string(i) +
                      " outside every live allocation");
        }
    }
}

std::vector<const void*> pointer_args(const stub::KernelSig* sig, const std::vector<std::vector<unsigned char>>& args)
{
    std::vector<const void*> out;
    for (size_t i = 0; i < sig->args.size(); ++i) {
        if (sig->args[i].kind == stub::kValue) continue;
        const void* p;
        std::memcpy(&p, args[i].data(), sizeof p);
        if (p) out.push_back(p);
    }
    return out;
}

void complete_upto(hipStream_t s, long long seq)
{
    auto& v = g_pending[s];
    std::vector<Launch> keep;
    for (auto& l : v)
        if (l.seq > seq) keep.push_back(l);
    v.swap(keep);
}

bool exec_in_flight(const void* e)
{
    for (auto& kv : g_pending)
        for (auto& l : kv.second)
            if (l.exec == e) return true;
    return false;
}

void enqueue(hipStream_t s, Launch l)
{
    l.seq = g_next_seq[s]++;
    g_pending[s].push_back(std::move(l));
}

}  // namespace

extern "C" {

hipError_t hipMalloc(void** ptr, size_t size)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!ptr) return hipErrorInvalidValue;
    // 256-byte aligned like device allocations
    void* p = std::aligned_alloc(256, (size + 255) / 256 * 256 + (size ? 0 : 256));
    if (!p) return hipErrorOutOfMemory;
    g_alloc[(uintptr_t)p] = size ? size : 1;
    *ptr = p;
    return hipSuccess;
}

hipError_t hipFree(void* ptr)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!ptr) return hipSuccess;
    auto it = g_alloc.find((uintptr_t)ptr);
    if (it == g_alloc.end()) {
        violation("hipFree of a pointer that is not a live allocation");
        return hipErrorInvalidValue;
    }
    for (auto& kv : g_pending)
        for (auto& l : kv.second)
            for (const void* p : l.ptrs)
                if (ptr_in_alloc_range(p, it->first, it->second)) {
                    violation("hipFree of memory that a launch in flight uses");
                    goto done;
                }
done:
    g_alloc.erase(it);
    ++g_frees;
    std::free(ptr);
    return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind)
{
    std::memmove(dst, src, n);
    return hipSuccess;
}

hipError_t hipGetDevice(int* d)
{
    *d = 0;
    return hipSuccess;
}

const char* hipGetErrorString(hipError_t e)
{
    return e == hipSuccess ? "hipSuccess" : "hip stub error";
}

hipError_t hipDeviceSynchronize(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.clear();
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending[s].clear();
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Event* ev = new Event();
    g_events.insert(ev);
    *e = (hipEvent_t)ev;
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e)
{
    return hipEventCreateWithFlags(e, 0);
}

// timing events of the stand-in measure nothing
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Event* ea = (Event*)a;
    Event* eb = (Event*)b;
    if (!g_events.count(ea) || !ea->live || !g_events.count(eb) || !eb->live) {
        violation("hipEventElapsedTime on a destroyed event");
        return hipErrorInvalidValue;
    }
    *ms = 0.f;
    return hipSuccess;
}

hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int)
{
    std::memset(prop, 0, sizeof *prop);
    std::strcpy(prop->gcnArchName, "stub");
    prop->multiProcessorCount = 1;
    return hipSuccess;
}

hipError_t hipGetLastError(void)
{
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Event* ev = (Event*)e;
    if (!g_events.count(ev) || !ev->live) {
        violation("hipEventRecord on a destroyed event");
        return hipErrorInvalidValue;
    }
    ev->stream = s;
    ev->seq = g_next_seq[s] - 1;
    return hipSuccess;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Event* ev = (Event*)e;
    if (!g_events.count(ev) || !ev->live) {
        violation("hipEventSynchronize on a destroyed event");
        return hipErrorInvalidValue;
    }
    if (ev->seq >= 0) complete_upto(ev->stream, ev->seq);
    return hipSuccess;
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Event* ev = (Event*)e;
    if (!g_events.count(ev) || !ev->live) {
        violation("hipEventDestroy of a destroyed event");
        return hipErrorInvalidValue;
    }
    ev->live = false;
    return hipSuccess;
}

hipError_t hipGraphCreate(hipGraph_t* g, unsigned int)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Graph* gr = new Graph();
    g_graphs.insert(gr);
    *g = (hipGraph_t)gr;
    return hipSuccess;
}

hipError_t hipGraphAddKernelNode(hipGraphNode_t* node, hipGraph_t g, const hipGraphNode_t* deps, size_t ndeps,
                                 const hipKernelNodeParams* prm)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Graph* gr = (Graph*)g;
    if (!g_graphs.count(gr)) {
        violation("hipGraphAddKernelNode on a destroyed graph");
        return hipErrorInvalidValue;
    }
    for (size_t i = 0; i < ndeps; ++i) {
        Node* d = (Node*)deps[i];
        if (!g_nodes.count(d) || d->graph != gr) {
            violation("graph node dependency is not a node of the same graph");
            return hipErrorInvalidValue;
        }
    }
    if (prm->gridDim.x < 1 || prm->gridDim.y < 1 || prm->gridDim.z < 1 || prm->blockDim.x < 1 ||
        prm->blockDim.x > 1024 || prm->sharedMemBytes > 65536) {
        violation("graph kernel node with an invalid launch configuration");
        return hipErrorInvalidConfiguration;
    }
    const stub::KernelSig* sig = stub::lookup(prm->func);
    if (!sig) {
        violation("graph kernel node with an unknown function");
        return hipErrorInvalidDeviceFunction;
    }
    if (prm->extra) violation("graph kernel node with 'extra' arguments");
    Node* n = new Node{gr, sig, capture_args(sig, prm->kernelParams), prm->func, prm->gridDim.x};
    g_nodes.insert(n);
    gr->nodes.push_back((hipGraphNode_t)n);
    *node = (hipGraphNode_t)n;
    return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Graph* gr = (Graph*)g;
    if (!g_graphs.count(gr)) {
        violation("hipGraphInstantiate of a destroyed graph");
        return hipErrorInvalidValue;
    }
    Exec* ex = new Exec();
    for (hipGraphNode_t h : gr->nodes) {
        Node* n = (Node*)h;
        ex->nodes.push_back(n);
        ex->args[n] = n->args;
    }
    g_execs.insert(ex);
    *e = (hipGraphExec_t)ex;
    return hipSuccess;
}

hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t e, hipGraphNode_t node, const hipKernelNodeParams* prm)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Exec* ex = (Exec*)e;
    if (!g_execs.count(ex) || !ex->live) {
        violation("node parameters set on a destroyed graph executable");
        return hipErrorInvalidValue;
    }
    Node* n = (Node*)node;
    if (!ex->args.count(n)) {
        violation("node parameters set for a node that is not in the executable");
        return hipErrorInvalidValue;
    }
    if (stub::lookup(prm->func) != n->sig) {
        violation("node parameters change the node's function");
        return hipErrorInvalidValue;
    }
    if (exec_in_flight(ex)) violation("node parameters rewritten while a launch of the executable is in flight");
    ex->args[n] = capture_args(n->sig, prm->kernelParams);
    ++g_updates;
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Exec* ex = (Exec*)e;
    if (!g_execs.count(ex) || !ex->live) {
        violation("launch of a destroyed graph executable");
        return hipErrorInvalidValue;
    }
    Launch l{};
    l.exec = ex;
    for (Node* n : ex->nodes) {
        check_launch_args(n->sig, ex->args[n]);
        const std::string why = stub::check_work_list(n->fn, n->grid, ex->args[n]);
        if (!why.empty()) violation(std::string(n->sig->name) + ": " + why);
        for (const void* p : pointer_args(n->sig, ex->args[n])) l.ptrs.push_back(p);
    }
    enqueue(s, std::move(l));
    ++g_graph_launches;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t e)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Exec* ex = (Exec*)e;
    if (!g_execs.count(ex) || !ex->live) {
        violation("hipGraphExecDestroy of a destroyed executable");
        return hipErrorInvalidValue;
    }
    if (exec_in_flight(ex)) violation("graph executable destroyed while a launch of it is in flight");
    ex->live = false;
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Graph* gr = (Graph*)g;
    if (!g_graphs.count(gr)) {
        violation("hipGraphDestroy of a destroyed graph");
        return hipErrorInvalidValue;
    }
    for (hipGraphNode_t h : gr->nodes) g_nodes.erase((Node*)h);
    g_graphs.erase(gr);
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t lds, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (grid.x < 1 || grid.y < 1 || grid.z < 1 || block.x < 1 || block.x > 1024 || lds > 65536) {
        violation("launch with an invalid configuration");
        return hipErrorInvalidConfiguration;
    }
    const stub::KernelSig* sig = stub::lookup(f);
    if (!sig) {
        violation("launch of an unknown function");
        return hipErrorInvalidDeviceFunction;
    }
    Launch l{};
    l.exec = nullptr;
    const auto captured = capture_args(sig, args);
    check_launch_args(sig, captured);
    l.ptrs = pointer_args(sig, captured);
    enqueue(s, std::move(l));
    ++g_launches;
    return hipSuccess;
}

}  // extern "C"

namespace stub {

int report(bool print)
{
    std::lock_guard<std::mutex> lk(g_mu);
    int total = 0;
    for (auto& kv : g_violations) total += kv.second;
    if (print) {
        std::printf("launches %lld, graph launches %lld, parameter updates %lld, frees %lld, live allocations %zu\n",
                    g_launches, g_graph_launches, g_updates, g_frees, g_alloc.size());
        for (auto& kv : g_violations) std::printf("violation x%d: %s\n", kv.second, kv.first.c_str());
        std::printf("violations %d\n", total);
    }
    return total;
}

void reset_violations()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_violations.clear();
}

}  // namespace stub
