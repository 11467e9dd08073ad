// stub_kernels.cpp -- the kernel table of the CPU stand-in (parameter lists
// of the batched and adjoint kernels, in the order the kernels declare them)
// and stand-ins of the plan code's kernel-table and fast-division helpers.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <string>

#include "../../paper_1110_5450_amd/csrc/kernels.hpp"
#include "stub_kernels.hpp"

namespace stub {
namespace {

constexpr ArgSig P{sizeof(void*), kDevicePtr};
constexpr ArgSig N{sizeof(void*), kNullablePtr};
constexpr ArgSig I{sizeof(int), kValue};
constexpr ArgSig N0{sizeof(sweep::InitialNormal), kValue};
constexpr ArgSig FX{sizeof(sweep::BatchFrameExt), kValue};
constexpr ArgSig D{sizeof(double), kValue};

const KernelSig kProfile{"kb_profile", {P, P, P, N, N, P}};
const KernelSig kFrame{"kb_frame", {P, P, P, N, N, N0, I, P, FX}};
const KernelSig kFrameLong{"kb_frame_long", {P, P, P, N, N, N0, I, P, FX}};
const KernelSig kFrameWave{"kb_frame_wave", {P, P, P, N, N, N0, I, P, FX}};
const KernelSig kArcPieces{"kb_arc_pieces", {P, P, P, N, N, D, P}};
const KernelSig kArcCumsum{"kb_arc_cumsum", {P, P, P}};
const KernelSig kArcParams{"kb_arc_params", {P, P, P, N, N, D, P, P, P}};
const KernelSig kSurface{"kb_surface", {P, P, P, P, P, N}};
const KernelSig kReduce{"kbw_reduce", {P, P, I, N, N, P, P, P, P}};
const KernelSig kRows{"kbw_rows", {P, P, P, N, N, P, P, P, P, P, I}};
const KernelSig kSamples{"kbw_samples", {P, P, P, N, N, N0, P, P, P, P, P, P, I, N}};
const KernelSig kFinal{"kbw_final", {P, P, P, N, N, N, P, P, P, P, P, P, P, P, I}};
const KernelSig kParamRec{"kbw_param_rec", {P, P, P, P, N, N, N, N, P, P, P, P, P, I, I, I}};
const KernelSig kParams{"kbw_params", {P, P, P, N, N, N, P, P, P, P, N, N, N, N}};

// distinct addresses standing in for kernel entry points
char g_profile, g_frame[8], g_frame_long[8], g_frame_wave[8], g_arc_pieces[8], g_arc_cumsum, g_arc_params[8], g_surface, g_reduce, g_rows, g_samples, g_final, g_rec_path, g_rec_prof, g_params;

const std::map<const void*, const KernelSig*>& table()
{
    static const std::map<const void*, const KernelSig*> t = [] {
        std::map<const void*, const KernelSig*> m;
        m[&g_profile] = &kProfile;
        for (int p = 1; p < 8; ++p) m[&g_frame[p]] = &kFrame;
        for (int p = 1; p < 8; ++p) m[&g_frame_long[p]] = &kFrameLong;
        for (int p = 1; p < 8; ++p) m[&g_frame_wave[p]] = &kFrameWave;
        for (int p = 1; p < 8; ++p) m[&g_arc_pieces[p]] = &kArcPieces;
        m[&g_arc_cumsum] = &kArcCumsum;
        for (int p = 1; p < 8; ++p) m[&g_arc_params[p]] = &kArcParams;
        m[&g_surface] = &kSurface;
        m[&g_reduce] = &kReduce;
        m[&g_rows] = &kRows;
        m[&g_samples] = &kSamples;
        m[&g_final] = &kFinal;
        m[&g_rec_path] = &kParamRec;
        m[&g_rec_prof] = &kParamRec;
        m[&g_params] = &kParams;
        return m;
    }();
    return t;
}

}  // namespace

const KernelSig* lookup(const void* fn)
{
    auto it = table().find(fn);
    return it == table().end() ? nullptr : it->second;
}

std::string check_work_list(const void* fn, unsigned grid, const std::vector<std::vector<unsigned char>>& args)
{
    int deg = 0;
    bool pieces = false;
    for (int p = 1; p < 8; ++p) {
        if (fn == &g_arc_pieces[p]) deg = p, pieces = true;
        if (fn == &g_arc_params[p]) deg = p;
    }
    if (!deg) return "";
    const sweep::BatchDesc* descs;
    const int2* chunks;
    std::memcpy(&descs, args[0].data(), sizeof descs);
    std::memcpy(&chunks, args[1].data(), sizeof chunks);
    for (unsigned b = 0; b < grid; ++b) {
        const sweep::BatchDesc& d = descs[chunks[b].x];
        if (d.p_path != deg)
            return "block " + std::to_string(b) + " of the degree-" + std::to_string(deg) + " launch names a sweep of degree " +
                   std::to_string(d.p_path);
        const int lim = pieces ? d.n_path - deg : d.n_u;
        if (chunks[b].y < 0 || chunks[b].y >= lim)
            return "block " + std::to_string(b) + " starts at index " + std::to_string(chunks[b].y) + " of " +
                   std::to_string(lim);
    }
    return "";
}

std::vector<const KernelSig*> all_kernels()
{
    return {&kProfile, &kFrame, &kFrameLong, &kFrameWave, &kArcPieces, &kArcCumsum, &kArcParams, &kSurface, &kReduce, &kRows, &kSamples, &kFinal, &kParamRec, &kParams};
}

}  // namespace stub

namespace sweep {

BatchedKernels batched_kernels(bool, bool, bool, bool, int, bool, bool, bool, bool)
{
    BatchedKernels k{};
    k.profile = &stub::g_profile;
    k.frame[0] = nullptr;
    k.frame_long[0] = nullptr;
    k.frame_wave[0] = nullptr;
    for (int p = 1; p < 8; ++p) k.frame[p] = &stub::g_frame[p];
    for (int p = 1; p < 8; ++p) k.frame_long[p] = &stub::g_frame_long[p];
    for (int p = 1; p < 8; ++p) k.frame_wave[p] = &stub::g_frame_wave[p];
    k.arc_pieces[0] = k.arc_params[0] = nullptr;
    for (int p = 1; p < 8; ++p) k.arc_pieces[p] = &stub::g_arc_pieces[p];
    k.arc_cumsum = &stub::g_arc_cumsum;
    for (int p = 1; p < 8; ++p) k.arc_params[p] = &stub::g_arc_params[p];
    k.surface = &stub::g_surface;
    return k;
}

BackwardKernels backward_kernels(bool, bool)
{
    return BackwardKernels{&stub::g_reduce, &stub::g_rows, &stub::g_samples, &stub::g_final, &stub::g_params,
                           &stub::g_rec_path, &stub::g_rec_prof};
}

void fastdiv_constants(int d, unsigned long long* m, int* shift)
{
    *m = (unsigned long long)d;
    *shift = 0;
}

}  // namespace sweep
