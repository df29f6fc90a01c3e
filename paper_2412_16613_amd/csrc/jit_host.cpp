// Per-network bit-sliced kernels compiled at run time with hipRTC.
//
// The general kernel (generic.hip) takes the reaction table as data, so it
// forms every weight kind in LDS and multiplies by each weight c_j bit by
// bit behind a run-time shift switch.  For a given network all of that is
// known before the first launch; this file writes the event loop of that
// network as source (weight kinds in registers, one compile-time shifted
// subtraction per set bit of c_j, the state change of each reaction as
// fixed mask updates, trailing reactions that change nothing left out since
// they cannot change which earlier reaction a lane selects) on top of the
// same device headers (in the one-wave-per-word and the producer/consumer
// forms), compiles it once per network and launches it through the module
// API.  It draws the same thresholds and computes the same first
// crossing as the general kernel, so results are identical.
//
// Frank-family networks whose product shift and unimolecular weight match
// no precompiled variant get the hand-written Frank kernels of wm_device.h
// compiled the same way, with those weights and the network's plane counts
// as template constants (per-replica and shared thresholds): the results are
// those of the precompiled run-time weight kernels, at the speed of the named
// workloads' kernels.

#include <hip/hiprtc.h>

#include <sstream>
#include <string>
#include <vector>

#include "host_internal.h"

namespace bwg {

extern const int kJitHeaderCount;
extern const char *const kJitHeaderNames[];
extern const char *const kJitHeaders[];

struct JitKernel {
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;  // one thread per word
    hipFunction_t pc = nullptr;  // producer/consumer form
    hipFunction_t sh = nullptr;  // Frank kernels: one shared threshold per event
    bool frank = false;          // the Frank-family kernel of wm_device.h
};

void jit_release(JitKernel *k)
{
    if (!k) return;
    if (k->mod) (void)hipModuleUnload(k->mod);
    delete k;
}

// threads per block of the one-wave-per-word kernels: 128 below 65 536
// words, 256 from there (measured 1.3-1.5x on general networks at 2^21 and
// 2^22 replicas; 128-thread blocks are placed unevenly there), as for the
// precompiled Frank kernels
constexpr int kJitBlockSmall = 128, kJitBlockLarge = 256;
// Events per ring half of the producer/consumer kernels: the ring holds
// 2 x 2 x PH events of BC planes for 128 words (BC KiB per event pair), so
// beyond 32 threshold planes it takes 2 to stay within the CU's LDS.
static int jit_pc_half(int BC) { return BC > 32 ? 2 : 4; }

// Source of network n's kernels with NB count planes and BC threshold planes:
// an event functor (weight kinds kept from event to event, selection, state
// change) and the two word loops of gen_device.h around it.
static std::string jit_source(const bwg_net &n, int NB, int BC)
{
    const GenNet &g = n.gen;
    static const char *const kPair[3][2] = {{"N[0]", "N[1]"}, {"N[0]", "N[2]"}, {"N[1]", "N[2]"}};
    // reactions that matter: up to the last one that changes the state
    int R = g.R;
    while (R > 0 && !((g.change >> (R - 1)) & 1u)) --R;
    uint32_t used = 0;
    for (int j = 0; j < R; ++j)
        if (g.c[j]) used |= 1u << g.kind[j];
    int last_j = -1, last_bit = -1;  // the final subtraction need not keep d
    for (int j = 0; j < R; ++j)
        if (g.c[j]) {
            last_j = j;
            last_bit = 31 - __builtin_clz(g.c[j]);
        }
    std::ostringstream o;
    o << "#include \"gen_device.h\"\n"
      << "namespace bwg {\n"
      << "constexpr int NB = " << NB << ", BC = " << BC << ", WH = 2 * NB;\n"
      << "struct NetEvent {\n";
    // pair counts and X (X - 1) / 2 the reactions use: formed once per launch,
    // then updated from each event's changes (App. B, for changes in -2..2)
    for (int k = 3; k < 9; ++k)
        if ((used >> k) & 1u) o << "    uint32_t h" << k << "[WH];\n";
    o << "    __device__ __forceinline__ void init(const uint32_t (&N)[3][NB])\n"
      << "    {\n";
    for (int k = 3; k < 9; ++k) {
        if (!((used >> k) & 1u)) continue;
        if (k < 6) {
            o << "        mul_planes<NB, WH>(h" << k << ", " << kPair[k - 3][0] << ", "
              << kPair[k - 3][1] << ");\n";
        } else {
            const int x = k - 6;
            o << "        {\n"
              << "            uint32_t xm[NB], p[WH];\n"
              << "#pragma unroll\n"
              << "            for (int q = 0; q < NB; ++q) xm[q] = N[" << x << "][q];\n"
              << "            add_pm1<NB>(xm, 0u, ~0u);\n"
              << "            mul_planes<NB, WH>(p, N[" << x << "], xm);\n"
              << "#pragma unroll\n"
              << "            for (int q = 0; q < WH; ++q) h" << k
              << "[q] = q + 1 < WH ? p[q + 1] : 0u;\n"
              << "        }\n";
        }
    }
    o << "    }\n"
      << "    __device__ __forceinline__ void operator()(uint32_t (&d)[BC], uint32_t act,\n"
      << "                                               uint32_t (&N)[3][NB], uint64_t &nreal)\n"
      << "    {\n";
    o << "        uint32_t lt = 0, realm = 0;\n"
      << "        uint32_t mk[3][4] = {};\n";
    static const int kSlot[5] = {3, 1, -1, 0, 2};  // delta -2..2 -> mask index
    for (int j = 0; j < R; ++j) {
        if (!g.c[j]) continue;  // weight 0: never selected
        const int k = g.kind[j];
        const std::string op =
            k < 3 ? ("N[" + std::to_string(k) + "]") : ("h" + std::to_string(k));
        const char *wp = k < 3 ? "NB" : "WH";
        o << "        {  // reaction " << j << "\n"
          << "            uint32_t br = 0;\n";
        for (int b = 0; b < 32; ++b) {
            if (!((g.c[j] >> b) & 1u)) continue;
            const bool keep = !(j == last_j && b == last_bit);
            o << "            br |= sub_shifted<" << b << ", BC, " << wp << ", "
              << (keep ? "true" : "false") << ">(d, " << op << ");\n";
        }
        o << "            const uint32_t ltj = lt | br;\n"
          << "            const uint32_t xi = ltj & ~lt & act;\n"
          << "            lt = ltj;\n";
        if ((g.change >> j) & 1u) o << "            realm |= xi;\n";
        for (int x = 0; x < 3; ++x) {
            const int dv = g.d[j][x];
            if (dv) o << "            mk[" << x << "][" << kSlot[dv + 2] << "] |= xi;\n";
        }
        o << "        }\n";
    }
    o << "        nreal += (uint32_t)__builtin_popcount(realm);\n";
    // species in order: a pair count takes the change of x times the other
    // species' current count (before that one's own change if it comes
    // later, after it if earlier: X'Y' - XY = dX Y + dY X'), X (X - 1) / 2
    // takes dX X + dX (dX - 1) / 2; then the count itself changes
    static const int kPairOf[3][3] = {{-1, 3, 4}, {3, -1, 5}, {4, 5, -1}};
    for (int x = 0; x < 3; ++x) {
        bool any = false;
        for (int j = 0; j < R; ++j) any |= g.c[j] && g.d[j][x];
        if (!any) continue;
        const std::string X = std::to_string(x);
        const std::string m = "mk[" + X + "][0], mk[" + X + "][1], mk[" + X + "][2], mk[" + X + "][3]";
        for (int y = 0; y < 3; ++y) {
            const int k = kPairOf[x][y];
            if (k >= 0 && ((used >> k) & 1u))
                o << "        add_scaled<NB, WH>(h" << k << ", N[" << y << "], " << m << ");\n";
        }
        if ((used >> (6 + x)) & 1u)
            o << "        add_scaled<NB, WH>(h" << 6 + x << ", N[" << x << "], " << m << ");\n"
              << "        add_one_three<WH>(h" << 6 + x << ", mk[" << x << "][1] | mk[" << x
              << "][2], mk[" << x << "][3]);\n";
        o << "        add_delta<NB>(N[" << x << "], " << m << ");\n";
    }
    o << "    }\n"
      << "};\n"
      << "extern \"C\" __global__ __launch_bounds__(" << kJitBlockLarge
      << ") void bwg_jit_word(WmArgs a)\n"
      << "{\n"
      << "    gen_word<NB, BC>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, NetEvent{});\n"
      << "}\n"
      << "extern \"C\" __global__ __launch_bounds__(256) void bwg_jit_pc(WmArgs a)\n"
      << "{\n"
      << "    constexpr int PH = " << jit_pc_half(BC) << ";\n"
      << "    __shared__ uint4 ring[2 * 2 * PH][BC / 4][64];\n"
      << "    __shared__ uint64_t wave_span[4];\n"
      << "    gen_word_pc<NB, BC, PH>(a, ring, wave_span, NetEvent{});\n"
      << "}\n"
      << "}  // namespace bwg\n";
    return o.str();
}

// Source of the kernels of a network of S species (any S up to 8) or an open
// network (counts capped at n_tot): the same structure as jit_source with
// the weight kinds of S species -- N_X, the pair counts N_X N_Y (x < y) and
// N_X (N_X - 1) / 2 -- and, for an open network, each reaction's selected
// lanes cleared where a count it raises by dv would pass the cap (count >=
// cap - dv + 1 before the event): the oracle's blocked firing.
static std::string jit_source_wide(const bwg_net &n, int NB, int BC)
{
    const int S = n.S, R0 = n.R;
    auto dv = [&](int j, int x) { return n.prod[j * S + x] - n.reac[j * S + x]; };
    auto changes = [&](int j) {
        for (int x = 0; x < S; ++x)
            if (dv(j, x)) return true;
        return false;
    };
    int R = R0;
    while (R > 0 && !changes(R - 1)) --R;
    // weight operand of each reaction: species x (unimolecular), pair (x, y)
    // or dimer x
    std::vector<std::string> opnd(R);
    std::vector<bool> wide_op(R);
    bool pair_used[8][8] = {}, dimer_used[8] = {};
    for (int j = 0; j < R; ++j) {
        int xs[2], k = 0;
        for (int x = 0; x < S; ++x)
            for (int m = 0; m < n.reac[j * S + x]; ++m) xs[k++] = x;
        if (k == 1) {
            opnd[j] = "N[" + std::to_string(xs[0]) + "]";
            wide_op[j] = false;
        } else if (xs[0] != xs[1]) {
            opnd[j] = "hp" + std::to_string(xs[0]) + std::to_string(xs[1]);
            wide_op[j] = true;
            if (n.q.c[j]) pair_used[xs[0]][xs[1]] = true;
        } else {
            opnd[j] = "hd" + std::to_string(xs[0]);
            wide_op[j] = true;
            if (n.q.c[j]) dimer_used[xs[0]] = true;
        }
    }
    int last_j = -1, last_bit = -1;
    for (int j = 0; j < R; ++j)
        if (n.q.c[j]) {
            last_j = j;
            last_bit = 63 - __builtin_clzll((uint64_t)n.q.c[j]);
        }
    std::ostringstream o;
    o << "#include \"gen_device.h\"\n"
      << "namespace bwg {\n"
      << "constexpr int NB = " << NB << ", BC = " << BC << ", S = " << S << ", WH = 2 * NB;\n"
      << "struct NetEvent {\n";
    for (int x = 0; x < S; ++x)
        for (int y = x + 1; y < S; ++y)
            if (pair_used[x][y]) o << "    uint32_t hp" << x << y << "[WH];\n";
    for (int x = 0; x < S; ++x)
        if (dimer_used[x]) o << "    uint32_t hd" << x << "[WH];\n";
    o << "    __device__ __forceinline__ void init(const uint32_t (&N)[S][NB])\n"
      << "    {\n";
    for (int x = 0; x < S; ++x)
        for (int y = x + 1; y < S; ++y)
            if (pair_used[x][y])
                o << "        mul_planes<NB, WH>(hp" << x << y << ", N[" << x << "], N[" << y << "]);\n";
    for (int x = 0; x < S; ++x) {
        if (!dimer_used[x]) continue;
        o << "        {\n"
          << "            uint32_t xm[NB], p[WH];\n"
          << "#pragma unroll\n"
          << "            for (int q = 0; q < NB; ++q) xm[q] = N[" << x << "][q];\n"
          << "            add_pm1<NB>(xm, 0u, ~0u);\n"
          << "            mul_planes<NB, WH>(p, N[" << x << "], xm);\n"
          << "#pragma unroll\n"
          << "            for (int q = 0; q < WH; ++q) hd" << x << "[q] = q + 1 < WH ? p[q + 1] : 0u;\n"
          << "        }\n";
    }
    o << "    }\n"
      << "    __device__ __forceinline__ void operator()(uint32_t (&d)[BC], uint32_t act,\n"
      << "                                               uint32_t (&N)[S][NB], uint64_t &nreal)\n"
      << "    {\n"
      << "        uint32_t lt = 0, realm = 0;\n"
      << "        uint32_t mk[S][4] = {};\n";
    static const int kSlot[5] = {3, 1, -1, 0, 2};  // change -2..2 -> mask index
    for (int j = 0; j < R; ++j) {
        const uint64_t c = (uint64_t)n.q.c[j];
        if (!c) continue;  // weight 0: never selected
        o << "        {  // reaction " << j << "\n"
          << "            uint32_t br = 0;\n";
        for (int b = 0; b < 32; ++b) {
            if (!((c >> b) & 1u)) continue;
            const bool keep = !(j == last_j && b == last_bit);
            o << "            br |= sub_shifted<" << b << ", BC, " << (wide_op[j] ? "WH" : "NB")
              << ", " << (keep ? "true" : "false") << ">(d, " << opnd[j] << ");\n";
        }
        o << "            const uint32_t ltj = lt | br;\n"
          << "            uint32_t xi = ltj & ~lt & act;\n"
          << "            lt = ltj;\n";
        if (n.open) {
            for (int x = 0; x < S; ++x)
                if (dv(j, x) > 0)
                    o << "            xi &= ~geq_const<NB, " << (n.n_tot - dv(j, x) + 1) << "u>(N[" << x
                      << "]);\n";
        }
        if (changes(j)) o << "            realm |= xi;\n";
        for (int x = 0; x < S; ++x)
            if (dv(j, x)) o << "            mk[" << x << "][" << kSlot[dv(j, x) + 2] << "] |= xi;\n";
        o << "        }\n";
    }
    o << "        nreal += (uint32_t)__builtin_popcount(realm);\n";
    // species in order: each pair count takes the change of x times the
    // other species' current count (X'Y' - XY = dX Y + dY X'), X (X - 1) / 2
    // takes dX X + dX (dX - 1) / 2; then the count itself changes
    for (int x = 0; x < S; ++x) {
        bool any = false;
        for (int j = 0; j < R; ++j) any |= n.q.c[j] && dv(j, x);
        if (!any) continue;
        const std::string X = std::to_string(x);
        const std::string m = "mk[" + X + "][0], mk[" + X + "][1], mk[" + X + "][2], mk[" + X + "][3]";
        for (int y = 0; y < S; ++y) {
            if (y == x) continue;
            const int a = x < y ? x : y, b = x < y ? y : x;
            if (pair_used[a][b])
                o << "        add_scaled<NB, WH>(hp" << a << b << ", N[" << y << "], " << m << ");\n";
        }
        if (dimer_used[x])
            o << "        add_scaled<NB, WH>(hd" << x << ", N[" << x << "], " << m << ");\n"
              << "        add_one_three<WH>(hd" << x << ", mk[" << x << "][1] | mk[" << x
              << "][2], mk[" << x << "][3]);\n";
        o << "        add_delta<NB>(N[" << x << "], " << m << ");\n";
    }
    o << "    }\n"
      << "};\n"
      << "extern \"C\" __global__ __launch_bounds__(" << kJitBlockLarge
      << ") void bwg_jit_word(WmArgs a)\n"
      << "{\n"
      << "    gen_word<NB, BC, S>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, NetEvent{});\n"
      << "}\n"
      << "extern \"C\" __global__ __launch_bounds__(256) void bwg_jit_pc(WmArgs a)\n"
      << "{\n"
      << "    constexpr int PH = " << jit_pc_half(BC) << ";\n"
      << "    __shared__ uint4 ring[2 * 2 * PH][BC / 4][64];\n"
      << "    __shared__ uint64_t wave_span[4];\n"
      << "    gen_word_pc<NB, BC, PH, S>(a, ring, wave_span, NetEvent{});\n"
      << "}\n"
      << "}  // namespace bwg\n";
    return o.str();
}

// Compiles src with hipRTC for gfx950 into a code object: host work only,
// no device needed.
static int jit_build(const std::string &src, std::vector<char> *code)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "bwg_jit_word.hip", kJitHeaderCount, kJitHeaders,
                            kJitHeaderNames) != HIPRTC_SUCCESS)
        return fail(BWG_EDEVICE, "hiprtcCreateProgram failed");
    // no packed-fp32 instructions in device code, as for the precompiled kernels
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang",
                          "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, 7, opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(BWG_EDEVICE, "run-time compile of the network's kernel failed: %.400s",
                    log.c_str());
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    code->assign(cs, 0);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return BWG_OK;
}

// Loads a code object's kernels (one wave per word and producer/consumer;
// for the Frank kernels also the shared-threshold instantiation) onto the
// current device.
static int jit_load(const std::vector<char> &code, bool frank, JitKernel **out)
{
    auto k = new JitKernel();
    k->frank = frank;
    hipError_t e = hipModuleLoadData(&k->mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&k->fn, k->mod, "bwg_jit_word");
    if (e == hipSuccess) e = hipModuleGetFunction(&k->pc, k->mod, "bwg_jit_pc");
    if (e == hipSuccess && frank) e = hipModuleGetFunction(&k->sh, k->mod, "bwg_jit_sh");
    if (e != hipSuccess) {
        jit_release(k);
        return fail(BWG_EDEVICE, "loading the network's kernel: %s", hipGetErrorString(e));
    }
    *out = k;
    return BWG_OK;
}

// Code object of network n's general kernel, built once (caller holds the
// network's lock).
static int jit_general_code(bwg_net *n)
{
    if (!n->jit_code.empty()) return BWG_OK;
    if (!n->gen_ok && !n->wide_ok)
        return fail(BWG_EUNSUPPORTED, "no general reaction table for this network");
    const int need_bc = n->q.B + (n->q.max_total == (1ll << n->q.B) ? 1 : 0);
    const int NB = n->q.b, BC = (need_bc + 3) / 4 * 4;
    if (BC > kMaxThresholdPlanes || NB > 14)
        return fail(BWG_EUNSUPPORTED, "network beyond 14 count / %d threshold planes",
                    kMaxThresholdPlanes);
    return jit_build(n->wide ? jit_source_wide(*n, NB, BC) : jit_source(*n, NB, BC),
                     &n->jit_code);
}

// The compiled kernel of network n, built and loaded on the first call
// (under the network's lock).
int jit_get(bwg_net *n, const JitKernel **out)
{
    std::lock_guard<std::mutex> lock(n->mu);
    if (n->jit) {
        *out = n->jit;
        return BWG_OK;
    }
    int rc = jit_general_code(n);
    if (rc) return rc;
    JitKernel *k = nullptr;
    rc = jit_load(n->jit_code, false, &k);
    if (rc) return rc;
    n->jit = k;
    *out = k;
    return BWG_OK;
}

// Source of the Frank-family kernels of wm_device.h for a network with its
// count and threshold planes, product shifts and unimolecular weight as
// compile-time constants (the precompiled kernels take them at run time
// unless the network is one of the named workloads): FA shifts the A + L and
// A + D weights, FI the L + D weight; with the molecule count NT and the
// selection planes BS the registers take their exact widths (WmShape).
static std::string jit_frank_source(int NB, int BC, int FA, int FI, int CU, int NT, int BS)
{
    std::ostringstream o;
    o << "#include \"wm_device.h\"\n"
      << "namespace bwg {\n"
      << "constexpr int NB = " << NB << ", BC = " << BC << ", FA = " << FA << ", FI = " << FI
      << ", CU = " << CU << ", NT = " << NT << ", BS = " << BS << ";\n"
      << "extern \"C\" __global__ __launch_bounds__(256) void bwg_jit_word(WmArgs a)\n"
      << "{\n"
      << "    wm_word<NB, BC, FA, CU, false, FI, NT, BS>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);\n"
      << "}\n"
      << "extern \"C\" __global__ __launch_bounds__(256) void bwg_jit_sh(WmArgs a)\n"
      << "{\n"
      << "    wm_word<NB, BC, FA, CU, true, FI, NT, BS>(a, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);\n"
      << "}\n"
      << "extern \"C\" __global__ __launch_bounds__(256) void bwg_jit_pc(WmArgs a)\n"
      << "{\n"
      << "    constexpr int PH = BC > 32 ? 2 : (BC == 20 ? 6 : 4);\n"
      << "    __shared__ uint4 ring[2 * 2 * PH][BC / 4][64];\n"
      << "    __shared__ uint64_t wave_span[4];\n"
      << "    wm_word_pc<NB, BC, FA, CU, PH, FI, NT, BS>(a, ring, wave_span);\n"
      << "}\n"
      << "}  // namespace bwg\n";
    return o.str();
}

// Template parameters of network n's compiled Frank kernel: count planes,
// threshold planes (whole Philox quads), the two product shifts (A + L and
// A + D; L + D), unimolecular weight.  A shift whose reactions are absent
// takes the other one's value (its subtraction is never run).
struct FrankParams {
    int NB, BC, FA, FI, CU, NT, BS;
};

static bool frank_params(const bwg_net &n, FrankParams *p)
{
    if (!n.shape_ok) return false;
    const int need_bc = n.q.B + (n.q.max_total == (1ll << n.q.B) ? 1 : 0);
    const int NB = n.q.b, BC = (need_bc + 3) / 4 * 4;
    const int fa = n.shape.fa, fi = n.shape.fi;
    const int FA = fa >= 0 ? fa : (fi >= 0 ? fi : 0);
    const int FI = fi >= 0 ? fi : FA;
    if (BC > kMaxThresholdPlanes || NB > 14 || NB < 1 || FA >= BC || FI >= BC ||
        n.shape.cu > 0x7FFFFFFFu)
        return false;
    if (n.n_tot < 1 || n.n_tot >= (1 << 14)) return false;
    // exact register widths need the molecule count and both bimolecular
    // kinds (A + L / A + D and L + D); NT = 0 keeps the general widths
    const int NT = (fa >= 0 && fi >= 0) ? (int)n.n_tot : 0;
    *p = FrankParams{NB, BC, FA, FI, (int)n.shape.cu, NT, need_bc};
    return true;
}

bool jit_frank_fits(const bwg_net *n)
{
    FrankParams p;
    return frank_params(*n, &p);
}

// Code object of network n's Frank-family kernel, built once (caller holds
// the network's lock); BWG_EUNSUPPORTED where the network's planes or
// weights do not fit the kernel's template parameters.
static int jit_frank_code(bwg_net *n)
{
    if (!n->jit_frank_code.empty()) return BWG_OK;
    FrankParams p;
    if (!frank_params(*n, &p))
        return fail(BWG_EUNSUPPORTED, "network beyond the compiled Frank kernel's range");
    return jit_build(jit_frank_source(p.NB, p.BC, p.FA, p.FI, p.CU, p.NT, p.BS),
                     &n->jit_frank_code);
}

// The compiled Frank-family kernel of network n (first call builds and
// loads it, under the network's lock).
int jit_frank_get(bwg_net *n, const JitKernel **out)
{
    std::lock_guard<std::mutex> lock(n->mu);
    if (n->jit_frank) {
        *out = n->jit_frank;
        return BWG_OK;
    }
    int rc = jit_frank_code(n);
    if (rc) return rc;
    JitKernel *k = nullptr;
    rc = jit_load(n->jit_frank_code, true, &k);
    if (rc) return rc;
    n->jit_frank = k;
    *out = k;
    return BWG_OK;
}

int jit_build_codes(bwg_net *n, bool general, bool frank)
{
    std::lock_guard<std::mutex> lock(n->mu);
    int rc = general ? jit_general_code(n) : BWG_OK;
    if (!rc && frank) rc = jit_frank_code(n);
    return rc;
}

hipError_t jit_launch(const JitKernel *k, const WmArgs &a, hipStream_t s)
{
    WmArgs arg = a;
    void *params[] = {&arg};
    if (a.zs) {
        // shared thresholds (Frank kernels only): one wave per word, the
        // block sizes of the precompiled shared-threshold kernels
        if (!k->sh) return hipErrorInvalidValue;
        const unsigned block = a.n_words >= 65536 ? 256u : 128u;
        const unsigned grid = (unsigned)((a.n_words + block - 1) / block);
        return hipModuleLaunchKernel(k->sh, grid, 1, 1, block, 1, 1, 0, s, params, nullptr);
    }
    // as for the Frank kernels: the producer/consumer form while the words
    // fill at most one wave per SIMD pair
    if (a.n_words <= 32768) {
        const unsigned grid = (unsigned)((a.n_words + 127) / 128);
        return hipModuleLaunchKernel(k->pc, grid, 1, 1, 256, 1, 1, 0, s, params, nullptr);
    }
    const unsigned block =
        (unsigned)(a.n_words >= 65536 ? kJitBlockLarge : kJitBlockSmall);
    const unsigned grid = (unsigned)((a.n_words + block - 1) / block);
    return hipModuleLaunchKernel(k->fn, grid, 1, 1, block, 1, 1, 0, s, params, nullptr);
}

}  // namespace bwg
