// Scoring network: creation (BatchNorm folding, precision conversion, device
// layouts), execution plan and the af_score_windows entry point.
#include <algorithm>
#include <cfenv>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fused_tiny.h"
#include "gn_kernels.h"
#include "internal.h"

using namespace afm;

namespace {

using LaunchFn = void (*)(const ConvArgs&, hipStream_t);

// Tile geometry of one conv kernel instantiation, needed on the host to lay out
// the weight image and to size the grid.
struct ConvCfg {
    LaunchFn fn = nullptr;
    int MT = 0, NT = 0, KC = 0, KWP = 0, WMAX = 1;
    int PB = 0;   // weight row pitch in the image (elements)
    int KL = 1;   // k values per lane per MFMA (swizzle unit)
    int SWR = 0;  // rows per swizzle step (0: no swizzle)
};

template <typename P, int KW, int S, int WM, int WN, int TM, int TN, int KC, int WMAX, int DB, bool TS>
void launch_conv(const ConvArgs& a, hipStream_t s) {
    constexpr int NT = WN * TN * 16;
    ConvArgs b = a;
    b.n_mtiles = a.wpt == 1 ? a.n_win * a.tiles_per_win : (a.n_win + a.wpt - 1) / a.wpt;
    const unsigned per_xcd = (unsigned)(b.n_mtiles + 7) / 8;   // the kernel's XCD-ordered grid
    hipLaunchKernelGGL((conv_mfma_kernel<P, KW, S, WM, WN, TM, TN, KC, WMAX, DB, TS>),
                       dim3(8 * per_xcd * (unsigned)(a.C_out / NT)), dim3(64 * WM * WN), 0, s, b);
}

// DB: the kernel's staging mode (0, 1 or 2; see conv_mfma_kernel).  TS: allow
// the tap-shift A-operand reuse where the kernel supports it.
template <typename P, int KW, int S, int WM, int WN, int TM, int TN, int KC, int WMAX, int DB, bool TS = true>
ConvCfg make_cfg() {
    ConvCfg c;
    c.fn = launch_conv<P, KW, S, WM, WN, TM, TN, KC, WMAX, DB, TS>;
    c.MT = WM * TM * 16;
    c.NT = WN * TN * 16;
    c.KC = KC;
    c.KWP = ChunkGeom<KW, KC, 4 * P::KL>::KWP;
    c.WMAX = WMAX;
    constexpr int OPB = (int)sizeof(typename P::Op);
    c.PB = OPB == 4 ? KC + 4 : (P::KL == 32 ? KC + 16 : KC);   // these three must match the kernel's PB, KL, SWR
    c.KL = P::KL;
    c.SWR = weight_swizzle_rows<OPB, KC>();
    return c;
}

using Cands = std::vector<ConvCfg>;

// Candidate tile shapes per layer class; the first is the default, the
// autotuner (af_net_autotune) may pick another by timing.
// FP32: 16-channel chunks, single LDS buffer (two workgroups per CU overlap
// staging with compute).
template <int KW, int S, typename P = PF32>
Cands cands_f32(int c_out) {
    if (c_out % 128 == 0)
        return {make_cfg<P, KW, S, 2, 2, 3, 4, 16, 1, false>(), make_cfg<P, KW, S, 2, 2, 6, 2, 16, 2, false>(),
                make_cfg<P, KW, S, 2, 2, 2, 4, 16, 1, false>(), make_cfg<P, KW, S, 2, 2, 6, 2, 16, 2, 2>(),
                make_cfg<P, KW, S, 4, 1, 3, 4, 16, 2, 0>(), make_cfg<P, KW, S, 4, 1, 3, 4, 16, 2, 2>()};
    if (c_out == 64)
        return {make_cfg<P, KW, S, 2, 2, 3, 2, 16, 1, false>(), make_cfg<P, KW, S, 4, 1, 3, 4, 16, 1, false>(),
                make_cfg<P, KW, S, 2, 2, 2, 2, 16, 1, false>(), make_cfg<P, KW, S, 2, 2, 6, 2, 16, 2, 2>(),
                make_cfg<P, KW, S, 4, 1, 3, 4, 16, 2, 2>()};
    if constexpr ((KW == 7 || KW == 3) && S == 1) {
        if (c_out == 32)
            return {make_cfg<P, KW, 1, 4, 1, 3, 2, 16, 1, false>(), make_cfg<P, KW, 1, 4, 1, 2, 2, 16, 1, false>(),
                    make_cfg<P, KW, 1, 2, 2, 6, 1, 16, 1, false>()};
        if (KW == 7 && c_out == 16)
            return {make_cfg<P, 7, 1, 4, 1, 4, 1, 16, 1, false>(), make_cfg<P, 7, 1, 4, 1, 2, 1, 16, 1, false>()};
    }
    return {};
}

// BF16 / FP8: a 192 x 64 tile of four waves stacked along M (48 x 64 each)
// in one LDS buffer (three workgroups per CU), the same with the next chunk
// prefetched into registers, the 192 x 64 tile of 2 x 2 waves, and a
// double-buffered 96-row tile (the 1x1 projections); 256 x 32/16 for the
// narrow layers.  The first is the default.
template <typename P, int KW, int S, int KC>
Cands cands_lowp(int c_out) {
    if constexpr (KC == 16) {
        if (KW == 7 && S == 1 && c_out == 16)
            return {make_cfg<P, 7, 1, 4, 1, 4, 1, 16, 1, true>(), make_cfg<P, 7, 1, 4, 1, 2, 1, 16, 1, true>()};
        return {};
    } else {
        if (c_out % 64 == 0) {
            Cands c{make_cfg<P, KW, S, 4, 1, 3, 4, KC, 2, 0, false>(), make_cfg<P, KW, S, 4, 1, 3, 4, KC, 2, 2, false>(),
                    make_cfg<P, KW, S, 2, 2, 6, 2, KC, 2, 0, false>(),
                    c_out % 128 == 0 ? make_cfg<P, KW, S, 2, 2, 3, 4, KC, 1, 1>() : make_cfg<P, KW, S, 2, 2, 3, 2, KC, 1, 1>()};
            // 384 x 64 of eight waves stacked along M: half the weight bytes
            // per MAC of the 192-row tiles (stride-1 k7 layers with 16-byte
            // operands; the FP32-in, FP32-out form would not fit the 128
            // registers of four waves per SIMD)
            constexpr bool f32_io = sizeof(typename P::Act) == 4 && sizeof(typename P::OAct) == 4;
            if constexpr (KW == 7 && S == 1 && P::KL == 8 && !P::kFP8 && !f32_io)
                c.push_back(make_cfg<P, 7, 1, 8, 1, 3, 4, KC, 4, 0, false>());
            return c;
        }
        if constexpr (KW == 7 && S == 1) {
            if (c_out == 32)
                return {make_cfg<P, 7, 1, 4, 1, 4, 2, KC, 1, true>(), make_cfg<P, 7, 1, 4, 1, 2, 2, KC, 1, true>(),
                        make_cfg<P, 7, 1, 4, 1, 2, 2, KC, 1, false, false>(),
                        make_cfg<P, 7, 1, 4, 1, 4, 2, KC, 1, false, false>()};
        }
        return {};
    }
}

// k3 convs of the GroupNorm net (BF16 operands, FP32 activations): the
// 64-row-multiple tiles as for k7, and for 32 output channels 256 x 32 tiles
// without the tap-shift reuse.
template <typename P, int S>
Cands cands_k3(int c_out) {
    if (c_out % 64 == 0) return cands_lowp<P, 3, S, 32>(c_out);
    if (S == 1 && c_out == 32)
        return {make_cfg<P, 3, 1, 4, 1, 4, 2, 32, 1, false, false>(), make_cfg<P, 3, 1, 4, 1, 2, 2, 32, 1, false, false>()};
    return {};
}

template <typename P, int KC>
Cands cands_shape_lowp(int kw, int s, int c_out) {
    if (kw == 7 && s == 1) return cands_lowp<P, 7, 1, KC>(c_out);
    if (kw == 7 && s == 2) return c_out >= 64 ? cands_lowp<P, 7, 2, KC>(c_out) : Cands{};
    if (kw == 1 && s == 2) return c_out >= 64 ? cands_lowp<P, 1, 2, KC>(c_out) : Cands{};
    return {};
}

// Convs of the GroupNorm net (k3, and 1x1 stride-2 projections): every one
// writes its output's statistics; AFF (a block's second conv) also normalises
// its input as it stages it.  FP32, or BF16 operands with FP32 activations.
template <bool AFF>
Cands gn_conv_candidates(af_precision p, int kw, int s, int c_in, int c_out) {
    if (p == AF_F32) {
        using P = PGn<PF32, AFF>;
        if (c_in % 16 != 0) return {};
        if (kw == 3 && s == 1) return cands_f32<3, 1, P>(c_out);
        if constexpr (!AFF) {
            if (kw == 3 && s == 2) return c_out >= 64 ? cands_f32<3, 2, P>(c_out) : Cands{};
            if (kw == 1 && s == 2) return c_out >= 64 ? cands_f32<1, 2, P>(c_out) : Cands{};
        }
        return {};
    }
    if (p != AF_BF16_F32ACT || c_in % 32 != 0) return {};
    using P = PGn<PBF16F, AFF>;
    if (kw == 3 && s == 1) return cands_k3<P, 1>(c_out);
    if constexpr (!AFF) {
        if (kw == 3 && s == 2) return cands_k3<P, 2>(c_out);
        if (kw == 1 && s == 2) return c_out >= 64 ? cands_lowp<P, 1, 2, 32>(c_out) : Cands{};
    }
    return {};
}

// role: 1 for the first conv of a residual block (it writes the block's inner
// activation), 2 for the second (it reads it), 0 for any other conv
Cands conv_candidates(af_precision p, int kw, int s, int c_in, int c_out, int role) {
    if (p == AF_F32) {
        if (c_in % 16 != 0) return {};
        if (kw == 7 && s == 1) return cands_f32<7, 1>(c_out);
        if (kw == 7 && s == 2) return c_out >= 64 ? cands_f32<7, 2>(c_out) : Cands{};
        if (kw == 1 && s == 2) return c_out >= 64 ? cands_f32<1, 2>(c_out) : Cands{};
        return {};
    }
    const bool kc32 = c_in % 32 == 0;
    if (kw == 1 && !kc32) return {};  // a 1x1 chunk must fill a whole 32-deep MFMA
    if (!kc32 && c_in % 16 != 0) return {};
    if (p == AF_BF16) {
        if (kc32) return cands_shape_lowp<PBF16, 32>(kw, s, c_out);
        return kw == 7 && s == 1 ? cands_lowp<PBF16, 7, 1, 16>(c_out) : Cands{};
    }
    if (p == AF_BF16_F32ACT) {
        // A block's inner activation feeds only the block's second conv, which
        // rounds it to a BF16 operand as it loads it; the first conv stores it
        // as BF16 directly (the same rounding of the same FP32 value), halving
        // its traffic without changing a bit of the result.  The first conv is
        // k7 with stride 1 or 2, the second k7 with stride 1.
        if (role == 1 && kw == 7) {
            if (s == 1) return kc32 ? cands_lowp<PBF16FB, 7, 1, 32>(c_out) : cands_lowp<PBF16FB, 7, 1, 16>(c_out);
            return kc32 && c_out >= 64 ? cands_lowp<PBF16FB, 7, 2, 32>(c_out) : Cands{};
        }
        if (role == 2 && kw == 7 && s == 1)
            return kc32 ? cands_lowp<PBF16BF, 7, 1, 32>(c_out) : cands_lowp<PBF16BF, 7, 1, 16>(c_out);
        if (kc32) return cands_shape_lowp<PBF16F, 32>(kw, s, c_out);
        return kw == 7 && s == 1 ? cands_lowp<PBF16F, 7, 1, 16>(c_out) : Cands{};
    }
    // FP8: k7 convs with >= 32-channel inputs on the 128-deep instruction
    // (a zero tap pads each 32-channel chunk from 224 to 256), plus
    // single-buffered tiles on the 32-deep one (no padding tap, 8-byte
    // operands: two workgroups fit a CU); 1x1 projections and 16-channel
    // inputs on the 32-deep one
    if (kc32 && kw == 7) {
        Cands c = cands_shape_lowp<PFP8X, 32>(kw, s, c_out);
        if (s == 1 && c_out == 32) {
            c.push_back(make_cfg<PFP8, 7, 1, 4, 1, 2, 2, 32, 1, false, false>());
            c.push_back(make_cfg<PFP8, 7, 1, 4, 1, 4, 2, 32, 1, false, false>());
        } else if (c_out % 64 == 0 && s == 1) {
            c.push_back(make_cfg<PFP8, 7, 1, 2, 2, 6, 2, 32, 2, 0, false>());
            c.push_back(make_cfg<PFP8, 7, 1, 4, 1, 3, 4, 32, 2, 0, false>());
            c.push_back(make_cfg<PFP8, 7, 1, 4, 1, 3, 4, 32, 2, 2, false>());
        } else if (c_out % 64 == 0 && s == 2) {
            c.push_back(make_cfg<PFP8, 7, 2, 2, 2, 6, 2, 32, 2, 0, false>());
            c.push_back(make_cfg<PFP8, 7, 2, 4, 1, 3, 4, 32, 2, 0, false>());
        }
        return c;
    }
    if (kc32) return kw == 1 && s == 2 && c_out >= 64 ? cands_lowp<PFP8, 1, 2, 32>(c_out) : Cands{};
    return kw == 7 && s == 1 ? cands_lowp<PFP8, 7, 1, 16>(c_out) : Cands{};
}

// ---- host rounding onto BF16 / E4M3 grids (round to nearest even) -----------------
double round_sig(double x, int sig, int min_exp, int step_exp) {
    if (x == 0.0) return 0.0;
    if (std::fabs(x) < std::ldexp(1.0, min_exp)) return std::ldexp(std::nearbyint(std::ldexp(x, -step_exp)), step_exp);
    int e;
    double m = std::frexp(x, &e);
    return std::ldexp(std::nearbyint(std::ldexp(m, sig)), e - sig);
}
uint16_t host_bf16_bits(double v) {
    float f = (float)round_sig(v, 8, -126, -133);  // exact: the value is on the BF16 grid
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
}
uint8_t host_e4m3_bits(double v) {
    double r = round_sig(v, 4, -6, -9);
    if (r > 448.0) r = 448.0;
    if (r < -448.0) r = -448.0;
    uint8_t sign = r < 0 ? 0x80 : 0;
    double a = std::fabs(r);
    if (a == 0.0) return sign;
    if (a < 0.015625) return sign | (uint8_t)std::lrint(a * 512.0);
    int e;
    double m = std::frexp(a, &e);           // a = m 2^e, m in [0.5, 1)
    int E = e - 1;                          // a = (2m) 2^E, 2m in [1, 2)
    int mant = (int)std::lrint((2.0 * m - 1.0) * 8.0);
    return sign | (uint8_t)(((E + 7) << 3) | mant);
}

enum Buf { BX = 0, BR = 1, BP = 2 };

// (rows per step, activation row pitch in BF16 elements) of the whole-network
// kernel's candidates (autotuned)
struct FusedShape {
    int rows, pitch;
    bool swz;
};
constexpr FusedShape kFusedSteps[] = {{32, 24, false}, {48, 24, false}, {64, 24, false},
                                      {32, 32, true}, {48, 32, true}, {64, 32, true}};

struct ConvOp {
    int c_in, c_out, kw, s, l_in, l_out, relu;
    int in_buf, out_buf, res_buf;  // res_buf < 0: none
    int amax_in, amax_out;         // FP8 slots
    size_t w_off, b_off;           // folded weights [C_out][KW][C_in] / bias offsets
    Cands cands;                   // tile shapes this layer can run with
    int cand = 0;                  // index of the one in use
    ConvCfg cfg;
    int wpt, tt, tiles_per_win;
    void* d_img = nullptr;         // weight image for cfg (device)
    // GroupNorm nets: gamma, beta of the conv's norm at gn_off of the net's
    // table; its scales and shifts go to slot gn_aff (0: a block's first conv,
    // 1: projection, 2: second conv); the second conv stages its input
    // through slot 0's and then ends the block: its output normalised, plus
    // the skip gn_res (through slot 1's when the block has a projection),
    // ReLU, into gn_out
    size_t gn_off = 0;
    int gn_aff = -1;
    int gn_out = -1, gn_res = -1, gn_res_aff = -1;
};

// M tiling of a layer for its tile height: several short windows per tile, or
// several tiles per window.
void set_tiling(ConvOp& op) {
    const int MT = op.cfg.MT;
    if (op.l_out >= MT) {
        op.wpt = 1; op.tt = MT; op.tiles_per_win = (op.l_out + MT - 1) / MT;
    } else if (MT % op.l_out == 0 && op.l_out % 16 == 0 && MT / op.l_out <= op.cfg.WMAX) {
        op.wpt = MT / op.l_out; op.tt = op.l_out; op.tiles_per_win = 1;
    } else {
        op.wpt = 1; op.tt = MT; op.tiles_per_win = 1;
    }
}

// Weight image of one conv for tile shape cfg: [C_out/NT][C_in/KC][KWP][NT][PB]
// in storage precision, taps >= KW and pad columns zero, BF16/FP8 rows
// swizzled; each chunk is the exact LDS image a workgroup copies with direct
// loads.  wscale: FP8 per-output-channel scales (FP64).
std::vector<unsigned char> build_image(const ConvOp& op, const ConvCfg& cfg, af_precision prec,
                                       const std::vector<double>& wfold, const std::vector<double>& wscale) {
    const size_t esz = prec == AF_F32 ? 4 : (prec == AF_FP8 ? 1 : 2);
    const int NT = cfg.NT, KC = cfg.KC, KWP = cfg.KWP, PB = cfg.PB;
    const int KLs = cfg.KL, SWR = cfg.SWR, SWU = KC / cfg.KL;
    const int n_chunks = op.c_in / KC;
    std::vector<unsigned char> img((size_t)(op.c_out / NT) * n_chunks * KWP * NT * PB * esz, 0);
    for (int o = 0; o < op.c_out; ++o) {
        const int nt = o / NT, n = o % NT;
        for (int j = 0; j < op.kw; ++j)
            for (int c = 0; c < op.c_in; ++c) {
                const int cc = c / KC, ci = c % KC;
                const int row = j * NT + n;   // row of the chunk's LDS image
                const int cs = SWR ? (((ci / KLs) ^ ((row / SWR) & (SWU - 1))) * KLs + ci % KLs) : ci;
                const size_t e = (((size_t)nt * n_chunks + cc) * KWP * NT + row) * PB + cs;
                const double v = wfold[op.w_off + ((size_t)o * op.kw + j) * op.c_in + c];
                if (prec == AF_F32) ((float*)img.data())[e] = (float)v;
                else if (prec == AF_BF16 || prec == AF_BF16_F32ACT) ((uint16_t*)img.data())[e] = host_bf16_bits(v);
                else img[e] = host_e4m3_bits(v / wscale[op.b_off + o]);
            }
    }
    return img;
}

}  // namespace

struct af_net {
    af_net_desc desc;
    af_precision prec;
    int device;
    int64_t macs;
    int stem_lconv, stem_lout;
    int64_t act_elems;  // per window, max over layers
    // GroupNorm nets, per window: conv output statistics ([blocks][2][C], max
    // over layers) and one slot of scales and shifts ([2][C], max over layers)
    int64_t gn_stats_elems = 0, gn_aff_elems = 0;
    int n_slots;
    int last_L, last_C;
    float fc_b;
    std::vector<ConvOp> ops;
    std::vector<double> wfold;    // folded conv weights, host copy for rebuilding images
    std::vector<double> wscale;   // FP8 per-output-channel weight scales
    float* d_b = nullptr;      // conv biases
    float* d_ws = nullptr;     // FP8 per-output-channel scales
    float* d_stem = nullptr;   // stem weights [C][in][k] then bias [C]
    float* d_fc = nullptr;     // fc weights [C_last], then the fc bias
    std::vector<double> bias64;        // folded conv biases (FP64), as created
    double fc_b64 = 0.0;               // fc bias as created
    std::vector<double> params_host;   // FP8 nets: the creation parameters (for calibration)
    double* d_tap = nullptr;           // calibration: per-conv input channel sums [ops][tap_pitch]
    int tap_pitch = 0;
    std::vector<void*> retired;        // weight images replaced by a tile switch (kept for captured graphs)
    int gn_groups = 0;         // > 0: GroupNorm net (stem's gamma, beta first in d_gn)
    float* d_gn = nullptr;     // GroupNorm gamma [C], beta [C] per norm layer
    // kernel timing (af_net_profile_begin/end): one event pair per launch
    bool profiling = false;
    struct Rec {
        int layer;
        int64_t windows;
        int64_t macs;   // per window
        hipEvent_t a, b;
    };
    // whole-network persistent kernel for the 16-channel two-block net (BF16)
    bool fused_ok = false, fused_on = false;
    int n_cu = 0;
    int fused_cand = 1;             // index into kFusedSteps: rows per step
    uint16_t* d_wfused = nullptr;   // [4][16][128]
    float* d_bfused = nullptr;      // [5][16]: stem, convs
    float* d_sfused = nullptr;      // [16][16] stem weights by k = input channel * 8 + tap
    std::vector<Rec> recs;
    std::vector<int64_t> layer_macs;  // per window: stem, convs..., gap/fc
};

namespace {
// bytes per stored activation (every buffer is sized for the widest kind)
size_t act_size(af_precision p) { return (p == AF_F32 || p == AF_BF16_F32ACT) ? 4 : 2; }

void drop_records(af_net* n) {
    for (auto& r : n->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    n->recs.clear();
}

void free_net(af_net* n) {
    if (!n) return;
    drop_records(n);
    for (ConvOp& op : n->ops)
        if (op.d_img) (void)hipFree(op.d_img);
    for (void* r : n->retired) (void)hipFree(r);
    if (n->d_b) (void)hipFree(n->d_b);
    if (n->d_ws) (void)hipFree(n->d_ws);
    if (n->d_stem) (void)hipFree(n->d_stem);
    if (n->d_fc) (void)hipFree(n->d_fc);
    if (n->d_gn) (void)hipFree(n->d_gn);
    if (n->d_wfused) (void)hipFree(n->d_wfused);
    if (n->d_bfused) (void)hipFree(n->d_bfused);
    if (n->d_sfused) (void)hipFree(n->d_sfused);
    delete n;
}
}  // namespace

namespace {
// groups == 0: BatchNorm net (folded); groups > 0: GroupNorm net
af_status create_net(const af_net_desc* d, int groups, const double* params, int64_t n_params,
                     af_precision prec, af_net** out) {
    AF_CHECK_ARG(d && params && out, "desc, params and out must be non-null");
    AF_CHECK_ARG(prec == AF_F32 || prec == AF_BF16 || prec == AF_FP8 || prec == AF_BF16_F32ACT,
                 "unknown precision %d", (int)prec);
    AF_CHECK_ARG(d->in_ch >= 1 && d->in_ch <= 4, "in_ch must be in [1, 4]");
    if (groups) {
        AF_CHECK_ARG(d->kernel == 3 && d->in_ch == 2, "GroupNorm nets are implemented for kernel 3 and 2 inputs");
        AF_CHECK_ARG(prec == AF_F32 || prec == AF_BF16_F32ACT,
                     "GroupNorm nets run in AF_F32 or AF_BF16_F32ACT");
        AF_CHECK_ARG(groups <= 256 && d->stem_ch % groups == 0, "groups must divide stem_ch");
        for (int st = 0; st < d->n_stages && st < 8; ++st)
            AF_CHECK_ARG(d->widths[st] % groups == 0 && d->widths[st] >= 16 && 1024 % d->widths[st] == 0,
                         "GroupNorm widths must be powers of two in [16, 1024] divisible by groups");
    } else {
        AF_CHECK_ARG(d->kernel == 7, "only kernel 7 is implemented");
    }
    AF_CHECK_ARG(d->stem_stride == 1 || d->stem_stride == 2, "stem_stride must be 1 or 2");
    AF_CHECK_ARG(d->n_stages >= 1 && d->n_stages <= 8, "n_stages must be in [1, 8]");
    AF_CHECK_ARG(d->window >= 16 && d->window <= 16384, "window must be in [16, 16384]");
    AF_CHECK_ARG(d->stem_ch >= 16 && 256 % d->stem_ch == 0, "stem_ch must divide 256 and be >= 16");
    const int K = d->kernel;
    af_net* net = new (std::nothrow) af_net();
    if (!net) { set_error("out of host memory"); return AF_ENOMEM; }
    net->desc = *d;
    net->prec = prec;
    net->gn_groups = groups;
    (void)hipGetDevice(&net->device);

    // ---- walk the architecture, fold BN, build the op list --------------------
    const double* p = params;
    const double* p_end = params + n_params;
    std::vector<float> stem;       // weights then bias
    std::vector<double> wfold;     // all MFMA conv weights, [C_out][KW][C_in], folded
    std::vector<float> bias;
    std::vector<float> gnp;        // GroupNorm nets: gamma, beta per norm layer
    size_t gn_off = 0;             // offset of the last conv's pair in gnp
    auto take_conv = [&](int c_out, int c_in, int kw, std::vector<double>& w, std::vector<double>& b) -> bool {
        const size_t nw = (size_t)c_out * c_in * kw;
        if (groups) {
            // weights as they are (no fold, no bias), then gamma and beta
            if (p + nw + 2 * (size_t)c_out > p_end) return false;
            w.assign(nw, 0.0);
            b.assign(c_out, 0.0);
            for (int o = 0; o < c_out; ++o)
                for (int c = 0; c < c_in; ++c)
                    for (int j = 0; j < kw; ++j) w[((size_t)o * kw + j) * c_in + c] = p[((size_t)o * c_in + c) * kw + j];
            gn_off = gnp.size();
            for (size_t i = 0; i < 2 * (size_t)c_out; ++i) gnp.push_back((float)p[nw + i]);
            p += nw + 2 * (size_t)c_out;
            return true;
        }
        if (p + nw + 4 * (size_t)c_out > p_end) return false;
        const double* W = p;
        const double *g = W + nw, *be = g + c_out, *mu = be + c_out, *var = mu + c_out;
        w.assign(nw, 0.0);
        b.assign(c_out, 0.0);
        for (int o = 0; o < c_out; ++o) {
            const double s = g[o] / std::sqrt(var[o] + 1e-5);
            b[o] = be[o] - mu[o] * s;
            for (int c = 0; c < c_in; ++c)
                for (int j = 0; j < kw; ++j)  // reorder to [o][j][c]
                    w[((size_t)o * kw + j) * c_in + c] = W[((size_t)o * c_in + c) * kw + j] * s;
        }
        p = var + c_out;
        return true;
    };
    std::vector<double> w, b;
    if (!take_conv(d->stem_ch, d->in_ch, K, w, b)) { free_net(net); set_error("params too short"); return AF_EINVAL; }
    stem.resize((size_t)d->stem_ch * d->in_ch * K + d->stem_ch);
    for (int o = 0; o < d->stem_ch; ++o)
        for (int c = 0; c < d->in_ch; ++c)
            for (int j = 0; j < K; ++j)
                stem[((size_t)o * d->in_ch + c) * K + j] = (float)w[((size_t)o * K + j) * d->in_ch + c];
    for (int o = 0; o < d->stem_ch; ++o) stem[(size_t)d->stem_ch * d->in_ch * K + o] = (float)b[o];
    net->stem_lconv = (d->window + 2 * (K / 2) - K) / d->stem_stride + 1;
    net->stem_lout = d->stem_pool ? (net->stem_lconv + 2 - 3) / 2 + 1 : net->stem_lconv;
    net->macs = (int64_t)net->stem_lconv * d->stem_ch * d->in_ch * K;
    net->layer_macs.push_back(net->macs);
    net->act_elems = (int64_t)net->stem_lout * d->stem_ch;

    int L = net->stem_lout, C = d->stem_ch, slot_x = 0, n_slots = 1;
    auto add_conv = [&](int c_in, int c_out, int kw, int s, int l_in, int relu, int in_buf, int out_buf,
                        int res_buf, int amax_in) -> bool {
        ConvOp op{};
        op.c_in = c_in; op.c_out = c_out; op.kw = kw; op.s = s; op.l_in = l_in;
        op.l_out = (l_in + 2 * (kw / 2) - kw) / s + 1;
        op.relu = relu; op.in_buf = in_buf; op.out_buf = out_buf; op.res_buf = res_buf;
        op.amax_in = amax_in;
        op.amax_out = n_slots++;
        op.w_off = wfold.size();
        op.b_off = bias.size();
        if (groups)   // the block's second conv reads BR
            op.cands = in_buf == BR ? gn_conv_candidates<true>(prec, kw, s, c_in, c_out)
                                    : gn_conv_candidates<false>(prec, kw, s, c_in, c_out);
        else
            op.cands = conv_candidates(prec, kw, s, c_in, c_out, out_buf == BR ? 1 : (in_buf == BR ? 2 : 0));
        op.cand = 0;
        op.cfg = op.cands.empty() ? ConvCfg{} : op.cands[0];
        if (!op.cfg.fn) {
            set_error("no conv kernel for kw=%d stride=%d c_in=%d c_out=%d", kw, s, c_in, c_out);
            return false;
        }
        if (!take_conv(c_out, c_in, kw, w, b)) { set_error("params too short"); return false; }
        if (groups) {   // raw conv; GroupNorm, residual and ReLU are applied later
            op.relu = 0;
            op.res_buf = -1;
            op.gn_off = gn_off;
        }
        set_tiling(op);
        wfold.insert(wfold.end(), w.begin(), w.end());
        for (int o = 0; o < c_out; ++o) bias.push_back((float)b[o]);
        net->bias64.insert(net->bias64.end(), b.begin(), b.end());
        net->macs += (int64_t)op.l_out * c_out * c_in * kw;
        net->layer_macs.push_back((int64_t)op.l_out * c_out * c_in * kw);
        net->act_elems = std::max<int64_t>(net->act_elems, (int64_t)op.l_out * c_out);
        if (groups) {
            net->gn_stats_elems = std::max<int64_t>(net->gn_stats_elems, (int64_t)(op.l_out + 15) / 16 * 2 * c_out);
            net->gn_aff_elems = std::max<int64_t>(net->gn_aff_elems, 2 * (int64_t)c_out);
        }
        net->ops.push_back(op);
        return true;
    };
    for (int st = 0; st < d->n_stages; ++st) {
        for (int bl = 0; bl < d->blocks[st]; ++bl) {
            const int wdt = d->widths[st];
            const int s = (bl == 0 && st > 0) ? 2 : 1;
            const bool proj = s != 1 || C != wdt;
            if (!add_conv(C, wdt, K, s, L, 1, BX, BR, -1, slot_x)) { free_net(net); return AF_EINVAL; }
            const int slot_r = net->ops.back().amax_out;
            const int l_out = net->ops.back().l_out;
            // conv2 runs after the projection: its parameters follow conv2's in the
            // parameter order, so read conv2 first and swap the two ops afterwards
            if (!add_conv(wdt, wdt, K, 1, l_out, 1, BR, BX, proj ? BP : BX, slot_r)) { free_net(net); return AF_EINVAL; }
            if (proj) {
                if (!add_conv(C, wdt, 1, s, L, 0, BX, BP, -1, slot_x)) { free_net(net); return AF_EINVAL; }
                std::swap(net->ops[net->ops.size() - 1], net->ops[net->ops.size() - 2]);
                std::swap(net->layer_macs[net->layer_macs.size() - 1], net->layer_macs[net->layer_macs.size() - 2]);
                slot_x = net->ops.back().amax_out;   // conv2 (now last) writes the block output
            } else {
                slot_x = net->ops.back().amax_out;
            }
            if (groups) {
                // buffers: conv1 X -> R (raw); with a projection, proj X -> P
                // (raw), then conv2 relu(GN1(R)) -> X (raw), and the block
                // ends GN2(X) + GNp(P) -> X, ReLU; without, conv2
                // relu(GN1(R)) -> P, then GN2(P) + X -> X, ReLU
                const size_t n_ops = net->ops.size();
                ConvOp& c1 = net->ops[n_ops - (proj ? 3 : 2)];
                ConvOp& c2 = net->ops[n_ops - 1];
                c1.gn_aff = 0;
                c2.gn_aff = 2; c2.gn_out = BX;
                if (proj) {
                    ConvOp& pj = net->ops[n_ops - 2];
                    pj.gn_aff = 1;
                    c2.out_buf = BX; c2.gn_res = BP; c2.gn_res_aff = 1;
                } else {
                    c2.out_buf = BP; c2.gn_res = BX; c2.gn_res_aff = -1;
                }
            }
            C = wdt;
            L = l_out;
        }
    }
    if (p + C + 1 != p_end) {
        free_net(net);
        set_error("params length mismatch: %lld left for an FC of %d inputs", (long long)(p_end - p), C);
        return AF_EINVAL;
    }
    if (256 % C != 0 && C % 256 != 0) {
        free_net(net);
        set_error("last width must divide 256 or be a multiple of it");
        return AF_EINVAL;
    }
    std::vector<float> fc(C + 1);
    for (int c = 0; c <= C; ++c) fc[c] = (float)p[c];   // weights, then the bias
    net->fc_b = (float)p[C];
    net->fc_b64 = p[C];
    net->tap_pitch = 1;
    for (const ConvOp& op : net->ops) net->tap_pitch = std::max(net->tap_pitch, op.c_in);
    if (prec == AF_FP8) net->params_host.assign(params, params + n_params);
    net->macs += C;
    net->layer_macs.push_back(C);
    if (groups) net->layer_macs.push_back(0);   // every GroupNorm launch, timed as one more layer
    net->last_L = L;
    net->last_C = C;
    net->n_slots = n_slots;

    // ---- FP8 weight scales and per-layer weight images -------------------------------------
    std::vector<double> wscale_full(bias.size(), 1.0);
    std::vector<float> wsc(bias.size(), 1.f);
    if (prec == AF_FP8) {
        for (const ConvOp& op : net->ops) {
            const size_t per = (size_t)op.kw * op.c_in;
            for (int o = 0; o < op.c_out; ++o) {
                const double* row = &wfold[op.w_off + o * per];
                double mx = 0.0;
                for (size_t i = 0; i < per; ++i) mx = std::max(mx, std::fabs(row[i]));
                const double sc = mx > 0 ? mx / 448.0 : 1.0;
                wscale_full[op.b_off + o] = sc;
                wsc[op.b_off + o] = (float)sc;
            }
        }
    }
    auto upload = [&](void** dst, const void* src, size_t bytes) -> bool {
        if (bytes == 0) return true;
        if (hipMalloc(dst, bytes) != hipSuccess) return false;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    for (ConvOp& op : net->ops) {
        std::vector<unsigned char> img = build_image(op, op.cfg, prec, wfold, wscale_full);
        if (!upload(&op.d_img, img.data(), img.size())) {
            free_net(net);
            set_error("device allocation/upload of the weights failed");
            return AF_ENOMEM;
        }
    }
    net->wfold = wfold;
    net->wscale = wscale_full;
    if (groups && !upload((void**)&net->d_gn, gnp.data(), gnp.size() * 4)) {
        free_net(net);
        set_error("device allocation/upload of the weights failed");
        return AF_ENOMEM;
    }
    if (!upload((void**)&net->d_b, bias.data(), bias.size() * 4) ||
        !upload((void**)&net->d_stem, stem.data(), stem.size() * 4) ||
        !upload((void**)&net->d_fc, fc.data(), fc.size() * 4) ||
        (prec == AF_FP8 && !upload((void**)&net->d_ws, wsc.data(), wsc.size() * 4))) {
        free_net(net);
        set_error("device allocation/upload of the weights failed");
        return AF_ENOMEM;
    }
    // fused whole-network path: stem 2->16 k7 s1, one stage of two 16-channel
    // blocks, BF16
    const bool tiny = !groups && d->in_ch == 2 && d->stem_ch == 16 && d->stem_stride == 1 && !d->stem_pool &&
                      d->n_stages == 1 && d->widths[0] == 16 && d->blocks[0] == 2 && net->ops.size() == 4;
    if (tiny && prec == AF_BF16) {
        // conv weights [layer][out][k = tap * 16 + in]; the eighth tap of the
        // second conv of each block is the identity (it adds the block input)
        std::vector<uint16_t> wf(4 * 16 * 128, 0);
        std::vector<float> bf(5 * 16), sf(16 * 16, 0.f);
        for (int o = 0; o < 16; ++o) {
            for (int c = 0; c < 2; ++c)
                for (int j = 0; j < 7; ++j) sf[o * 16 + c * 8 + j] = stem[((size_t)o * 2 + c) * 7 + j];
            bf[o] = stem[(size_t)16 * 2 * 7 + o];
        }
        for (int l = 0; l < 4; ++l) {
            const ConvOp& op = net->ops[l];
            for (int o = 0; o < 16; ++o) {
                for (int j = 0; j < 7; ++j)
                    for (int c = 0; c < 16; ++c)
                        wf[((size_t)l * 16 + o) * 128 + j * 16 + c] =
                            host_bf16_bits(wfold[op.w_off + ((size_t)o * 7 + j) * 16 + c]);
                if (l == 1 || l == 3) wf[((size_t)l * 16 + o) * 128 + 7 * 16 + o] = host_bf16_bits(1.0);
                bf[(l + 1) * 16 + o] = bias[op.b_off + o];
            }
        }
        if (!upload((void**)&net->d_wfused, wf.data(), wf.size() * 2) ||
            !upload((void**)&net->d_bfused, bf.data(), bf.size() * 4) ||
            !upload((void**)&net->d_sfused, sf.data(), sf.size() * 4)) {
            free_net(net);
            set_error("device allocation/upload of the fused weights failed");
            return AF_ENOMEM;
        }
        net->fused_ok = net->fused_on = true;
    }
    if (hipDeviceGetAttribute(&net->n_cu, hipDeviceAttributeMultiprocessorCount, net->device) != hipSuccess)
        net->n_cu = 256;
    *out = net;
    return AF_OK;
}
}  // namespace

extern "C" af_status af_net_create(const af_net_desc* d, const double* params, int64_t n_params,
                                   af_precision prec, af_net** out) {
    clear_error();
    return create_net(d, 0, params, n_params, prec, out);
}

extern "C" af_status af_net_create_gn(const af_net_desc* d, int32_t groups, const double* params,
                                      int64_t n_params, af_precision prec, af_net** out) {
    clear_error();
    AF_CHECK_ARG(groups >= 1, "groups must be >= 1");
    return create_net(d, groups, params, n_params, prec, out);
}

extern "C" int af_net_fused(const af_net* net) { return net && net->fused_ok && net->fused_on ? 1 : 0; }

extern "C" af_status af_net_set_fused(af_net* net, int enable) {
    clear_error();
    AF_CHECK_ARG(net, "net must be non-null");
    AF_CHECK_ARG(!enable || net->fused_ok, "this net has no fused path (needs the 16-channel two-block net in BF16)");
    net->fused_on = enable != 0;
    return AF_OK;
}

extern "C" void af_net_destroy(af_net* net) { free_net(net); }
extern "C" int64_t af_net_macs(const af_net* net) { return net ? net->macs : 0; }

namespace {
size_t buf_bytes(const af_net* net, int64_t batch) {
    return align_up((size_t)batch * net->act_elems * act_size(net->prec), 256);
}
size_t amax_bytes(const af_net* net, int64_t batch) {
    return net->prec == AF_FP8 ? align_up((size_t)net->n_slots * batch * 4, 256) : 0;
}
// GroupNorm nets: the statistics buffer, then three slots of scales and shifts
size_t gn_stats_bytes(const af_net* net, int64_t batch) {
    return align_up((size_t)batch * net->gn_stats_elems * 4, 256);
}
size_t gn_aff_bytes(const af_net* net, int64_t batch) {
    return align_up((size_t)batch * net->gn_aff_elems * 4, 256);
}
}  // namespace

namespace {
template <typename P>
bool launch_stem_p(const af_net_desc& d, const StemArgs& sa, int nb, size_t lds, hipStream_t s) {
    if (d.in_ch != 2 || d.kernel != 7) return false;
    if (d.stem_ch == 16 && d.stem_stride == 1 && !d.stem_pool)
        hipLaunchKernelGGL((stem2_kernel<P, 16, 1, false>), dim3(nb), dim3(256), lds, s, sa);
    else if (d.stem_ch == 32 && d.stem_stride == 2 && d.stem_pool)
        hipLaunchKernelGGL((stem_mfma_kernel<P, 32>), dim3(nb), dim3(256), StemMfmaGeom::lds_bytes(sa.window), s, sa);
    else if (d.stem_ch == 32 && d.stem_stride == 1 && !d.stem_pool)
        hipLaunchKernelGGL((stem2_kernel<P, 32, 1, false>), dim3(nb), dim3(256), lds, s, sa);
    else
        return false;
    return true;
}
bool launch_stem(af_precision p, const af_net_desc& d, const StemArgs& sa, int nb, size_t lds, hipStream_t s) {
    if (p == AF_F32) return launch_stem_p<PF32>(d, sa, nb, lds, s);
    if (p == AF_BF16) return launch_stem_p<PBF16>(d, sa, nb, lds, s);
    if (p == AF_BF16_F32ACT) return launch_stem_p<PF32>(d, sa, nb, lds, s);   // FP32 stem output
    return launch_stem_p<PFP8>(d, sa, nb, lds, s);
}
}  // namespace

extern "C" size_t af_score_workspace_bytes(const af_net* net, int64_t batch) {
    if (!net || batch < 1) return 0;
    return 3 * buf_bytes(net, batch) + amax_bytes(net, batch) + gn_stats_bytes(net, batch) +
           3 * gn_aff_bytes(net, batch);
}

namespace {
af_status score_batches(const af_net* net, const float* y, int64_t ld_y, int64_t n, int64_t stride,
                        int64_t n_windows, const int64_t* shift, int64_t wrap, const int64_t* table, int n_entries,
                        float* logits, void* ws, size_t ws_bytes, hipStream_t s);

// The whole-network kernel with candidate `cand` (kFusedSteps), on a
// persistent grid of as many one-wavefront workgroups as the occupancy query
// says fit the device at once; they take windows from the queue counter
// fa.next, which a fill kernel clears first (no memset node in a captured
// graph).
bool launch_fused(int cand, int n_cu, const FusedTinyArgs& fa, hipStream_t s) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, s, (uint32_t*)fa.next, (int64_t)1, 0u);
    auto go = [&](auto kernel) -> bool {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, 64, 0) != hipSuccess || occ < 1) occ = 1;
        const int64_t grid = std::min<int64_t>(fa.n_windows, (int64_t)occ * n_cu);
        hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(64), 0, s, fa);
        return hipPeekAtLastError() == hipSuccess;
    };
    switch (cand) {
        case 0: return go(fused_tiny_bf16_kernel<32, 24, false>);
        case 1: return go(fused_tiny_bf16_kernel<48, 24, false>);
        case 2: return go(fused_tiny_bf16_kernel<64, 24, false>);
        case 3: return go(fused_tiny_bf16_kernel<32, 32, true>);
        case 4: return go(fused_tiny_bf16_kernel<48, 32, true>);
        default: return go(fused_tiny_bf16_kernel<64, 32, true>);
    }
}
}

extern "C" af_status af_score_windows(const af_net* net, const float* y, int64_t n_ch, int64_t ld_y, int64_t n,
                                      int64_t stride, int64_t n_windows, const int64_t* ch_shift, int64_t wrap,
                                      float* logits, void* ws, size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(net && y, "net and y must be non-null");
    AF_CHECK_ARG(logits || n_windows == 0, "logits must be non-null");
    AF_CHECK_ARG(n_ch == net->desc.in_ch, "n_ch %lld does not match the net's %d inputs", (long long)n_ch, net->desc.in_ch);
    AF_CHECK_ARG(n >= 1 && ld_y >= n && stride >= 1 && n_windows >= 0, "need n >= 1, ld_y >= n, stride >= 1, n_windows >= 0");
    AF_CHECK_ARG(wrap >= 0 && wrap <= n, "wrap must be in [0, n]");
    int dev = -1;
    (void)hipGetDevice(&dev);
    AF_CHECK_ARG(dev == net->device, "net was created on device %d, current device is %d", net->device, dev);
    const int window = net->desc.window;
    AF_CHECK_ARG(wrap == 0 || wrap >= window, "wrap must be 0 or at least the window length %d", window);
    int64_t shift[4] = {0, 0, 0, 0};
    for (int c = 0; c < n_ch; ++c) {
        shift[c] = ch_shift ? ch_shift[c] : 0;
        AF_CHECK_ARG(shift[c] >= 0, "ch_shift must be non-negative");
        if (wrap == 0 && n_windows > 0)
            AF_CHECK_ARG((n_windows - 1) * stride + shift[c] + window <= n,
                         "window %lld of channel %d ends past n = %lld", (long long)(n_windows - 1), c, (long long)n);
    }
    if (n_windows == 0) return AF_OK;
    return score_batches(net, y, ld_y, n, stride, n_windows, shift, wrap, nullptr, 0, logits, ws, ws_bytes,
                         (hipStream_t)stream);
}

namespace {
// Score n_windows windows in passes of the largest batch the workspace holds.
// Plain mode (table == null): window i of channel c starts at i*stride + shift[c]
// (mod wrap).  Timeslide mode: addressing comes from the device work table.
af_status score_batches(const af_net* net, const float* y, int64_t ld_y, int64_t n, int64_t stride,
                        int64_t n_windows, const int64_t* shift, int64_t wrap, const int64_t* table, int n_entries,
                        float* logits, void* ws, size_t ws_bytes, hipStream_t s) {
    const int window = net->desc.window;
    const int64_t n_ch = net->desc.in_ch;
    af_net* mnet0 = const_cast<af_net*>(net);   // timing records only
    // the whole-network kernel indexes samples with 32 bits
    if (net->fused_ok && net->fused_on && n_ch * ld_y < (1LL << 31)) {
        FusedTinyArgs fa{};
        StemArgs& sa = fa.st;
        sa.y = y; sa.ld_y = ld_y; sa.n = n; sa.stride = stride; sa.wrap = wrap; sa.first_window = 0;
        sa.table = table; sa.n_entries = n_entries;
        for (int c = 0; c < 4; ++c) sa.shift[c] = c < n_ch ? shift[c] : 0;
        sa.n_ch = (int)n_ch; sa.window = window;
        fa.wstem = net->d_sfused; fa.wconv = net->d_wfused; fa.bias = net->d_bfused; fa.fc = net->d_fc;
        fa.logits = logits; fa.n_windows = n_windows;
        AF_CHECK_ARG(ws && ws_bytes >= 256, "workspace too small: the whole-network kernel needs 256 bytes");
        fa.next = (unsigned int*)ws;
        af_net::Rec r{1, n_windows, net->macs, nullptr, nullptr};
        if (net->profiling) {
            if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess ||
                hipEventRecord(r.a, s) != hipSuccess) { set_error("profiling event failed"); return AF_EHIP; }
        }
        if (!launch_fused(net->fused_cand, net->n_cu, fa, s)) {
            set_error("whole-network kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
            return AF_EHIP;
        }
        if (net->profiling) {
            if (hipEventRecord(r.b, s) != hipSuccess) { set_error("profiling event failed"); return AF_EHIP; }
            mnet0->recs.push_back(r);
        }
        return AF_OK;
    }
    int64_t batch = 0;
    {
        // largest batch that fits the workspace
        int64_t lo = 0, hi = n_windows;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (af_score_workspace_bytes(net, mid) <= ws_bytes) lo = mid; else hi = mid - 1;
        }
        batch = lo;
    }
    AF_CHECK_ARG(ws && batch >= 1, "workspace too small: one window needs %zu bytes", af_score_workspace_bytes(net, 1));
    AF_CHECK_ARG(batch * net->act_elems < (1LL << 31) && batch < (1LL << 24), "batch too large");
    const size_t bb = buf_bytes(net, batch);
    void* buf[3] = {ws, (char*)ws + bb, (char*)ws + 2 * bb};
    uint32_t* amax = net->prec == AF_FP8 ? (uint32_t*)((char*)ws + 3 * bb) : nullptr;
    float* gn_stats = nullptr;
    float* gn_aff[3] = {nullptr, nullptr, nullptr};
    if (net->gn_groups) {
        char* g0 = (char*)ws + 3 * bb + amax_bytes(net, batch);
        gn_stats = (float*)g0;
        for (int k = 0; k < 3; ++k)
            gn_aff[k] = (float*)(g0 + gn_stats_bytes(net, batch) + k * gn_aff_bytes(net, batch));
    }
    const af_net_desc& d = net->desc;
    af_net* mnet = const_cast<af_net*>(net);  // timing records only; the weights stay read-only
    auto t_begin = [&](int layer, int64_t nw) -> bool {
        if (!net->profiling) return true;
        af_net::Rec r{layer, nw, net->layer_macs[layer], nullptr, nullptr};
        if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return false;
        if (hipEventRecord(r.a, s) != hipSuccess) return false;
        mnet->recs.push_back(r);
        return true;
    };
    auto t_end = [&]() -> bool {
        return !net->profiling || hipEventRecord(mnet->recs.back().b, s) == hipSuccess;
    };

    for (int64_t w0 = 0; w0 < n_windows; w0 += batch) {
        const int nb = (int)std::min<int64_t>(batch, n_windows - w0);
        if (amax) {
            const int64_t cnt = (int64_t)net->n_slots * batch;
            hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, amax, cnt, 0u);
        }
        StemArgs sa{};
        sa.y = y; sa.ld_y = ld_y; sa.n = n; sa.stride = stride; sa.wrap = wrap; sa.first_window = w0;
        sa.table = table; sa.n_entries = n_entries;
        for (int c = 0; c < 4; ++c) sa.shift[c] = shift[c];
        sa.n_ch = (int)n_ch; sa.window = window;
        sa.w = net->d_stem; sa.b = net->d_stem + (size_t)d.stem_ch * d.in_ch * d.kernel;
        sa.out = buf[BX]; sa.amax_out = amax;
        sa.C = d.stem_ch; sa.KW = d.kernel; sa.s0 = d.stem_stride; sa.pool = d.stem_pool;
        sa.L_conv = net->stem_lconv; sa.L_out = net->stem_lout;
        const size_t stem_lds = (size_t)n_ch * window * sizeof(float);
        const int gn_layer = (int)net->layer_macs.size() - 1;
        if (!t_begin(0, nb)) { set_error("profiling event failed"); return AF_EHIP; }
        constexpr int STEM_MAXR = 48;
        if (net->gn_groups && d.stem_ch == 32 && d.stem_pool && net->stem_lconv % 64 == 0 &&
            net->stem_lconv / 32 <= STEM_MAXR) {
            // conv, GroupNorm, ReLU and pool in one pass into X
            sa.out = buf[BX];
            hipLaunchKernelGGL((gn_stem_fused_kernel<2, 3, STEM_MAXR>), dim3(nb), dim3(1024), stem_lds, s, sa,
                               (const float*)net->d_gn, (const float*)net->d_gn + 32, net->gn_groups);
            AF_LAUNCHED();
            t_end();
        } else if (net->gn_groups) {
            // conv, GroupNorm, ReLU (and pool) in two passes over the staged window into X
            sa.out = buf[BX];
            hipLaunchKernelGGL((gn_stem_kernel<2, 3>), dim3(nb), dim3(256), stem_lds, s, sa,
                               (const float*)net->d_gn, (const float*)net->d_gn + d.stem_ch, net->gn_groups);
            AF_LAUNCHED();
            t_end();
        } else if (!launch_stem(net->prec, d, sa, nb, stem_lds, s)) {
            if (net->prec == AF_F32 || net->prec == AF_BF16_F32ACT)
                hipLaunchKernelGGL(stem_kernel<PF32>, dim3(nb), dim3(256), stem_lds, s, sa);
            else if (net->prec == AF_BF16) hipLaunchKernelGGL(stem_kernel<PBF16>, dim3(nb), dim3(256), stem_lds, s, sa);
            else hipLaunchKernelGGL(stem_kernel<PFP8>, dim3(nb), dim3(256), stem_lds, s, sa);
        }
        if (!net->gn_groups) {
            AF_LAUNCHED();
            t_end();
        }
        int layer = 0;
        for (const ConvOp& op : net->ops) {
            ++layer;
            ConvArgs a{};
            a.in = buf[op.in_buf];
            a.out = buf[op.out_buf];
            a.res = op.res_buf >= 0 ? buf[op.res_buf] : nullptr;
            a.w = op.d_img;
            a.bias = net->d_b + op.b_off;
            a.wscale = net->d_ws ? net->d_ws + op.b_off : nullptr;
            a.amax_in = amax ? amax + (size_t)op.amax_in * batch : nullptr;
            a.amax_out = amax ? amax + (size_t)op.amax_out * batch : nullptr;
            a.C_in = op.c_in; a.C_out = op.c_out; a.L_in = op.l_in; a.L_out = op.l_out;
            a.relu = op.relu;
            a.n_win = nb;
            a.wpt = op.wpt;
            a.tt = op.tt;
            a.tiles_per_win = op.tiles_per_win;
            if (net->d_tap)   // calibration of an FP8 net: this FP32 net's conv input sums
                hipLaunchKernelGGL(channel_sum_kernel, dim3((unsigned)op.c_in), dim3(256), 0, s,
                                   (const float*)buf[op.in_buf], (int64_t)nb * op.l_in, op.c_in,
                                   net->d_tap + (size_t)(layer - 1) * net->tap_pitch);
            if (net->gn_groups) {
                a.gn_stats = gn_stats;
                a.in_aff = op.in_buf == BR ? gn_aff[0] : nullptr;
            }
            if (!t_begin(layer, nb)) { set_error("profiling event failed"); return AF_EHIP; }
            op.cfg.fn(a, s);
            AF_LAUNCHED();
            t_end();
            if (net->gn_groups) {
                // the statistics become this conv's scales and shifts; a
                // block's second conv then ends the block
                if (!t_begin(gn_layer, nb)) { set_error("profiling event failed"); return AF_EHIP; }
                hipLaunchKernelGGL(gn_finalize_kernel, dim3((unsigned)nb), dim3(256), 0, s, (const float*)gn_stats,
                                   (op.l_out + 15) / 16, op.l_out, op.c_out, net->gn_groups,
                                   (const float*)net->d_gn + op.gn_off, (const float*)net->d_gn + op.gn_off + op.c_out,
                                   gn_aff[op.gn_aff]);
                AF_LAUNCHED();
                if (op.gn_out >= 0) {
                    GnApplyArgs g{};
                    g.in = (const float*)buf[op.out_buf];
                    g.res = (const float*)buf[op.gn_res];
                    g.out = (float*)buf[op.gn_out];
                    g.aff = gn_aff[op.gn_aff];
                    g.res_aff = op.gn_res_aff >= 0 ? gn_aff[op.gn_res_aff] : nullptr;
                    g.LC4 = op.l_out * op.c_out / 4;
                    g.C = op.c_out;
                    g.relu = 1;
                    constexpr int U = 4;
                    g.n_slice = (g.LC4 + 256 * U - 1) / (256 * U);
                    hipLaunchKernelGGL(gn_apply_kernel<U>, dim3((unsigned)(g.n_slice * nb)), dim3(256), 0, s, g);
                    AF_LAUNCHED();
                }
                t_end();
            }
        }
        if (!t_begin(layer + 1, nb)) { set_error("profiling event failed"); return AF_EHIP; }
        if (act_size(net->prec) == 4)
            hipLaunchKernelGGL(gap_fc_kernel<PF32>, dim3(nb), dim3(256), 0, s, buf[BX], net->last_L, net->last_C,
                               (const float*)net->d_fc, logits + w0);
        else
            hipLaunchKernelGGL(gap_fc_kernel<PBF16>, dim3(nb), dim3(256), 0, s, buf[BX], net->last_L, net->last_C,
                               (const float*)net->d_fc, logits + w0);
        AF_LAUNCHED();
        t_end();
    }
    return AF_OK;
}

}  // namespace

size_t timeslide_table_bytes(int64_t n_seg, int64_t n_slides) {
    return align_up((size_t)(n_seg * n_slides) * 4 * sizeof(int64_t), 256);
}

extern "C" int64_t af_timeslide_n_windows(const int64_t* seg_len, int64_t n_seg, int64_t n_slides, int64_t window,
                                          int64_t stride) {
    if (!seg_len || n_seg < 0 || n_slides < 0 || window < 1 || stride < 1) return -1;
    int64_t tot = 0;
    for (int64_t sg = 0; sg < n_seg; ++sg)
        if (seg_len[sg] >= window) tot += n_slides * ((seg_len[sg] - window) / stride + 1);
    return tot;
}

extern "C" size_t af_timeslide_workspace_bytes(const af_net* net, int64_t n_seg, int64_t n_slides, int64_t batch) {
    if (!net || n_seg < 1 || n_slides < 1 || batch < 1) return 0;
    return timeslide_table_bytes(n_seg, n_slides) + af_score_workspace_bytes(net, batch);
}

namespace {
// Build the (segment, slide) table; returns the window total or -1 on error.
int64_t build_table(const af_net* net, const int64_t* seg_off, const int64_t* seg_len, int64_t n_seg,
                    const int64_t* shifts, int64_t n_slides, int64_t stride, int64_t n, std::vector<int64_t>& tab) {
    const int64_t window = net->desc.window;
    tab.assign((size_t)(n_seg * n_slides) * 4, 0);
    int64_t tot = 0;
    for (int64_t sg = 0; sg < n_seg; ++sg) {
        if (!(seg_off[sg] >= 0 && seg_len[sg] >= 0 && seg_off[sg] + seg_len[sg] <= n)) {
            set_error("segment %lld [%lld, +%lld) is not inside [0, n)", (long long)sg, (long long)seg_off[sg],
                      (long long)seg_len[sg]);
            return -1;
        }
        const int64_t nw = seg_len[sg] >= window ? (seg_len[sg] - window) / stride + 1 : 0;
        for (int64_t k = 0; k < n_slides; ++k) {
            if (shifts[k] < 0) { set_error("shifts must be non-negative"); return -1; }
            int64_t* e = &tab[(size_t)(sg * n_slides + k) * 4];
            e[0] = seg_off[sg];
            e[1] = seg_len[sg];
            e[2] = seg_len[sg] > 0 ? shifts[k] % seg_len[sg] : 0;
            e[3] = tot;
            tot += nw;
        }
    }
    return tot;
}

af_status check_timeslide_args(const af_net* net, int64_t n_ch, int64_t ld_y, int64_t n, int64_t stride,
                               int64_t n_seg, int64_t n_slides) {
    AF_CHECK_ARG(n_ch == net->desc.in_ch, "n_ch %lld does not match the net's %d inputs", (long long)n_ch, net->desc.in_ch);
    AF_CHECK_ARG(n >= 1 && ld_y >= n && stride >= 1 && n_seg >= 1 && n_slides >= 1,
                 "need n >= 1, ld_y >= n, stride >= 1, n_seg >= 1, n_slides >= 1");
    AF_CHECK_ARG(n_seg * n_slides < (1LL << 30), "too many (segment, slide) pairs");
    int dev = -1;
    (void)hipGetDevice(&dev);
    AF_CHECK_ARG(dev == net->device, "net was created on device %d, current device is %d", net->device, dev);
    return AF_OK;
}
}  // namespace

extern "C" af_status af_timeslide_prepare(const af_net* net, const int64_t* seg_off, const int64_t* seg_len,
                                          int64_t n_seg, const int64_t* shifts, int64_t n_slides, int64_t stride,
                                          int64_t n, void* ws, size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(net && seg_off && seg_len && shifts, "net, seg_off, seg_len and shifts must be non-null");
    af_status st = check_timeslide_args(net, net->desc.in_ch, n, n, stride, n_seg, n_slides);
    if (st != AF_OK) return st;
    std::vector<int64_t> tab;
    if (build_table(net, seg_off, seg_len, n_seg, shifts, n_slides, stride, n, tab) < 0) return AF_EINVAL;
    const size_t tb = timeslide_table_bytes(n_seg, n_slides);
    AF_CHECK_ARG(ws && ws_bytes >= tb + af_score_workspace_bytes(net, 1),
                 "workspace too small: need at least %zu bytes", tb + af_score_workspace_bytes(net, 1));
    hipStream_t s = (hipStream_t)stream;
    // the table is a few KB; a blocking copy keeps its host storage simple
    AF_HIP(hipMemcpyAsync(ws, tab.data(), tab.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    AF_HIP(hipStreamSynchronize(s));
    return AF_OK;
}

extern "C" af_status af_score_timeslides_prepared(const af_net* net, const float* y, int64_t n_ch, int64_t ld_y,
                                                  int64_t n, int64_t n_seg, int64_t n_slides, int64_t stride,
                                                  int64_t n_windows, float* logits, void* ws, size_t ws_bytes,
                                                  af_stream stream) {
    clear_error();
    AF_CHECK_ARG(net && y, "net and y must be non-null");
    af_status st = check_timeslide_args(net, n_ch, ld_y, n, stride, n_seg, n_slides);
    if (st != AF_OK) return st;
    AF_CHECK_ARG(n_windows >= 0 && (logits || n_windows == 0), "bad n_windows or logits");
    if (n_windows == 0) return AF_OK;
    const size_t tb = timeslide_table_bytes(n_seg, n_slides);
    AF_CHECK_ARG(ws && ws_bytes >= tb + af_score_workspace_bytes(net, 1),
                 "workspace too small: need at least %zu bytes", tb + af_score_workspace_bytes(net, 1));
    int64_t zero[4] = {0, 0, 0, 0};
    return score_batches(net, y, ld_y, n, stride, n_windows, zero, 0, (const int64_t*)ws, (int)(n_seg * n_slides),
                         logits, (char*)ws + tb, ws_bytes - tb, (hipStream_t)stream);
}

extern "C" af_status af_score_timeslides(const af_net* net, const float* y, int64_t n_ch, int64_t ld_y, int64_t n,
                                         const int64_t* seg_off, const int64_t* seg_len, int64_t n_seg,
                                         const int64_t* shifts, int64_t n_slides, int64_t stride, float* logits,
                                         void* ws, size_t ws_bytes, af_stream stream) {
    clear_error();
    AF_CHECK_ARG(net && y && seg_off && seg_len && shifts, "net, y, seg_off, seg_len and shifts must be non-null");
    af_status st = check_timeslide_args(net, n_ch, ld_y, n, stride, n_seg, n_slides);
    if (st != AF_OK) return st;
    std::vector<int64_t> tab;
    const int64_t tot = build_table(net, seg_off, seg_len, n_seg, shifts, n_slides, stride, n, tab);
    if (tot < 0) return AF_EINVAL;
    AF_CHECK_ARG(logits || tot == 0, "logits must be non-null");
    if (tot == 0) return AF_OK;
    st = af_timeslide_prepare(net, seg_off, seg_len, n_seg, shifts, n_slides, stride, n, ws, ws_bytes, stream);
    if (st != AF_OK) return st;
    return af_score_timeslides_prepared(net, y, n_ch, ld_y, n, n_seg, n_slides, stride, tot, logits, ws, ws_bytes,
                                        stream);
}

namespace afm {
int net_window(const af_net* net) { return net->desc.window; }
int net_in_ch(const af_net* net) { return net->desc.in_ch; }
int net_device(const af_net* net) { return net->device; }

af_status score_table(const af_net* net, const float* y, int64_t ld_y, int64_t n, int64_t stride,
                      int64_t n_windows, const int64_t* table, int n_entries, float* logits, void* ws,
                      size_t ws_bytes, hipStream_t s) {
    int64_t zero[4] = {0, 0, 0, 0};
    if (n_windows == 0) return AF_OK;
    return score_batches(net, y, ld_y, n, stride, n_windows, zero, 0, table, n_entries, logits, ws, ws_bytes, s);
}
}  // namespace afm

namespace {
// Switch a conv layer to candidate `idx`: a weight image in that candidate's
// layout replaces the layer's current one.
af_status switch_candidate(af_net* net, ConvOp& op, int idx) {
    ConvOp next = op;
    next.cand = idx;
    next.cfg = op.cands[idx];
    set_tiling(next);
    std::vector<unsigned char> img = build_image(next, next.cfg, net->prec, net->wfold, net->wscale);
    void* d_img = nullptr;
    if (hipMalloc(&d_img, img.size()) != hipSuccess ||
        hipMemcpy(d_img, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) {
        if (d_img) (void)hipFree(d_img);
        set_error("weight image upload failed");
        return AF_ENOMEM;
    }
    // a graph captured earlier may still launch the old image with the old
    // tiling (the same logits bit for bit): keep it until the net is destroyed
    net->retired.push_back(op.d_img);
    next.d_img = d_img;
    op = next;
    return AF_OK;
}
}  // namespace

extern "C" af_status af_net_autotune(af_net* net, int64_t batch, void* ws, size_t ws_bytes, af_stream stream,
                                     int64_t* n_changed) {
    clear_error();
    AF_CHECK_ARG(net && ws, "net and ws must be non-null");
    AF_CHECK_ARG(batch >= 1 && batch < (1LL << 24) && batch * net->act_elems < (1LL << 31), "bad batch size");
    AF_CHECK_ARG(ws_bytes >= af_score_workspace_bytes(net, batch), "workspace too small for batch %lld",
                 (long long)batch);
    int dev = -1;
    (void)hipGetDevice(&dev);
    AF_CHECK_ARG(dev == net->device, "net was created on device %d, current device is %d", net->device, dev);
    hipStream_t s = (hipStream_t)stream;
    const size_t bb = buf_bytes(net, batch);
    void* buf[3] = {ws, (char*)ws + bb, (char*)ws + 2 * bb};
    uint32_t* amax = net->prec == AF_FP8 ? (uint32_t*)((char*)ws + 3 * bb) : nullptr;
    // GroupNorm nets: statistics, then the scales and shifts the second conv
    // of a block reads (zero while timing)
    float* gn_stats = nullptr;
    const float* gn_aff0 = nullptr;
    if (net->gn_groups) {
        char* g0 = (char*)ws + 3 * bb + amax_bytes(net, batch);
        gn_stats = (float*)g0;
        gn_aff0 = (const float*)(g0 + gn_stats_bytes(net, batch));
        const int64_t gw = (int64_t)((gn_stats_bytes(net, batch) + gn_aff_bytes(net, batch)) / 4);
        hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((gw + 255) / 256)), dim3(256), 0, s, (uint32_t*)g0, gw, 0u);
    }
    // defined contents: activations zero, FP8 maxima 1.0
    const int64_t words = (int64_t)(3 * bb / 4);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, (uint32_t*)ws, words, 0u);
    if (amax) {
        const int64_t cnt = (int64_t)net->n_slots * batch;
        hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, amax, cnt, 0x3F800000u);
    }
    AF_LAUNCHED();
    hipEvent_t e0, e1;
    AF_HIP(hipEventCreate(&e0));
    AF_HIP(hipEventCreate(&e1));
    int64_t changed = 0;
    af_status result = AF_OK;
    if (net->fused_ok) {
        // rows per step of the whole-network kernel, timed in its steady
        // state: 256 windows per CU (tens per persistent workgroup, so the
        // last round's tail does not decide the ranking), read from the zeroed
        // workspace as a two-channel series (windows 64 samples apart; the
        // kernel's work per window does not depend on the data); fewer if the
        // workspace holds fewer
        const int64_t stride_t = 64, window = net->desc.window;
        const int64_t cap = (int64_t)(3 * bb / sizeof(float));
        int64_t nw_t = 256LL * net->n_cu;
        while (nw_t > 1 && 2 * ((nw_t - 1) * stride_t + window) + nw_t + 1 > cap) nw_t /= 2;
        const int64_t n = (nw_t - 1) * stride_t + window;
        FusedTinyArgs fa{};
        StemArgs& sa = fa.st;
        sa.y = (const float*)ws; sa.ld_y = n; sa.n = n; sa.stride = stride_t;
        sa.n_ch = 2; sa.window = net->desc.window;
        fa.wstem = net->d_sfused; fa.wconv = net->d_wfused; fa.bias = net->d_bfused; fa.fc = net->d_fc;
        fa.logits = (float*)ws + 2 * n; fa.n_windows = nw_t;
        fa.next = (unsigned int*)((float*)ws + 2 * n + nw_t);
        AF_CHECK_ARG((size_t)(2 * n + nw_t + 1) * sizeof(float) <= 3 * bb, "workspace too small for batch %lld",
                     (long long)batch);
        int best = net->fused_cand;
        float best_ms = 1e30f;
        for (int ci = 0; ci < (int)(sizeof(kFusedSteps) / sizeof(kFusedSteps[0])) && result == AF_OK; ++ci) {
            bool ok = launch_fused(ci, net->n_cu, fa, s);   // warm-up
            (void)hipEventRecord(e0, s);
            for (int rep = 0; rep < 3 && ok; ++rep) ok = launch_fused(ci, net->n_cu, fa, s);
            (void)hipEventRecord(e1, s);
            hipError_t err = ok ? hipEventSynchronize(e1) : hipGetLastError();
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess) {
                set_error("autotune: timing failed: %s", hipGetErrorString(err));
                result = AF_EHIP;
                break;
            }
            if (ms < best_ms) { best_ms = ms; best = ci; }
        }
        if (result == AF_OK && best != net->fused_cand) {
            net->fused_cand = best;
            ++changed;
        }
    }
    for (ConvOp& op : net->ops) {
        if (result != AF_OK) break;
        if (op.cands.size() < 2) continue;
        int best = op.cand;
        float best_ms = 1e30f;
        for (int ci = 0; ci < (int)op.cands.size() && result == AF_OK; ++ci) {
            ConvOp trial = op;
            trial.cfg = op.cands[ci];
            set_tiling(trial);
            std::vector<unsigned char> img = build_image(trial, trial.cfg, net->prec, net->wfold, net->wscale);
            void* d_img = nullptr;
            if (hipMalloc(&d_img, img.size()) != hipSuccess ||
                hipMemcpy(d_img, img.data(), img.size(), hipMemcpyHostToDevice) != hipSuccess) {
                if (d_img) (void)hipFree(d_img);
                set_error("autotune: weight image upload failed");
                result = AF_ENOMEM;
                break;
            }
            ConvArgs a{};
            a.in = buf[op.in_buf];
            a.out = buf[op.out_buf];
            a.res = op.res_buf >= 0 ? buf[op.res_buf] : nullptr;
            a.w = d_img;
            a.bias = net->d_b + op.b_off;
            a.wscale = net->d_ws ? net->d_ws + op.b_off : nullptr;
            a.amax_in = amax ? amax + (size_t)op.amax_in * batch : nullptr;
            a.amax_out = nullptr;   // keep the maxima at 1.0 while timing
            a.C_in = op.c_in; a.C_out = op.c_out; a.L_in = op.l_in; a.L_out = op.l_out;
            a.relu = op.relu; a.n_win = (int)batch;
            a.wpt = trial.wpt; a.tt = trial.tt; a.tiles_per_win = trial.tiles_per_win;
            a.gn_stats = gn_stats;
            a.in_aff = net->gn_groups && op.in_buf == BR ? gn_aff0 : nullptr;
            trial.cfg.fn(a, s);   // warm-up
            (void)hipEventRecord(e0, s);
            for (int rep = 0; rep < 3; ++rep) trial.cfg.fn(a, s);
            (void)hipEventRecord(e1, s);
            hipError_t err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            (void)hipFree(d_img);
            if (err != hipSuccess) {
                set_error("autotune: timing failed: %s", hipGetErrorString(err));
                result = AF_EHIP;
                break;
            }
            if (ms < best_ms) { best_ms = ms; best = ci; }
        }
        if (result != AF_OK) break;
        if (best != op.cand) {
            // the old image may still be read by work queued on another stream
            if (hipDeviceSynchronize() != hipSuccess) {
                set_error("autotune: device synchronisation failed");
                result = AF_EHIP;
                break;
            }
            result = switch_candidate(net, op, best);
            if (result != AF_OK) break;
            ++changed;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (n_changed) *n_changed = changed;
    return result;
}

extern "C" af_status af_net_layer_tile(const af_net* net, int64_t layer, int32_t* mt, int32_t* nt,
                                       int32_t* n_candidates, int32_t* chosen) {
    clear_error();
    AF_CHECK_ARG(net && mt && nt && n_candidates && chosen, "bad arguments");
    AF_CHECK_ARG(layer >= 1 && layer <= (int64_t)net->ops.size(), "layer must be a conv index in [1, %zu]",
                 net->ops.size());
    const ConvOp& op = net->ops[layer - 1];
    *mt = op.cfg.MT;
    *nt = op.cfg.NT;
    *n_candidates = (int32_t)op.cands.size();
    *chosen = op.cand;
    return AF_OK;
}

extern "C" af_status af_net_set_layer_tile(af_net* net, int64_t layer, int32_t chosen) {
    clear_error();
    AF_CHECK_ARG(net, "net must be non-null");
    AF_CHECK_ARG(layer >= 1 && layer <= (int64_t)net->ops.size(), "layer must be a conv index in [1, %zu]",
                 net->ops.size());
    ConvOp& op = net->ops[layer - 1];
    AF_CHECK_ARG(chosen >= 0 && chosen < (int32_t)op.cands.size(), "layer %lld has %zu tile candidates",
                 (long long)layer, op.cands.size());
    if (chosen == op.cand) return AF_OK;
    int dev = -1;
    (void)hipGetDevice(&dev);
    AF_CHECK_ARG(dev == net->device, "net was created on device %d, current device is %d", net->device, dev);
    AF_HIP(hipDeviceSynchronize());   // the old image may still be in use
    return switch_candidate(net, op, chosen);
}

extern "C" int64_t af_net_n_layers(const af_net* net) { return net ? (int64_t)net->layer_macs.size() : 0; }

extern "C" af_status af_net_profile_begin(af_net* net) {
    clear_error();
    AF_CHECK_ARG(net, "net must be non-null");
    drop_records(net);
    net->profiling = true;
    return AF_OK;
}

extern "C" af_status af_net_profile_end(af_net* net, int64_t n_layers, double* ms, int64_t* launches,
                                        double* flops) {
    clear_error();
    AF_CHECK_ARG(net, "net must be non-null");
    AF_CHECK_ARG(n_layers == (int64_t)net->layer_macs.size() && ms && launches && flops,
                 "need arrays of af_net_n_layers() = %zu entries", net->layer_macs.size());
    net->profiling = false;
    for (int64_t i = 0; i < n_layers; ++i) { ms[i] = 0.0; launches[i] = 0; flops[i] = 0.0; }
    for (auto& r : net->recs) {
        float t = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            set_error("reading profiling events failed");
            drop_records(net);
            return AF_EHIP;
        }
        ms[r.layer] += t;
        launches[r.layer] += 1;
        flops[r.layer] += 2.0 * (double)r.macs * (double)r.windows;
    }
    drop_records(net);
    return AF_OK;
}

extern "C" af_status af_net_calibrate(af_net* net, const float* y, int64_t n_ch, int64_t ld_y, int64_t n,
                                      int64_t stride, int64_t n_windows, void* ws, size_t ws_bytes,
                                      af_stream stream) {
    clear_error();
    AF_CHECK_ARG(net && y && ws, "net, y and ws must be non-null");
    AF_CHECK_ARG(net->prec == AF_FP8 && !net->gn_groups && !net->params_host.empty(),
                 "calibration applies to FP8 nets");
    AF_CHECK_ARG(n_ch == net->desc.in_ch, "n_ch %lld does not match the net's %d inputs", (long long)n_ch,
                 net->desc.in_ch);
    AF_CHECK_ARG(n >= 1 && ld_y >= n && stride >= 1 && n_windows >= 1 && n_windows < (1LL << 24),
                 "need n >= 1, ld_y >= n, stride >= 1, 1 <= n_windows < 2^24");
    AF_CHECK_ARG((n_windows - 1) * stride + net->desc.window <= n, "calibration window %lld ends past n = %lld",
                 (long long)(n_windows - 1), (long long)n);
    int dev = -1;
    (void)hipGetDevice(&dev);
    AF_CHECK_ARG(dev == net->device, "net was created on device %d, current device is %d", net->device, dev);
    hipStream_t s = (hipStream_t)stream;

    // the same network in FP32: its activations give the conv input means and
    // its logits the reference of the FC shift
    af_net* twin = nullptr;
    af_status st = create_net(&net->desc, 0, net->params_host.data(), (int64_t)net->params_host.size(), AF_F32,
                              &twin);
    if (st != AF_OK) return st;
    double* d_tap = nullptr;
    float* d_l = nullptr;
    auto done = [&](af_status r) {
        if (d_tap) (void)hipFree(d_tap);
        if (d_l) (void)hipFree(d_l);
        free_net(twin);
        return r;
    };
    if (ws_bytes < af_score_workspace_bytes(twin, 1)) {
        set_error("workspace too small: calibration needs at least %zu bytes", af_score_workspace_bytes(twin, 1));
        return done(AF_EINVAL);
    }
    const size_t pitch = (size_t)twin->tap_pitch, n_tap = net->ops.size() * pitch;
    if (hipMalloc(&d_tap, n_tap * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_l, 2 * (size_t)n_windows * sizeof(float)) != hipSuccess) {
        set_error("device allocation for calibration failed");
        return done(AF_ENOMEM);
    }
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((2 * n_tap + 255) / 256)), dim3(256), 0, s,
                       (uint32_t*)d_tap, (int64_t)(2 * n_tap), 0u);
    int64_t zero[4] = {0, 0, 0, 0};
    twin->d_tap = d_tap;
    st = score_batches(twin, y, ld_y, n, stride, n_windows, zero, 0, nullptr, 0, d_l, ws, ws_bytes, s);
    twin->d_tap = nullptr;
    if (st != AF_OK) return done(st);
    std::vector<double> sums(n_tap);
    if (hipMemcpyAsync(sums.data(), d_tap, n_tap * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("calibration: reading the input sums failed");
        return done(AF_EHIP);
    }

    // each conv's bias less (W_q - W') mu, FP64, from the weights as created
    std::vector<float> bias(net->bias64.size());
    for (size_t k = 0; k < net->ops.size(); ++k) {
        const ConvOp& op = net->ops[k];
        const double cnt = (double)n_windows * op.l_in;
        for (int o = 0; o < op.c_out; ++o) {
            const double sc = net->wscale[op.b_off + o];
            double shift = 0.0;
            for (int j = 0; j < op.kw; ++j)
                for (int c = 0; c < op.c_in; ++c) {
                    const double w = net->wfold[op.w_off + ((size_t)o * op.kw + j) * op.c_in + c];
                    const double q = std::min(448.0, std::max(-448.0, round_sig(w / sc, 4, -6, -9)));
                    shift += (q * sc - w) * (sums[k * pitch + c] / cnt);
                }
            bias[op.b_off + o] = (float)(net->bias64[op.b_off + o] - shift);
        }
    }
    const int C = net->last_C;
    float fcb = (float)net->fc_b64;
    // work already queued with this net on other streams reads the old biases
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(net->d_b, bias.data(), bias.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(net->d_fc + C, &fcb, sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("calibration: bias upload failed");
        return done(AF_EHIP);
    }
    // then the FC bias less the mean logit shift that remains
    st = score_batches(net, y, ld_y, n, stride, n_windows, zero, 0, nullptr, 0, d_l + n_windows, ws, ws_bytes, s);
    if (st != AF_OK) return done(st);
    std::vector<float> l(2 * (size_t)n_windows);
    if (hipMemcpyAsync(l.data(), d_l, l.size() * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_error("calibration: reading the logits failed");
        return done(AF_EHIP);
    }
    double d = 0.0;
    for (int64_t i = 0; i < n_windows; ++i) d += (double)l[n_windows + i] - (double)l[i];
    d /= (double)n_windows;
    fcb = (float)(net->fc_b64 - d);
    if (hipMemcpy(net->d_fc + C, &fcb, sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        set_error("calibration: bias upload failed");
        return done(AF_EHIP);
    }
    net->fc_b = fcb;
    return done(AF_OK);
}

extern "C" af_status af_net_fused_tile(const af_net* net, int32_t* rows, int32_t* n_candidates, int32_t* chosen) {
    clear_error();
    AF_CHECK_ARG(net && rows && n_candidates && chosen, "bad arguments");
    AF_CHECK_ARG(net->fused_ok, "this net has no whole-network kernel");
    *rows = kFusedSteps[net->fused_cand].rows;
    *n_candidates = (int32_t)(sizeof(kFusedSteps) / sizeof(kFusedSteps[0]));
    *chosen = net->fused_cand;
    return AF_OK;
}

extern "C" af_status af_net_set_fused_tile(af_net* net, int32_t chosen) {
    clear_error();
    AF_CHECK_ARG(net && net->fused_ok, "this net has no whole-network kernel");
    AF_CHECK_ARG(chosen >= 0 && chosen < (int32_t)(sizeof(kFusedSteps) / sizeof(kFusedSteps[0])),
                 "candidate %d out of range", (int)chosen);
    net->fused_cand = chosen;   // kernel arguments only: graphs captured earlier keep theirs
    return AF_OK;
}
