// Launch planning of one pair-sum evaluation: the launch shape (waves per
// workgroup, split groups per target tile) and the workspace carve-up.  Kept
// apart from the C ABI so that the pair kernels' sources and their planner
// can be fingerprinted together.
#include "s2d_internal.h"

#include <algorithm>
#include <cstdlib>

namespace s2d {

namespace {
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

size_t rec_bytes(int op, int mode) {
    if (slp_sources(op)) return mode == S2D_FP64 ? sizeof(RecSlp64) : sizeof(RecSlp32);
    return mode == S2D_FP64 ? sizeof(RecDlp64) : sizeof(RecDlp32);
}

Plan make_plan(int op, int mode, const s2d_curves *s, const s2d_targets *t, int cus) {
    Plan p{};
    p.op = op;
    p.mode = mode;
    p.tpt = 1;
    // Launch shape: one target tile (64 targets) per workgroup of W waves,
    // each wave a source split, and G split groups (workgroups) per tile.
    // G = 1 when the source records fit comfortably in one XCD's L2 (4 MB)
    // and the tiles alone give at least two rounds of 8 waves per SIMD;
    // otherwise G grows to fill the chip (few targets, many sources), and is
    // a multiple of 8 when the records exceed the L2 budget, so that every
    // XCD streams only its own groups' sources.  S2D_WAVES and S2D_GROUPS
    // override the shape for tuning sweeps.
    static const int env_waves = [] {
        const char *e = std::getenv("S2D_WAVES");
        const int v = e ? std::atoi(e) : 0;
        return (v >= 1 && v <= kMaxPairWaves) ? v : 0;
    }();
    static const int env_groups = [] {
        const char *e = std::getenv("S2D_GROUPS");
        return e ? std::max(0, std::atoi(e)) : 0;
    }();
    constexpr size_t kL2Budget = (size_t)3 << 20;
    p.n_src = s->n_nodes;
    p.n_trg = t->n;
    p.n_sb = (p.n_src + kSuperBlock - 1) / kSuperBlock;
    p.n_tiles = (p.n_trg + kWave - 1) / kWave;
    if (p.n_sb > 0 && p.n_tiles > 0) {
        const bool fits = (size_t)p.n_sb * kSuperBlock * rec_bytes(op, mode) <= kL2Budget;
        const int64_t fill = (int64_t)cus * 4 * 16;
        const int64_t gmax = std::max<int64_t>(1, (p.n_sb + 7) / 8);
        int64_t G = 1;
        if (!(fits && p.n_tiles * kMaxPairWaves >= fill))
            G = std::min<int64_t>(std::max<int64_t>(1, (fill + p.n_tiles * kMaxPairWaves - 1) /
                                                           (p.n_tiles * kMaxPairWaves)), gmax);
        if (!fits && gmax >= 8) G = std::min<int64_t>((std::max<int64_t>(G, 8) + 7) / 8 * 8, gmax / 8 * 8);
        G = std::min<int64_t>(G, 65536);
        if (env_groups) G = std::min<int64_t>(env_groups, p.n_sb);
        // W: the full width, or fewer when the group has fewer superblocks.
        int W = (int)std::min<int64_t>(kMaxPairWaves, (p.n_sb + G - 1) / G);
        if (env_waves) W = env_waves;
        p.waves = W;
        p.n_groups = (int)G;
        p.n_splits = (int)(W * G);
        p.sb_per_split = (p.n_sb + p.n_splits - 1) / p.n_splits;
        p.n_blocks = p.n_tiles * G;
    } else {
        p.waves = 1;
        p.n_groups = 1;
        p.sb_per_split = 0;
        p.n_splits = 0;
        p.n_blocks = 0;
    }
    p.self = false;    // set by the caller once images are known
    size_t off = 0;
    p.off_rec = off;
    off = align256(off + (size_t)p.n_sb * kSuperBlock * rec_bytes(op, mode));
    p.off_rec64 = off;
    if (mode == S2D_FP32C && s2d::near_fp64(op))
        off = align256(off + (size_t)p.n_sb * kSuperBlock * rec_bytes(op, S2D_FP64));
    p.off_sub = off;
    if (mode == S2D_FP32C)
        off = align256(off + (size_t)p.n_sb * (kSuperBlock / kSubBlock) * sizeof(s2d::SubInfo));
    p.off_sbsum = off;
    if (op == S2D_OP_SLP && mode == S2D_FP32C) off = align256(off + (size_t)p.n_sb * 2 * sizeof(double));
    p.off_part = off;
    if (p.n_groups > 1) off = align256(off + (size_t)p.n_groups * 2 * (size_t)p.n_trg * sizeof(double));
    p.off_self = off;
    p.off_kress = off;
    if (op == S2D_OP_SLP && t->on_curve && p.n_trg > 0) {
        off = align256(off + 2 * (size_t)p.n_trg * sizeof(double));
        p.off_kress = off;
        off = align256(off + (size_t)p.n_src * sizeof(double));
    }
    p.total = off;
    return p;
}

}  // namespace s2d
