// Host-side Haar feature enumeration (Section 2.2).
//
// Type order 3h, 3v, 2h, 2v, 4 (the order in which Section 2.2 adds the
// per-type counts and Section 3.3.2 assigns feature groups).  Base cell grid
// (columns x rows): 3x1, 1x3, 2x1, 1x2, 2x2.  Cells are cw x ch pixels, scaled
// independently; index order type, cw, ch, y, x (x fastest).
#include <algorithm>
#include <vector>

#include "common.h"

namespace vjb {

static const int kBaseW[5] = {3, 1, 2, 1, 2};
static const int kBaseH[5] = {1, 3, 1, 2, 2};

bool valid_feature_set(const boost_feature_set* fs) {
    if (!fs) return false;
    if (fs->window_w < 1 || fs->window_w > kMaxWindow || fs->window_h < 1 || fs->window_h > kMaxWindow) return false;
    if (fs->type_mask == 0 || (fs->type_mask & ~BOOST_ALL_TYPES) != 0) return false;
    return true;
}

// Positions along one axis summed over all cell sizes: sum_c (L - b*c + 1).
static int64_t axis_sum(int L, int b) {
    int64_t s = 0;
    for (int c = 1; b * c <= L; ++c) s += L - b * c + 1;
    return s;
}

static int64_t type_count(int W, int H, int t) { return axis_sum(W, kBaseW[t]) * axis_sum(H, kBaseH[t]); }

int64_t host_feature_count(const boost_feature_set* fs) {
    if (!valid_feature_set(fs)) return -1;
    int64_t total = 0;
    for (int t = 0; t < 5; ++t)
        if (fs->type_mask & (1u << t)) total += type_count(fs->window_w, fs->window_h, t);
    return total;
}

int host_feature_desc(const boost_feature_set* fs, int64_t j, boost_feature* out) {
    const int W = fs->window_w, H = fs->window_h;
    for (int t = 0; t < 5; ++t) {
        if (!(fs->type_mask & (1u << t))) continue;
        const int64_t tc = type_count(W, H, t);
        if (j >= tc) { j -= tc; continue; }
        const int bw = kBaseW[t], bh = kBaseH[t];
        const int64_t sy = axis_sum(H, bh);
        for (int cw = 1; bw * cw <= W; ++cw) {
            const int64_t nx = W - bw * cw + 1;
            if (j >= nx * sy) { j -= nx * sy; continue; }
            for (int ch = 1; bh * ch <= H; ++ch) {
                const int64_t ny = H - bh * ch + 1;
                if (j >= nx * ny) { j -= nx * ny; continue; }
                out->type = t; out->cell_w = cw; out->cell_h = ch;
                out->y = (int32_t)(j / nx); out->x = (int32_t)(j % nx);
                return BOOST_OK;
            }
        }
    }
    return BOOST_E_INVALID;
}

void host_feature_table(const boost_feature_set* fs, uint32_t* out) {
    const int W = fs->window_w, H = fs->window_h;
    int64_t j = 0;
    for (int t = 0; t < 5; ++t) {
        if (!(fs->type_mask & (1u << t))) continue;
        const int bw = kBaseW[t], bh = kBaseH[t];
        for (int cw = 1; bw * cw <= W; ++cw)
            for (int ch = 1; bh * ch <= H; ++ch)
                for (int y = 0; y + bh * ch <= H; ++y)
                    for (int x = 0; x + bw * cw <= W; ++x) out[j++] = pack_feature(t, x, y, cw, ch);
    }
}

// Order in which the one-time preparation visits the features (each XCD
// runs a contiguous share of it).  Features whose corners lie on the same
// integral-image rows (types one cell high, and the 2x2 type: same y and
// cell height) or columns (types one cell wide: same x and cell width) are
// adjacent, so one XCD's L2 holds the corner planes a run of features reads
// (50 to 75 planes of n words for 24x24 windows).  The groups of the types
// are interleaved in proportion to the types' sizes, so every XCD's share
// has the same mix of feature types.
void host_sort_order(const uint32_t* ftab, int64_t F, uint32_t* order) {
    // group id: type, then (x, cw) or (y, ch) in 5 + 5 bits (cell sizes 1..32)
    constexpr int kKeys = 1 << 10;
    std::vector<int64_t> count(5 * kKeys, 0);
    std::vector<uint32_t> gid((size_t)F);
    int64_t type_total[5] = {0, 0, 0, 0, 0};
    for (int64_t j = 0; j < F; ++j) {
        int t, x, y, cw, ch;
        unpack_feature(ftab[j], t, x, y, cw, ch);
        const uint32_t key = kBaseW[t] == 1 ? (uint32_t)(x << 5 | (cw - 1)) : (uint32_t)(y << 5 | (ch - 1));
        gid[(size_t)j] = (uint32_t)(t * kKeys) + key;
        ++count[gid[(size_t)j]];
        ++type_total[t];
    }
    struct Group { double pos; uint32_t id; };
    std::vector<Group> groups;
    for (int t = 0; t < 5; ++t) {
        int64_t before = 0;
        for (int k = 0; k < kKeys; ++k) {
            const int64_t sz = count[(size_t)(t * kKeys + k)];
            if (sz == 0) continue;
            groups.push_back(Group{((double)before + 0.5 * (double)sz) / (double)type_total[t], (uint32_t)(t * kKeys + k)});
            before += sz;
        }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.pos < b.pos; });
    std::vector<int64_t> at(5 * kKeys, 0);
    int64_t p = 0;
    for (const Group& g : groups) { at[g.id] = p; p += count[g.id]; }
    for (int64_t j = 0; j < F; ++j) order[at[gid[(size_t)j]]++] = (uint32_t)j;
}

KeyGeom make_geom(int64_t n, int lanes) {
    KeyGeom g;
    g.n = n;
    g.nc = (n + 7) / 8;
    g.q = (int32_t)(g.nc / lanes);
    g.rem = (int32_t)(g.nc % lanes);
    g.row_units = (g.nc + 15) / 16 * 16;   // 256-byte aligned rows
    g.narrow = n <= kNarrowMaxN ? 1 : 0;
    g.lanes = lanes;
    return g;
}

int64_t ii_stride_of(int64_t n) { return (n + 63) / 64 * 64; }

}  // namespace vjb
