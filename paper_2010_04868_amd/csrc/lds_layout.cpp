// LDS padding of the time-skewed nD band kernel, chosen by simulating its
// LDS address streams against the bank structure.
//
// Bank model of gfx950's LDS, as measured with SQ_LDS_BANK_CONFLICT on
// in-bounds access patterns: an LDS instruction is served a group of lanes
// per cycle, in lane order, and two lanes of one group conflict when their
// element indices are equal modulo the group's slot count but the elements
// differ (equal elements broadcast); conflicting lanes serialise.
//   ds_read_b64          32 lanes per cycle, slot = element mod 32
//   ds_write_b64         16 lanes per cycle, slot = element mod 16
//   ds_read/write_b32    32 lanes per cycle, slot = element mod 32
// The kernel's layout has two free paddings: the sub-row stride S (distance
// between the C sub-rows of a plane row, the transposed layout) and the
// plane stride PSP (distance between the LDS planes of successive time
// levels).  For every candidate
// pair this file replays, for every wave of a workgroup, the addresses the
// kernel computes (level-plane reads and writes of the lanes, staging writes
// of level 0 and staging reads of level k) and keeps the pair with the
// fewest LDS cycles.  The replay mirrors the index arithmetic of tstp_tile
// in tstp_nd.hpp; a change there must be made here too.
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "tstp_nd.hpp"

namespace tvs {
namespace nd {

namespace {

struct BankRule {
    int lanes, slots;
};
BankRule read_rule(int) { return {32, 32}; }
BankRule write_rule(int eb) { return eb == 8 ? BankRule{16, 16} : BankRule{32, 32}; }
constexpr int kPeriod = 32;  // paddings repeat their bank behaviour with this period

// An LDS address as a linear form in the two paddings: a = cs*S + cp*PSP + c0.
struct Lin {
    int cs, cp, c0;
    bool operator==(const Lin& o) const { return cs == o.cs && cp == o.cp && c0 == o.c0; }
};

// The accesses of one workgroup, cut into LDS cycles: each cycle holds the
// distinct address forms of the lanes it serves (equal forms broadcast) and
// a weight (how often the kernel issues that access per step).
struct Access {
    std::vector<std::vector<Lin>> cycles;
    std::vector<int> weight;
    std::vector<int> slots;
};

Access replay(int D, bool box, int eb, int C, int W, int H, int k, int lanemap, int NT,
              int G) {
    const int Gx = W / C;
    const int R = D == 3 ? 3 : 1, MID = D == 3 ? 1 : 0;
    const int nwaves = (NT + 63) / 64;
    const int PS = H * W;
    const int npt = (PS + NT - 1) / NT;
    Access acc;
    // one wave-wide instruction: lane l's form, or nothing if inactive
    auto emit = [&](const std::vector<std::pair<bool, Lin>>& lanes, int weight, BankRule rule) {
        const size_t lpc = (size_t)rule.lanes;
        for (size_t c0 = 0; c0 < lanes.size(); c0 += lpc) {
            std::vector<Lin> u;
            for (size_t l = c0; l < c0 + lpc && l < lanes.size(); ++l) {
                if (!lanes[l].first) continue;
                bool dup = false;
                for (auto& x : u) dup = dup || x == lanes[l].second;
                if (!dup) u.push_back(lanes[l].second);
            }
            if (!u.empty()) {
                acc.cycles.push_back(u);
                acc.weight.push_back(weight);
                acc.slots.push_back(rule.slots);
            }
        }
    };
    auto lane_jg = [&](int tid, int* j, int* g) {
        if (lanemap == 0) {
            *j = 1 + tid % k;
            *g = tid / k;
        } else {
            *j = 1 + tid / G;
            *g = tid % G;
        }
    };
    std::vector<std::pair<bool, Lin>> lanes(64);
    for (int w = 0; w < nwaves; ++w) {
        // lane reads of the level-(j-1) plane: (j-1)*PSP + ly*Wp + r*Wp + pos
        for (int r = 0; r < R; ++r)
            for (int i = 0; i < C + 2; ++i) {
                if (!(box || r == MID || (i >= 1 && i <= C))) continue;
                for (int l = 0; l < 64; ++l) {
                    const int tid = w * 64 + l;
                    lanes[l].first = tid < NT;
                    if (tid >= NT) continue;
                    int j, g;
                    lane_jg(tid, &j, &g);
                    const int ly = D == 3 ? g / Gx : 0, gx = g - ly * Gx;
                    Lin a{C * (ly + r), j - 1, 0};
                    if (i == 0) {
                        a.cs += C - 1;
                        a.c0 += gx;
                    } else if (i <= C) {
                        a.cs += i - 1;
                        a.c0 += gx + 1;
                    } else {
                        a.c0 += gx + 2;
                    }
                    lanes[l].second = a;
                }
                emit(lanes, 1, read_rule(eb));
            }
        // lane writes of the level-j plane: j*PSP + (ly+1)*Wp (3D) + gx + 1 + c*S
        for (int c = 0; c < C; ++c) {
            for (int l = 0; l < 64; ++l) {
                const int tid = w * 64 + l;
                lanes[l].first = tid < NT;
                if (tid >= NT) continue;
                int j, g;
                lane_jg(tid, &j, &g);
                const int ly = D == 3 ? g / Gx : 0, gx = g - ly * Gx;
                lanes[l].second = Lin{(D == 3 ? C * (ly + 1) : 0) + c, j, gx + 1};
            }
            emit(lanes, 1, write_rule(eb));
        }
        // staging: level-0 writes and level-k reads use the same addresses
        // (every thread reads for the level-k store, also without an element)
        for (int i = 0; i < npt; ++i) {
            for (int l = 0; l < 64; ++l) {
                const int tid = w * 64 + l;
                const int e = tid + i * NT;
                lanes[l].first = tid < NT && e < PS;
                if (!lanes[l].first) continue;
                const int yl = D == 3 ? e / W : 0, xl = e - yl * W;
                lanes[l].second = Lin{(D == 3 ? C * (yl + 1) : 0) + xl % C, 0, xl / C + 1};
            }
            emit(lanes, 1, write_rule(eb));
            emit(lanes, 1, read_rule(eb));
        }
    }
    return acc;
}

// LDS cycles of all accesses for one choice of paddings.
int64_t cost(const Access& acc, int S, int PSP) {
    int64_t total = 0;
    int count[64];
    for (size_t c = 0; c < acc.cycles.size(); ++c) {
        const int slots = acc.slots[c];
        for (int q = 0; q < slots; ++q) count[q] = 0;
        int deg = 0;
        for (const Lin& a : acc.cycles[c]) {
            const int64_t addr = (int64_t)a.cs * S + (int64_t)a.cp * PSP + a.c0;
            deg = std::max(deg, ++count[addr % slots]);
        }
        total += (int64_t)deg * acc.weight[c];
    }
    return total;
}

std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int, int, int, int, int>, LdsLayout> g_cache;

}  // namespace

LdsLayout lds_layout(int D, bool box, int eb, int C, int W, int H, int k, int lanemap, int NT,
                     int G) {
    const auto key = std::make_tuple(D, (int)box, eb, C, W, H, k, lanemap, NT);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_cache.find(key);
        if (it != g_cache.end()) return it->second;
    }
    const Access acc = replay(D, box, eb, C, W, H, k, lanemap, NT, G);
    const int Gx = W / C;
    const int period = kPeriod;
    // Padding must not cost occupancy: workgroups per CU are limited by waves
    // (four per SIMD at the kernel's register use) and by LDS; keep only
    // layouts that fit as many workgroups as the unpadded one.
    const int planes = 2 * (k + 1);
    const int by_waves = std::max(1, 16 / ((NT + 63) / 64));
    auto occupancy = [&](int PSP) {
        const int64_t bytes = (int64_t)planes * PSP * eb;
        return (int)std::min<int64_t>(by_waves, (160 * 1024) / std::max<int64_t>(bytes, 1));
    };
    auto plane_base = [&](int S) { return D == 3 ? (H + 2) * C * S : C * S; };
    const int occ0 = occupancy(plane_base(Gx + 2));
    LdsLayout best{Gx + 2, C * (Gx + 2), plane_base(Gx + 2)};
    int64_t best_cost = -1;
    // S >= Gx + 2 (a pad column on each side of every sub-row); PSP >= the
    // plane's extent.  One bank period of candidates for each is enough.
    for (int S = Gx + 2; S < Gx + 2 + period; ++S) {
        const int base = plane_base(S);
        for (int PSP = base; PSP < base + period; ++PSP) {
            if (occupancy(PSP) < occ0) break;
            const int64_t c = cost(acc, S, PSP);
            if (best_cost < 0 || c < best_cost) {
                best_cost = c;
                best = LdsLayout{S, C * S, PSP};
            }
        }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache[key] = best;
    return best;
}

}  // namespace nd
}  // namespace tvs
