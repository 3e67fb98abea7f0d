// Bank-conflict-free gather schedule of the down pass (host, at problem
// creation).
//
// The down term of row u of X gathers, for every column d, the row's
// elements at the hop targets d' of the down sector (Eq. 1; the targets come
// from the forward map, Sec. III).  The pattern is the same for every row, so
// it is scheduled once.  The LDS holds each staged row as a plane whose
// element d' sits in bank d' mod 32, and a half-wave (32 lanes, 32 columns)
// reads without bank conflicts when its 32 addresses fall in 32 different
// banks.  For each group of 32 consecutive columns the hops form a bipartite
// multigraph lanes x banks (an edge per hop: lane d - 32 g, bank d' mod 32);
// a proper edge colouring with Delta colours (Delta = the largest lane or
// bank degree; Koenig's theorem, built edge by edge with alternating-path
// swaps) gives Delta steps in which every lane takes at most one hop and
// every bank serves at most one lane.  Lanes without a hop at a step read a
// zero from a pad of 32 words behind the plane, in a bank no lane uses at
// that step, and add nothing.
//
// Steps are grouped by hop magnitude (all steps of the smaller magnitude
// first, then the larger, each group a multiple of 4 steps), so the magnitude
// of a step is the same in every lane; its sign comes with the lane's entry.
// Entry (16 bits): the byte address of the target in its plane of
// kSchedPlane words (whose last 32 words are the zero pad), with bit 0 set
// when the hop's amplitude is minus the magnitude.  Layout: wave w (64
// columns, two groups) has S_w steps, the first B_w of the smaller magnitude;
// word i of a lane holds steps 2i (low half) and 2i + 1, and a lane's words
// are stored four at a time, words[off_w + q * 256 + lane * 4 + j] = word
// 4q + j, the last two of an odd number of pairs as words[off_w + q * 256 +
// lane * 2 + j].
#include <algorithm>
#include <cmath>
#include <vector>

#include "pdz_internal.h"

namespace pdz {

namespace {

// Edge colouring of one group: edges (lane, bank) -> colour, with `delta` colours.
std::vector<int> colour_group(const std::vector<std::pair<int, int>>& edges, int delta) {
    const int m = (int)edges.size();
    std::vector<int> col(m, -1);
    std::vector<int> at_lane(32 * delta, -1), at_bank(32 * delta, -1);   // edge holding a colour
    for (int e = 0; e < m; ++e) {
        const int u = edges[e].first, v = edges[e].second;
        int a = 0, b = 0;
        while (at_lane[u * delta + a] >= 0) ++a;   // free at the lane
        while (at_bank[v * delta + b] >= 0) ++b;   // free at the bank
        if (at_bank[v * delta + a] >= 0) {
            // a is taken at v: swap colours a and b along the alternating path
            // that starts at v with colour a (it cannot reach u)
            std::vector<int> path;
            int node = v, side = 1, c = a;   // side 1: bank, 0: lane
            while (true) {
                const int ed = side ? at_bank[node * delta + c] : at_lane[node * delta + c];
                if (ed < 0) break;
                path.push_back(ed);
                node = side ? edges[ed].first : edges[ed].second;
                side ^= 1;
                c = (c == a) ? b : a;
            }
            for (int ed : path) {   // unhook, then re-hook with the other colour
                at_lane[edges[ed].first * delta + col[ed]] = -1;
                at_bank[edges[ed].second * delta + col[ed]] = -1;
            }
            for (int ed : path) {
                col[ed] = (col[ed] == a) ? b : a;
                at_lane[edges[ed].first * delta + col[ed]] = ed;
                at_bank[edges[ed].second * delta + col[ed]] = ed;
            }
        }
        col[e] = a;
        at_lane[u * delta + a] = e;
        at_bank[v * delta + a] = e;
    }
    return col;
}

}  // namespace

pdz_status build_down_schedule(const SectorTables& t, const std::vector<double>& coef, DownSchedule* out,
                               hipStream_t s) {
    *out = DownSchedule{};
    const uint64_t D = t.D;
    // rows of at least 1024 elements (the wide down pass) that fit a plane
    if (D < 1024 || D + 32 > (uint64_t)kSchedPlane || t.max_hops == 0) return ok();
    const uint32_t P = kSchedPlane;   // words per plane, zero pad in the last 32
    // hop lists from the slot-major 32-bit table
    std::vector<uint32_t> ell((size_t)t.max_hops * D);
    std::vector<uint8_t> cnt(D);
    PDZ_HIP(hipMemcpyAsync(ell.data(), t.ell, ell.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PDZ_HIP(hipMemcpyAsync(cnt.data(), t.count, D, hipMemcpyDeviceToHost, s));
    PDZ_HIP(hipStreamSynchronize(s));
    // at most two hop magnitudes
    std::vector<double> mags;
    for (uint64_t d = 0; d < D; ++d)
        for (int h = 0; h < cnt[d]; ++h) {
            const double m = std::fabs(coef[ell[(size_t)h * D + d] >> kTargetBits]);
            if (std::find(mags.begin(), mags.end(), m) == mags.end()) mags.push_back(m);
            if (mags.size() > 2) return ok();
        }
    std::sort(mags.begin(), mags.end());
    if (mags.empty()) return ok();
    const int ncls = (int)mags.size();
    const uint64_t nwaves = (D + 63) / 64;
    std::vector<uint32_t> off(nwaves + 1, 0);
    std::vector<uint16_t> steps(nwaves, 0), split(nwaves, 0);
    std::vector<uint32_t> words;
    words.reserve(D * 24);
    for (uint64_t w = 0; w < nwaves; ++w) {
        // per magnitude class: the colouring of each half-wave, steps = max over the two halves
        std::vector<uint16_t> ent;   // [step][lane]
        int S = 0, B = 0;
        for (int cls = 0; cls < ncls; ++cls) {
            std::vector<std::pair<int, int>> edges[2];
            std::vector<uint16_t> val[2];
            int delta[2] = {0, 0};
            for (int half = 0; half < 2; ++half) {
                std::vector<int> ldeg(32, 0), bdeg(32, 0);
                for (int l = 0; l < 32; ++l) {
                    const uint64_t d = w * 64 + half * 32 + l;
                    if (d >= D) continue;
                    for (int h = 0; h < cnt[d]; ++h) {
                        const uint32_t e = ell[(size_t)h * D + d];
                        const double c = coef[e >> kTargetBits];
                        if ((std::fabs(c) == mags[0] ? 0 : 1) != cls) continue;
                        const uint32_t tg = e & kTargetMask;
                        edges[half].push_back({l, (int)(tg % 32)});
                        val[half].push_back((uint16_t)((tg << 1) | (c < 0.0 ? 1u : 0u)));   // target, sign
                        ++ldeg[l];
                        ++bdeg[tg % 32];
                    }
                }
                delta[half] = std::max(*std::max_element(ldeg.begin(), ldeg.end()),
                                       *std::max_element(bdeg.begin(), bdeg.end()));
            }
            int Sc = std::max(delta[0], delta[1]);
            Sc = (Sc + 3) & ~3;   // the kernel walks the steps four at a time
            const size_t base = ent.size() / 64;
            ent.resize((base + Sc) * 64);
            for (int half = 0; half < 2; ++half) {
                const std::vector<int> col = colour_group(edges[half], std::max(delta[half], 1));
                std::vector<int> at((size_t)std::max(Sc, 1) * 32, -1);   // edge of lane l at step t
                std::vector<uint32_t> used(std::max(Sc, 1), 0u);          // banks used at step t
                for (size_t e = 0; e < col.size(); ++e) {
                    at[(size_t)col[e] * 32 + edges[half][e].first] = (int)e;
                    used[col[e]] |= 1u << edges[half][e].second;
                }
                for (int st = 0; st < Sc; ++st) {
                    uint32_t freeb = ~used[st];
                    for (int l = 0; l < 32; ++l) {
                        const int e = at[(size_t)st * 32 + l];
                        uint16_t v;
                        if (e >= 0) {
                            v = (uint16_t)(((val[half][e] >> 1) << 2) | (val[half][e] & 1u));
                        } else {
                            const int b = __builtin_ctz(freeb);   // a bank no lane reads at this step
                            freeb &= freeb - 1u;
                            v = (uint16_t)((P - 32 + b) << 2);
                        }
                        ent[(base + st) * 64 + half * 32 + l] = v;
                    }
                }
            }
            if (cls == 0) B = Sc;
            S += Sc;
        }
        if (ncls == 1) B = S;
        if (S > kSchedMaxSteps) return ok();   // the kernel holds at most kSchedMaxSteps steps per wave
        // check: each half-wave step reads 32 different banks, and each column's
        // scheduled (target, sign, magnitude) triples are its hop list
        for (int half = 0; half < 2; ++half) {
            for (int st = 0; st < S; ++st) {
                uint32_t seen = 0u;
                for (int l = 0; l < 32; ++l) seen |= 1u << ((ent[(size_t)st * 64 + half * 32 + l] >> 2) % 32u);
                if (seen != 0xFFFFFFFFu) return fail(PDZ_EDEVICE, "gather schedule: a bank is read twice in one step");
            }
            for (int l = 0; l < 32; ++l) {
                const uint64_t d = w * 64 + half * 32 + l;
                std::vector<uint32_t> want, got;
                if (d < D)
                    for (int h = 0; h < cnt[d]; ++h) {
                        const uint32_t e = ell[(size_t)h * D + d];
                        const double c = coef[e >> kTargetBits];
                        const uint32_t cls = std::fabs(c) == mags[0] ? 0u : 1u;
                        want.push_back(((e & kTargetMask) << 2) | (c < 0.0 ? 1u : 0u) | (cls << 20));
                    }
                for (int st = 0; st < S; ++st) {
                    const uint16_t v = ent[(size_t)st * 64 + half * 32 + l];
                    if ((uint32_t)(v >> 2) < P - 32) got.push_back((uint32_t)v | ((st >= B ? 1u : 0u) << 20));
                    else if (v & 1u) return fail(PDZ_EDEVICE, "gather schedule: an idle lane carries a sign");
                }
                std::sort(want.begin(), want.end());
                std::sort(got.begin(), got.end());
                if (want != got) return fail(PDZ_EDEVICE, "gather schedule: a column's hops differ from its hop list");
            }
        }
        steps[w] = (uint16_t)S;
        split[w] = (uint16_t)B;
        off[w] = (uint32_t)words.size();
        // word i of lane l (steps 2i, 2i + 1): four words of a lane side by side (one 16-byte load),
        // the last two (when S / 2 is not a multiple of 4) as a pair
        const int nw = S / 2;
        auto word = [&](int i, int l) {
            return (uint32_t)ent[(size_t)(2 * i) * 64 + l] | ((uint32_t)ent[(size_t)(2 * i + 1) * 64 + l] << 16);
        };
        for (int q = 0; 4 * q < nw; ++q) {
            const int g = std::min(4, nw - 4 * q);
            for (int l = 0; l < 64; ++l)
                for (int j = 0; j < g; ++j) words.push_back(word(4 * q + j, l));
        }
    }
    off[nwaves] = (uint32_t)words.size();
    // per wave one record: word offset, then S | B << 16
    std::vector<uint32_t> meta(2 * nwaves);
    for (uint64_t w = 0; w < nwaves; ++w) {
        meta[2 * w] = off[w];
        meta[2 * w + 1] = (uint32_t)steps[w] | ((uint32_t)split[w] << 16);
    }
    PDZ_HIP(hipMalloc(&out->words, std::max<size_t>(1, words.size()) * sizeof(uint32_t)));
    PDZ_HIP(hipMalloc(&out->meta, meta.size() * sizeof(uint32_t)));
    PDZ_HIP(hipMemcpy(out->words, words.data(), words.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    PDZ_HIP(hipMemcpy(out->meta, meta.data(), meta.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    out->plane = P;
    out->mag0 = mags[0];
    out->mag1 = mags.size() > 1 ? mags[1] : mags[0];
    out->nwords = words.size();
    return ok();
}

void free_down_schedule(DownSchedule* sc) {
    if (sc->words) (void)hipFree(sc->words);
    if (sc->meta) (void)hipFree(sc->meta);
    *sc = DownSchedule{};
}

}  // namespace pdz
