// Host-side checks of the library's building, compression, serialization and key map,
// built with AddressSanitizer and UndefinedBehaviorSanitizer (no GPU, no HIP runtime):
// random pattern sets at every compression level are built, exported, walked over the
// exported records and compared with a brute-force match set, saved, loaded (the
// round trip must be exact) and loaded again after every truncation and many single-bit
// flips (each must be refused). Exit status 0 when every check holds.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pfac.h"
#include "scan_internal.h"

struct pfac_automaton;
namespace pfac {
// The host-only automata built here never reach a device.
void release_device_copies(pfac_automaton *) {}
size_t workspace_count(pfac_automaton *) { return 0; }
}  // namespace pfac

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(uint32_t n) {  // xorshift64*, then modulo
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32) % n;
}

static int fails = 0;
#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            fails++;                                                  \
        }                                                             \
    } while (0)

// Match set by definition: (start << 32 | id), sorted.
static std::vector<uint64_t> brute(const std::vector<std::vector<uint8_t>> &P, const std::vector<uint8_t> &T) {
    std::vector<uint64_t> out;
    for (size_t s = 0; s < T.size(); s++)
        for (size_t j = 0; j < P.size(); j++)
            if (s + P[j].size() <= T.size() && memcmp(&T[s], P[j].data(), P[j].size()) == 0)
                out.push_back(((uint64_t)s << 32) | j);
    return out;
}

// Walk every start over the exported records (Eq. 1, ids by rank; see pfac.h).
static std::vector<uint64_t> walk(pfac_automaton *a, uint32_t alphabet, const std::vector<uint8_t> &T) {
    pfac_table_info_t info;
    pfac_table_info(a, &info);
    const uint32_t R = info.table_records, W = (alphabet + 31) / 32, S = info.shared_base;
    std::vector<uint32_t> first(R), bm((size_t)R * W), rank(R), rf(info.n_patterns + 1), ri(info.n_patterns + 1);
    std::vector<uint8_t> term(R);
    CHECK(pfac_export_records(a, first.data(), bm.data(), term.data(), rank.data(), R) == PFAC_OK);
    CHECK(pfac_export_rank_ids(a, rf.data(), rf.size(), ri.data(), ri.size()) == PFAC_OK);
    std::vector<uint64_t> out;
    for (size_t s = 0; s < T.size(); s++) {
        uint32_t q = 0, u = 0, add = 0;
        for (size_t i = s; i < T.size(); i++) {
            const uint32_t c = T[i];
            if (c >= alphabet || !((bm[(size_t)q * W + c / 32] >> (c % 32)) & 1)) break;
            uint32_t below = 0;
            for (uint32_t w = 0; w < c / 32; w++) below += __builtin_popcount(bm[(size_t)q * W + w]);
            below += __builtin_popcount(bm[(size_t)q * W + c / 32] & ((1u << (c % 32)) - 1u));
            const uint32_t y = first[q] + below;
            CHECK(y < R);
            if (y >= R) break;
            if (y < S) u = y;
            else add += term[q] + rank[y];
            q = y;
            if (term[q]) {
                const uint32_t r = q < S ? rank[q] : rank[u] + add;
                CHECK(r + 1 < rf.size());
                if (r + 1 >= rf.size()) break;
                for (uint32_t x = rf[r]; x < rf[r + 1]; x++) out.push_back(((uint64_t)s << 32) | ri[x]);
            }
        }
    }
    std::sort(out.begin(), out.end());
    return out;
}

// packet_end (the packet-batch walks' end) against a linear search, on offsets held in
// an array of exactly n_packets + 1 words (the sanitizer sees any read past it), also
// for offsets that end before the batch's bytes (positions past the last offset).
static void check_packet_end() {
    for (int trial = 0; trial < 200; trial++) {
        const uint32_t np = rnd(12);
        uint64_t *off = new uint64_t[np + 1];
        off[0] = 0;
        for (uint32_t i = 1; i <= np; i++) off[i] = off[i - 1] + rnd(5);  // empty packets too
        const uint64_t n = off[np] + rnd(6);  // bytes may run past the last offset
        for (uint64_t s = 0; s < n + 2; s++) {
            uint64_t want = off[np];
            for (uint32_t i = 0; i < np; i++)
                if (off[i + 1] > s) {
                    want = off[i + 1];
                    break;
                }
            CHECK(pfac::packet_end(off, np, s) == want);
        }
        delete[] off;
    }
}

int main() {
    check_packet_end();
    const uint32_t alphabets[] = {2, 4, 26, 256};
    const uint32_t levels[] = {0, 1, 3, 255};
    for (int trial = 0; trial < 48; trial++) {
        const uint32_t alphabet = alphabets[trial % 4];
        const uint32_t n = 1 + rnd(60);
        std::vector<std::vector<uint8_t>> P(n);
        std::vector<uint8_t> bytes;
        std::vector<uint64_t> off{0};
        for (auto &p : P) {
            p.resize(1 + rnd(9));
            for (auto &c : p) c = (uint8_t)rnd(alphabet);
            bytes.insert(bytes.end(), p.begin(), p.end());
            off.push_back(bytes.size());
        }
        std::vector<uint8_t> T(300 + rnd(300));
        for (auto &c : T) c = (uint8_t)rnd(alphabet < 256 ? alphabet + 1 : 256);
        for (int k = 0; k < 10; k++) {  // plants
            const auto &p = P[rnd(n)];
            const size_t o = rnd((uint32_t)(T.size() - p.size()));
            std::copy(p.begin(), p.end(), T.begin() + o);
        }
        const std::vector<uint64_t> want = brute(P, T);
        for (uint32_t lv : levels) {
            pfac_build_options opt{};
            opt.merge_levels = lv;
            pfac_automaton *a = nullptr;
            CHECK(pfac_build_ex(bytes.data(), off.data(), n, alphabet, &opt, &a) == PFAC_OK);
            if (!a) continue;
            CHECK(walk(a, alphabet, T) == want);
            uint64_t size = 0;
            CHECK(pfac_save(a, nullptr, 0, &size) == PFAC_ECAPACITY);
            std::vector<uint8_t> blob(size);
            CHECK(pfac_save(a, blob.data(), size, &size) == PFAC_OK);
            pfac_automaton *b = nullptr;
            CHECK(pfac_load(blob.data(), blob.size(), &b) == PFAC_OK);
            if (b) {
                CHECK(walk(b, alphabet, T) == want);
                uint64_t size2 = 0;
                std::vector<uint8_t> blob2(size);
                CHECK(pfac_save(b, blob2.data(), size, &size2) == PFAC_OK && blob2 == blob);
                pfac_destroy(b);
            }
            // every truncation, then single-bit flips: refused, nothing read out of bounds
            for (size_t cut = 0; cut < blob.size(); cut += (trial % 3 == 0 ? 1 : 7)) {
                std::vector<uint8_t> part(blob.begin(), blob.begin() + cut);
                part.reserve(1);  // a valid pointer also at size 0
                pfac_automaton *c = nullptr;
                CHECK(pfac_load(part.data(), part.size(), &c) == PFAC_EFORMAT && !c);
            }
            for (int f = 0; f < 64; f++) {
                std::vector<uint8_t> bad = blob;
                bad[rnd((uint32_t)bad.size())] ^= (uint8_t)(1u << rnd(8));
                pfac_automaton *c = nullptr;
                CHECK(pfac_load(bad.data(), bad.size(), &c) == PFAC_EFORMAT && !c);
            }
            pfac_destroy(a);
        }
        // key map over a random packet split of the text
        std::vector<uint64_t> po{0};
        while (po.back() < T.size()) po.push_back(std::min<uint64_t>(T.size(), po.back() + rnd(40)));
        std::vector<uint64_t> keys;
        for (int k = 0; k < 50; k++) keys.push_back(((uint64_t)rnd((uint32_t)T.size()) << 32) | rnd(1000));
        std::vector<uint32_t> pk(keys.size()), st(keys.size()), id(keys.size());
        CHECK(pfac_key_to_packet(keys.data(), keys.size(), po.data(), (uint32_t)po.size() - 1, pk.data(), st.data(),
                                 id.data()) == PFAC_OK);
        for (size_t k = 0; k < keys.size(); k++) {
            const uint64_t s = keys[k] >> 32;
            CHECK(po[pk[k]] <= s && s < po[pk[k] + 1] && po[pk[k]] + st[k] == s && id[k] == (uint32_t)keys[k]);
        }
    }
    if (fails) {
        fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    printf("host sanitize: all checks passed\n");
    return 0;
}
