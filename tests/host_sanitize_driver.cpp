// Exercise the library's host-only code (paper_2002_02503_amd/csrc/host.cpp)
// on synthetic inputs, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer (tests/test_host_sanitizers.py): lattice tables,
// argument checks (every limit, and values at the edges of the integer
// types), the two-step kernel's fit rules, checkpoint header checks (short, foreign and mismatched buffers),
// the layout rearrangement of a state (every lattice and layout, degenerate
// boxes included, checked to be a permutation that round-trips), and the tune
// cache (malformed lines).  Any sanitizer report exits non-zero; a failed
// expectation exits 2.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "host.hpp"

using namespace lbm;

static int g_fail = 0;
#define EXPECT(cond)                                                              \
    do {                                                                          \
        if (!(cond)) {                                                            \
            std::fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
            g_fail = 1;                                                           \
        }                                                                         \
    } while (0)

static bool boxes_ok(int lat, int dtype, std::vector<int64_t> dims, std::vector<double> tau, std::string* why)
{
    LatticeInfo L;
    if (!lattice_info(lat, &L)) return false;
    return check_boxes(L, dtype, int(tau.size()), dims.data(), tau.data(), why);
}

static void test_tables()
{
    for (int lat = 0; lat < 4; ++lat) {
        LatticeInfo L;
        EXPECT(lattice_info(lat, &L));
        EXPECT(int(L.c.size()) == 3 * L.Q && int(L.w.size()) == L.Q && int(L.mrow.size()) == L.Q);
        double sw = 0;
        std::vector<int> seen(L.Q, 0);
        for (int i = 0; i < L.Q; ++i) {
            sw += L.w[i];
            EXPECT(L.mrow[i] >= 0 && L.mrow[i] < L.Q);
            if (L.mrow[i] >= 0 && L.mrow[i] < L.Q) seen[L.mrow[i]]++;
        }
        for (int m = 0; m < L.Q; ++m) EXPECT(seen[m] == 1);
        EXPECT(sw > 1 - 1e-12 && sw < 1 + 1e-12);
    }
    LatticeInfo L;
    EXPECT(!lattice_info(-1, &L) && !lattice_info(4, &L) && !lattice_info(std::numeric_limits<int>::max(), &L));
    EXPECT(storage_bytes(0) == 8 && storage_bytes(1) == 4 && storage_bytes(2) == 2 && storage_bytes(3) == 2);
    EXPECT(storage_bytes(-1) == 0 && storage_bytes(4) == 0);
}

static void test_checks()
{
    std::string why;
    const int64_t big = std::numeric_limits<int64_t>::max();
    const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
    EXPECT(boxes_ok(1, 1, {8, 8, 8}, {0.6}, &why));
    EXPECT(boxes_ok(0, 0, {64, 64, 1}, {0.8}, &why));
    EXPECT(boxes_ok(1, 1, {64, 64, 64, 16, 17, 18}, {0.6, 0.9}, &why));
    struct Bad {
        int lat, dtype;
        std::vector<int64_t> dims;
        std::vector<double> tau;
    };
    const std::vector<Bad> bad = {
        {1, 1, {0, 8, 8}, {0.6}},
        {1, 1, {8, -1, 8}, {0.6}},
        {1, 1, {big, 8, 8}, {0.6}},
        {1, 1, {8, big, big}, {0.6}},
        {1, 1, {std::numeric_limits<int64_t>::min(), 1, 1}, {0.6}},
        {1, 1, {1, 65535, 65535}, {0.6}},
        {1, 1, {1, 65536, 1}, {0.6}},
        {1, 1, {1, 1, 65536}, {0.6}},
        {1, 1, {8, 8, 8}, {0.5}},
        {1, 1, {8, 8, 8}, {nan}},
        {1, 1, {8, 8, 8}, {inf}},
        {1, 1, {8, 8, 8}, {-inf}},
        {0, 1, {8, 8, 2}, {0.6}},
        {0, 0, {1 << 28, 1, 1}, {0.6}},
        {1, 2, {1 << 20, 256, 65535}, {0.6}},
        {1, 1, {1 << 20, 1 << 20, 1}, {0.6}},
        {1, 0, {1024, 1024, 14, 8, 8, 8}, {0.6, 0.7}},
        {1, 0, {(1 << 21) + 1, 1, 1, 8, 8, 8}, {0.6, 0.7}},
        {1, 1, {8, 8, 8, 8, 0, 8}, {0.6, 0.7}},
        {1, 1, {INT32_MAX, INT32_MAX, 1, INT32_MAX, INT32_MAX, 1}, {0.6, 0.6}},
    };
    for (const Bad& b : bad) {
        why.clear();
        EXPECT(!boxes_ok(b.lat, b.dtype, b.dims, b.tau, &why));
        EXPECT(!why.empty());
    }
    EXPECT(geometry_hash({8, 8, 8}) != geometry_hash({8, 8, 9}));
    EXPECT(geometry_hash({}) == geometry_hash({}));
}

static void test_two_step_fits()
{
    // lattice codes: 0 D2Q9, 1 D3Q19, 2 D3Q39, 3 D3Q15; dtype codes: 0 FP64 .. 3 BF16
    LatticeInfo q9, q19, q39, q15;
    lattice_info(0, &q9);
    lattice_info(1, &q19);
    lattice_info(2, &q39);
    lattice_info(3, &q15);
    const int64_t big = std::numeric_limits<int64_t>::max();
    for (int dtype = 0; dtype < 4; ++dtype) {
        EXPECT(two_step_fits(q19, dtype, 256, 256, 256));
        EXPECT(two_step_fits(q15, dtype, 64, 8, 1));
        EXPECT(!two_step_fits(q9, dtype, 64, 64, 1));
        EXPECT(!two_step_fits(q39, dtype, 64, 64, 64));
        EXPECT(!two_step_fits(q19, dtype, 96, 32, 4));   // nx not a multiple of 64
        EXPECT(!two_step_fits(q19, dtype, 64, 6, 4));    // ny not a multiple of 4
        EXPECT(!two_step_fits(q19, dtype, 0, 16, 4));
        EXPECT(!two_step_fits(q19, dtype, 64, 16, 0));
        EXPECT(!two_step_fits(q19, dtype, -64, 16, 4));
        EXPECT(!two_step_fits(q19, dtype, big, big, big));
        EXPECT(!two_step_fits(q19, dtype, 64, int64_t(1) << 40, 1));
    }
    EXPECT(two_step_fits(q19, 0, 64, 12, 3));    // FP64 tile: 64 x 4
    EXPECT(!two_step_fits(q19, 1, 64, 12, 3));   // FP32 tile: 64 x 8
    EXPECT(!two_step_fits(q19, 4, 64, 16, 3));   // unknown dtype
    // one z-plane of populations must stay below 2 GiB: Q nx ny elem < 2^31
    EXPECT(two_step_fits(q19, 1, 8192, 3440, 1));    // 19 * 8192 * 3440 * 4 = 2141 MB < 2^31
    EXPECT(!two_step_fits(q19, 1, 8192, 3456, 1));   // 19 * 8192 * 3456 * 4 > 2^31
    EXPECT(!two_step_fits(q19, 0, 8192, 3440, 1));
}

static void test_checkpoint()
{
    CkptHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    hd.magic = kCkptMagic;
    hd.lattice = 1;
    hd.dtype = 1;
    hd.K = 3;
    hd.nbox = 1;
    hd.nsites = 512;
    hd.t = 7;
    hd.geometry_hash = geometry_hash({8, 8, 8});
    hd.payload_bytes = 512 * 19 * 4;
    std::vector<char> buf(sizeof(hd) + hd.payload_bytes, 0);
    std::memcpy(buf.data(), &hd, sizeof(hd));
    std::string why;
    EXPECT(check_checkpoint(buf.data(), buf.size(), hd, &why));
    EXPECT(!check_checkpoint(nullptr, buf.size(), hd, &why));
    for (size_t n : {size_t(0), size_t(1), sizeof(hd) - 1, sizeof(hd), buf.size() - 1}) {
        // a short buffer is rejected before its bytes are read
        std::vector<char> part(buf.begin(), buf.begin() + long(n));
        EXPECT(!check_checkpoint(part.empty() ? nullptr : part.data(), n, hd, &why));
    }
    auto mutated = [&](auto&& change) {
        CkptHeader m = hd;
        change(m);
        std::vector<char> b2 = buf;
        std::memcpy(b2.data(), &m, sizeof(m));
        return check_checkpoint(b2.data(), b2.size(), hd, &why);
    };
    EXPECT(!mutated([](CkptHeader& m) { m.magic ^= 1; }));
    EXPECT(!mutated([](CkptHeader& m) { m.lattice = 2; }));
    EXPECT(!mutated([](CkptHeader& m) { m.dtype = 0; }));
    EXPECT(!mutated([](CkptHeader& m) { m.K = 2; }));
    EXPECT(!mutated([](CkptHeader& m) { m.nbox = 2; }));
    EXPECT(!mutated([](CkptHeader& m) { m.nsites = -1; }));
    EXPECT(!mutated([](CkptHeader& m) { m.geometry_hash ^= 1; }));
    EXPECT(!mutated([](CkptHeader& m) { m.payload_bytes = ~uint64_t(0); }));
    EXPECT(!mutated([](CkptHeader& m) { m.t = -5; }));
    EXPECT(mutated([](CkptHeader& m) { m.t = 123456789; }));
}

static void test_relayout()
{
    const int64_t shapes[][3] = {{1, 1, 1}, {2, 3, 1}, {1, 2, 3}, {5, 3, 2}, {7, 4, 3}, {3, 1, 5}};
    for (int lat = 0; lat < 4; ++lat) {
        LatticeInfo L;
        lattice_info(lat, &L);
        for (const auto& s : shapes) {
            if (L.D == 2 && s[2] != 1) continue;
            for (size_t elem : {size_t(2), size_t(4), size_t(8)}) {
                const size_t n = size_t(L.Q) * size_t(s[0] * s[1] * s[2]);
                // value k (k-th element of the natural layout), stored in elem bytes
                std::vector<char> nat(n * elem), lay(n * elem, 0), back(n * elem, 0);
                for (size_t k = 0; k < n; ++k) {
                    uint64_t v = k + 1;
                    std::memcpy(nat.data() + k * elem, &v, elem < 8 ? elem : 8);
                }
                for (int layout : {int(kSwapped), int(kTwistEven), int(kTwistOdd), int(kNatural)}) {
                    std::fill(lay.begin(), lay.end(), 0);
                    std::fill(back.begin(), back.end(), 0);
                    relayout_host(L, s[0], s[1], s[2], elem, layout, false, nat.data(), lay.data());
                    relayout_host(L, s[0], s[1], s[2], elem, layout, true, lay.data(), back.data());
                    EXPECT(nat == back);
                    // a permutation: every value appears once in the rearranged state
                    std::vector<int> count(n, 0);
                    for (size_t k = 0; k < n; ++k) {
                        uint64_t v = 0;
                        std::memcpy(&v, lay.data() + k * elem, elem < 8 ? elem : 8);
                        if (v >= 1 && v <= n) count[v - 1]++;
                    }
                    size_t ones = 0;
                    for (int c : count) ones += (c == 1);
                    // 2-byte values wrap past 65535, smaller boxes stay distinct
                    if (elem > 2 || n < 65535) EXPECT(ones == n);
                }
            }
        }
    }
}

static void test_tune_cache(const char* dir)
{
    const std::string path = std::string(dir) + "/tune_cache.txt";
    {
        std::FILE* f = std::fopen(path.c_str(), "w");
        EXPECT(f != nullptr);
        if (!f) return;
        std::fputs("garbage without a bar\n", f);
        std::fputs(" | 1 2 3\n", f);
        std::fputs("key-a | 1 64\n", f);        // too few fields
        std::fputs("key-a | x y z\n", f);       // not numbers
        std::fputs("key-a | 3 256 0\n", f);
        std::fputs("key-ab | 9 9 9\n", f);      // another key with the same prefix
        std::string longline(100000, 'k');
        std::fputs((longline + " | 1 1 1\n").c_str(), f);
        std::fputs("key-a | 5 192 0 trailing words", f);  // no final newline
        std::fclose(f);
    }
    LaunchChoice c{0, 0, 0};
    EXPECT(tune_cache_lookup(path.c_str(), "key-a", &c));
    EXPECT(c.kernel == 5 && c.block == 192 && c.grid == 0);
    EXPECT(!tune_cache_lookup(path.c_str(), "key-b", &c));
    EXPECT(!tune_cache_lookup(nullptr, "key-a", &c));
    EXPECT(!tune_cache_lookup("", "key-a", &c));
    EXPECT(!tune_cache_lookup((std::string(dir) + "/missing.txt").c_str(), "key-a", &c));
    tune_cache_store(path.c_str(), "key-b", LaunchChoice{1, 128, 2048});
    tune_cache_store(nullptr, "key-b", LaunchChoice{1, 128, 2048});
    EXPECT(tune_cache_lookup(path.c_str(), "key-b", &c) && c.kernel == 1 && c.block == 128 && c.grid == 2048);
}

int main(int argc, char** argv)
{
    const char* dir = argc > 1 ? argv[1] : ".";
    test_tables();
    test_checks();
    test_two_step_fits();
    test_checkpoint();
    test_relayout();
    test_tune_cache(dir);
    if (g_fail) return 2;
    std::printf("host sanitizer driver: ok\n");
    return 0;
}
