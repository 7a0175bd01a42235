// Host-only parts of the library (host.hpp): no HIP call, so the file also
// builds and runs under the host sanitizers.
#include "host.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>

#include "lattice.hpp"

namespace lbm {

template <class L>
static void fill_info(LatticeInfo* out)
{
    out->D = L::D;
    out->Q = L::Q;
    out->two_n = L::TWO_N;
    out->k_default = L::K_DEFAULT;
    out->k_max = L::K_MAX;
    out->R = L::R;
    out->T0 = L::T0;
    out->c.resize(L::Q * 3);
    out->w.resize(L::Q);
    out->mrow.resize(L::Q);
    for (int i = 0; i < L::Q; ++i) {
        for (int a = 0; a < 3; ++a) out->c[i * 3 + a] = L::c[i][a];
        out->w[i] = L::w[i];
        out->mrow[i] = mem_row<L>(i);
    }
}

bool lattice_info(int lat, LatticeInfo* out)
{
    switch (lat) {
    case kD2Q9: fill_info<D2Q9>(out); return true;
    case kD3Q15: fill_info<D3Q15>(out); return true;
    case kD3Q19: fill_info<D3Q19>(out); return true;
    case kD3Q39: fill_info<D3Q39>(out); return true;
    default: return false;
    }
}

size_t storage_bytes(int dtype)
{
    switch (dtype) {
    case 0: return 8;
    case 1: return 4;
    case 2: return 2;
    case 3: return 2;
    default: return 0;
    }
}

// *why := "box <box>: <what>"
static bool reject(std::string* why, int box, const char* what)
{
    *why = "box " + std::to_string(box) + ": " + what;
    return false;
}

bool check_boxes(const LatticeInfo& L, int dtype, int nbox, const int64_t* dims, const double* tau, std::string* why)
{
    const size_t elem = storage_bytes(dtype);
    int64_t total = 0;
    for (int b = 0; b < nbox; ++b) {
        const int64_t* d = dims + 3 * b;
        for (int a = 0; a < 3; ++a)
            if (d[a] < 1 || d[a] > INT32_MAX) {
                char buf[128];
                snprintf(buf, sizeof(buf), "box %d: dims[%d] = %lld outside [1, 2^31)", b, a, (long long)d[a]);
                *why = buf;
                return false;
            }
        const int64_t nx = d[0], ny = d[1], nz = d[2];
        // the step kernels index x-rows r = z ny + y in 32 bits
        if (ny * nz > INT32_MAX) return reject(why, b, "ny * nz must be below 2^31");
        if (L.D == 2 && nz != 1) return reject(why, b, "a 2-D lattice needs nz == 1");
        if (!std::isfinite(tau[b]) || !(tau[b] > 0.5)) return reject(why, b, "tau must be finite and > 1/2");
        total += nx * ny * nz;
        if (total > kMaxSites) return reject(why, b, "the total site count must be at most 2^36");
        // lane offsets inside one population row are formed in 32 bits
        if (nx * int64_t(elem) > INT32_MAX)
            return reject(why, b, "a population row (nx * storage bytes) must be below 2 GiB");
        // y and z are grid coordinates of the single-box kernels
        if (ny > 65535 || nz > 65535) return reject(why, b, "ny and nz must be at most 65535");
        if (nbox > 1) {
            // a batch box is addressed with 32-bit element offsets
            const uint64_t padded = (uint64_t(nx * ny * nz) + kBlockSites - 1) / kBlockSites * kBlockSites;
            if (padded * uint64_t(L.Q) * elem >= (uint64_t(1) << 31))
                return reject(why, b, "a box of a batch must hold less than 2 GiB of populations");
            // the batched step splits a lane's site with a float reciprocal,
            // exact while x0 + 64 stays below 2^22
            if (nx > (int64_t(1) << 21)) return reject(why, b, "a box of a batch needs nx at most 2^21");
        }
    }
    return true;
}

bool two_step_fits(const LatticeInfo& L, int dtype, int64_t nx, int64_t ny, int64_t nz)
{
    const size_t elem = storage_bytes(dtype);
    if (L.D != 3 || L.R != 1 || elem == 0) return false;
    if (nx < 1 || ny < 1 || nz < 1 || nx > INT32_MAX || ny > INT32_MAX || nz > INT32_MAX) return false;
    if (nx % kTwoStepTileX != 0 || ny % two_step_tile_y(elem) != 0) return false;
    const uint64_t plane_sites = uint64_t(nx) * uint64_t(ny);  // below 2^62
    return plane_sites <= ((uint64_t(1) << 31) - 1) / (uint64_t(L.Q) * elem);
}

uint64_t geometry_hash(const std::vector<int64_t>& dims)
{
    uint64_t x = 1469598103934665603ULL;  // FNV-1a over the dims
    for (int64_t d : dims) {
        for (int k = 0; k < 8; ++k) {
            x ^= uint64_t((d >> (8 * k)) & 0xff);
            x *= 1099511628211ULL;
        }
    }
    return x;
}

bool check_checkpoint(const void* buf, size_t bytes, const CkptHeader& expect, std::string* why)
{
    if (!buf || bytes < sizeof(CkptHeader) + expect.payload_bytes) {
        char msg[128];
        snprintf(msg, sizeof(msg), "checkpoint buffer needs %zu bytes", size_t(sizeof(CkptHeader) + expect.payload_bytes));
        *why = msg;
        return false;
    }
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (hd.magic != kCkptMagic) {
        *why = "not a checkpoint written by lbm_get_state";
        return false;
    }
    if (hd.lattice != expect.lattice || hd.dtype != expect.dtype || hd.K != expect.K || hd.nbox != expect.nbox ||
        hd.nsites != expect.nsites || hd.geometry_hash != expect.geometry_hash ||
        hd.payload_bytes != expect.payload_bytes) {
        *why = "checkpoint does not match this handle (lattice, dtype, K or geometry)";
        return false;
    }
    if (hd.t < 0) {
        *why = "checkpoint has a negative time";
        return false;
    }
    return true;
}

void relayout_host(const LatticeInfo& L, int64_t nx, int64_t ny, int64_t nz, size_t elem, int layout,
                   bool to_natural, const char* src, char* dst)
{
    const int64_t tile = int64_t(L.Q) * nx;
    auto wrap = [](int64_t v, int64_t n) { return ((v % n) + n) % n; };
    for (int j = 0; j < L.Q; ++j) {
        const int jo = (j == 0) ? 0 : ((j & 1) ? j + 1 : j - 1);
        int64_t o[3];
        for (int a = 0; a < 3; ++a) {
            const int c = L.c[j * 3 + a];
            o[a] = (layout == kSwapped) ? c : (layout == kNatural ? 0 : (c > 0 ? c : 0));
        }
        const int64_t r = (layout == kNatural || layout == kTwistEven) ? L.mrow[j] : L.mrow[jo];
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y) {
                const int64_t zs = wrap(z + o[2], nz), ys = wrap(y + o[1], ny);
                const int64_t lay_row = (zs * ny + ys) * tile + r * nx;
                const int64_t nat_row = (z * ny + y) * tile + int64_t(L.mrow[j]) * nx;
                for (int64_t x = 0; x < nx; ++x) {
                    const int64_t xs = wrap(x + o[0], nx);
                    if (to_natural) std::memcpy(dst + (nat_row + x) * elem, src + (lay_row + xs) * elem, elem);
                    else std::memcpy(dst + (lay_row + xs) * elem, src + (nat_row + x) * elem, elem);
                }
            }
    }
}

bool tune_cache_lookup(const char* path, const std::string& key, LaunchChoice* out)
{
    if (!path || !*path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
        std::istringstream rest(line.substr(bar + 3));
        LaunchChoice c;
        if (rest >> c.kernel >> c.block >> c.grid) {
            *out = c;  // the last entry for a key wins
            found = true;
        }
    }
    return found;
}

void tune_cache_store(const char* path, const std::string& key, const LaunchChoice& c)
{
    if (!path || !*path) return;
    // a last line without its newline (a write cut short, an edit) must not
    // swallow the new entry
    bool newline = false;
    {
        std::ifstream in(path, std::ios::binary | std::ios::ate);
        if (in && in.tellg() > 0) {
            in.seekg(-1, std::ios::end);
            char last = '\n';
            newline = in.get(last) && last != '\n';
        }
    }
    std::ofstream out(path, std::ios::app);
    if (newline) out << "\n";
    out << key << " | " << c.kernel << " " << c.block << " " << c.grid << "\n";
}

}  // namespace lbm
