// A plain C++ client of the correlator library, for the test suite: it uses
// only include/corr.h and the HIP runtime API (no Python, no torch in the
// process).  It channelises 8-bit real samples into int8 spectra, correlates
// them, dumps the visibilities to host memory, exercises one error path, and
// writes its inputs and outputs as raw files for the test to compare with the
// oracle.
//
//   corr_client <out_dir>
//     samples.bin : int8  [N][A*2C]        the real samples
//     inv.bin     : float [C]              the per-channel scale
//     spectra.bin : int8  [A][C][N][2]     corr_copy_spectra (public layout)
//     vis.bin     : int32 [C][N(N+1)/2][2] corr_dump_visibilities (lower, channel-major)
//     status.txt  : one line per checked call: name status
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "corr.h"

namespace {

constexpr int kStations = 12, kChannels = 64, kSpectra = 100;

bool write_file(const std::string &path, const void *data, size_t bytes) {
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(data, 1, bytes, f) == bytes;
    return std::fclose(f) == 0 && ok;
}

// xorshift32: a fixed, seeded sample source (not part of the method).
uint32_t next(uint32_t &s) {
    s ^= s << 13;
    s ^= s >> 17;
    s ^= s << 5;
    return s;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 2) {
        std::fprintf(stderr, "usage: %s <out_dir>\n", argv[0]);
        return 2;
    }
    const std::string dir = argv[1];
    const int N = kStations, C = kChannels, A = kSpectra;
    const int64_t ld = (int64_t)A * 2 * C;

    // Samples: a tone in channel 5 with a per-stream phase, plus uniform noise
    // of +-12, rounded to int8.
    std::vector<int8_t> samples((size_t)N * ld);
    uint32_t seed = 12345u;
    for (int p = 0; p < N; ++p)
        for (int64_t n = 0; n < ld; ++n) {
            const double tone = 9.0 * std::cos(2.0 * M_PI * (double)((5 * n) % (2 * C)) / (2.0 * C) + 0.4 * p);
            const double noise = (double)(next(seed) % 25u) - 12.0;
            samples[(size_t)p * ld + n] = (int8_t)std::lround(tone + noise);
        }
    std::vector<float> inv(C, (float)(16.0 / std::sqrt(C * 52.0)));

    corr_params params = {N, 1, C, A, CORR_INT8, CORR_TRI_LOWER, CORR_CHAN_MAJOR, 0, 0};
    const int64_t vis_bytes = corr_visibility_bytes(&params);
    const int64_t spec_bytes = corr_spectra_bytes(&params, A);
    FILE *st = std::fopen((dir + "/status.txt").c_str(), "w");
    if (!st || vis_bytes <= 0 || spec_bytes <= 0) return 3;

    corr_handle h = nullptr;
    corr_status s = corr_create(&params, nullptr, &h);
    std::fprintf(st, "corr_create %d\n", (int)s);
    if (s != CORR_OK) return 4;

    int8_t *d_samples = nullptr;
    float *d_inv = nullptr;
    if (hipMalloc((void **)&d_samples, samples.size()) != hipSuccess ||
        hipMalloc((void **)&d_inv, C * sizeof(float)) != hipSuccess ||
        hipMemcpy(d_samples, samples.data(), samples.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_inv, inv.data(), C * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return 5;

    s = corr_fengine_real8(h, d_samples, ld, A, d_inv);
    std::fprintf(st, "corr_fengine_real8 %d\n", (int)s);
    s = corr_xengine(h, nullptr, A, nullptr);
    std::fprintf(st, "corr_xengine %d\n", (int)s);
    // Asking for more spectra than are held is a state error, reported without a launch.
    s = corr_xengine(h, nullptr, A + 1, nullptr);
    std::fprintf(st, "corr_xengine_too_many %d %s\n", (int)s, corr_status_string(s));

    std::vector<int32_t> vis((size_t)vis_bytes / 4);
    std::vector<int8_t> spec((size_t)spec_bytes);
    s = corr_dump_visibilities(h, vis.data(), 0, 1);
    std::fprintf(st, "corr_dump_visibilities %d\n", (int)s);
    s = corr_copy_spectra(h, spec.data(), 0);
    std::fprintf(st, "corr_copy_spectra %d\n", (int)s);
    s = corr_destroy(h);
    std::fprintf(st, "corr_destroy %d\n", (int)s);
    std::fclose(st);
    (void)hipFree(d_samples);
    (void)hipFree(d_inv);

    const bool ok = write_file(dir + "/samples.bin", samples.data(), samples.size()) &&
                    write_file(dir + "/inv.bin", inv.data(), inv.size() * sizeof(float)) &&
                    write_file(dir + "/spectra.bin", spec.data(), spec.size()) &&
                    write_file(dir + "/vis.bin", vis.data(), vis.size() * sizeof(int32_t));
    std::printf("corr_client: %d streams x %d channels x %d spectra, int8, %s\n", N, C, A,
                ok ? "files written" : "write failed");
    return ok ? 0 : 6;
}
