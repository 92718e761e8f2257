// mobius_tune.cpp -- autotuner of the hop-kernel launch parameters.
//
// For one context and storage precision the tuner times the metered hop
// D_{p,1-p} (both parities alternately) for every candidate of
//   prefetch depth of the direction loop   {0, 1, 2}
//   link staging in LDS                    {off, on}
//   XCD-contiguous block order             {off, on}
//   non-temporal link loads                {off, on}
//   FP16 colour multiply on the matrix cores {off, on} (with staging, Ls % 4 == 0)
// and keeps the fastest in the context; every later operator application,
// solve and force evaluation of the context launches with it.  Results can be
// cached in a text file (one line per lattice, Ls, precision and device)
// named by MOBIUS_TUNE_CACHE, so that a run re-uses the measurement of an
// earlier one.
#include "mobius_internal.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

namespace mobius {
namespace {

std::string cache_key(const mobius_ctx *ctx, int prec)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    std::ostringstream k;
    k << ctx->g.L[0] << 'x' << ctx->g.L[1] << 'x' << ctx->g.L[2] << 'x' << ctx->g.L[3] << " Ls"
      << ctx->g.Ls << " brick" << ctx->g.brick[0] << 'x' << ctx->g.brick[1] << 'x'
      << ctx->g.brick[2] << " prec" << prec << ' ' << arch << " v2";
    return k.str();
}

bool cache_lookup(const std::string &path, const std::string &key, HopTuning &t, double &us)
{
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {  // the last entry for a key wins
        const size_t bar = line.find(" | ");
        if (bar == std::string::npos || line.compare(0, bar, key) != 0 || bar != key.size()) continue;
        std::istringstream v(line.substr(bar + 3));
        HopTuning c;
        double u;
        if (v >> c.prefetch >> c.stage_links >> c.xcd_remap >> c.nt_links >> c.mfma >> u) {
            t = c;
            us = u;
            found = true;
        }
    }
    return found;
}

void cache_store(const std::string &path, const std::string &key, const HopTuning &t, double us)
{
    std::ofstream f(path, std::ios::app);
    f.precision(17);  // the time reads back exactly
    f << key << " | " << t.prefetch << ' ' << t.stage_links << ' ' << t.xcd_remap << ' '
      << t.nt_links << ' ' << t.mfma << ' ' << us << '\n';
}

}  // namespace

int tune(mobius_ctx *ctx, int prec, int reps, mobius_tune_result *out, hipStream_t st)
{
    const char *cache = std::getenv("MOBIUS_TUNE_CACHE");
    const std::string key = cache_key(ctx, prec);
    HopTuning best = ctx->tune[prec];
    double best_us = 0;
    if (cache && cache_lookup(cache, key, best, best_us)) {
        ctx->tune[prec] = best;
        ctx->tuned_us[prec] = best_us;
    } else {
        const Geometry &g = ctx->g;
        const int64_t fb = field_bytes(g, prec);
        hipError_t e = ctx->scratch.ensure(2 * fb);
        if (e != hipSuccess) return set_error(MOBIUS_ENOMEM, hipGetErrorString(e));
        char *in = static_cast<char *>(ctx->scratch.p);
        char *outf = in + fb;
        // timed on a seeded field of Gaussian magnitudes (zeros would take
        // the FP16 path's zero-norm shortcut), output cleared
        e = launch_fill_random(prec, in, g.N5, 12345u, st);
        if (e == hipSuccess) e = launch_zero(outf, fb, st);
        if (e != hipSuccess) return set_error(MOBIUS_EHIP, hipGetErrorString(e));
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return set_error(MOBIUS_EHIP, "hipEventCreate failed");
        const int nrep = reps > 0 ? reps : 10;
        best_us = 1e300;
        int rc = MOBIUS_OK;
        const int nmf = prec == MOBIUS_F16 && g.Ls % 4 == 0 ? 2 : 1;
        for (int mf = 0; mf < nmf && rc == MOBIUS_OK; ++mf)
        for (int pf = 0; pf < 3 && rc == MOBIUS_OK; ++pf)
            for (int stage = 0; stage < 2 && rc == MOBIUS_OK; ++stage)
                for (int remap = 0; remap < 2 && rc == MOBIUS_OK; ++remap)
                    for (int nt = 0; nt < 2 && rc == MOBIUS_OK; ++nt) {
                        // the matrix-core loop has one prefetch depth and needs staging
                        if (mf && (pf != 2 || !stage)) continue;
                        HopTuning c;
                        c.prefetch = pf;
                        c.stage_links = stage;
                        c.xcd_remap = remap;
                        c.nt_links = nt;
                        c.mfma = mf;
                        HopArgs a;
                        a.prec = prec;
                        a.dag = 0;
                        a.epi = 0;
                        a.in = in;
                        a.out = outf;
                        a.nrhs = 1;
                        a.tune = &c;
                        auto run = [&](int n) {
                            for (int r = 0; r < n; ++r)
                                for (int par = 0; par < 2; ++par) {
                                    a.out_parity = par;
                                    hipError_t x = launch_hop(g, ctx->c, hop_links(ctx, prec, a.dag),
                                                              static_cast<const int32_t *>(ctx->nbr.p), a, st);
                                    if (x != hipSuccess) return x;
                                }
                            return hipSuccess;
                        };
                        float ms = 0;
                        if ((e = run(2)) != hipSuccess || (e = hipEventRecord(e0, st)) != hipSuccess ||
                            (e = run(nrep)) != hipSuccess || (e = hipEventRecord(e1, st)) != hipSuccess ||
                            (e = hipEventSynchronize(e1)) != hipSuccess ||
                            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
                            rc = set_error(MOBIUS_EHIP, hipGetErrorString(e));
                            break;
                        }
                        const double us = 1e3 * ms / (2.0 * nrep);
                        if (us < best_us) {
                            best_us = us;
                            best = c;
                        }
                    }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (rc != MOBIUS_OK) return rc;
        ctx->tune[prec] = best;
        ctx->tuned_us[prec] = best_us;
        if (cache) cache_store(cache, key, best, best_us);
    }
    if (out) {
        out->prec = prec;
        out->prefetch = best.prefetch;
        out->stage_links = best.stage_links;
        out->xcd_remap = best.xcd_remap;
        out->nt_links = best.nt_links;
        out->mfma = best.mfma;
        out->hop_us = best_us;
    }
    return MOBIUS_OK;
}

}  // namespace mobius
