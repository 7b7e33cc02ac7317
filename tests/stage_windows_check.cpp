/*
 * Host check of the staged resample + FFT kernel (stage_body.h), no GPU:
 * the plan-time planner lays out the staging windows for a geometry, then
 * every LDS write and read the kernel would make is replayed on the host
 * with the kernel's own index arithmetic (the chunk-to-row division by the
 * window's magic number, the row bases, the tap positions from
 * sample_pos).  A read that falls outside the window, outside the staging
 * buffer or on a pixel the window did not stage counts as a failure.  The
 * trig table is built as the plan builds it (first octant, exact
 * symmetries).  Prints one line per geometry; exit status = failures.
 */
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>
#include "stage_body.h"
using namespace zmk;

static void unit_circle(int N, std::vector<double>& cs) {
    cs.assign(2 * (size_t)N, 0.0);
    const int q4 = N / 4;
    const long double two_pi = 6.283185307179586476925286766559L;
    for (int a = 0; a < N; ++a) {
        const int qd = a / q4, b = a % q4;
        double c, s;
        if (2 * b <= q4) { const long double t = two_pi * b / N; c = (double)cosl(t); s = (double)sinl(t); }
        else { const long double t = two_pi * (q4 - b) / N; c = (double)sinl(t); s = (double)cosl(t); }
        double cc = c, ss = s;
        switch (qd) { case 1: cc = -s; ss = c; break; case 2: cc = -c; ss = -s; break; case 3: cc = s; ss = -c; break; default: break; }
        cs[2 * (size_t)a] = cc; cs[2 * (size_t)a + 1] = ss;
    }
}

template <int A2>
static int check(int H, int W, int R) {
    constexpr int A = 4096, NTHR = 1024;
    using SS = StageShape<A, A2, NTHR>;
    constexpr int NT = SS::NT, P = SS::P, kStep = A / 32, CAP = SS::kCap;
    const int D = std::min(H, W);
    const int Rp = (R + 31) / 32 * 32;
    const double cx = 0.5 * (W - 1), cy = 0.5 * (H - 1), rpx = 0.5 * D;
    std::vector<double> spx(R), trig;
    for (int r = 0; r < R; ++r) spx[r] = (double)(2 * r + 1) * rpx / (double)(2 * R);
    unit_circle(A, trig);
    std::vector<StageWin> wins; std::vector<int> rows;
    auto t0 = std::chrono::steady_clock::now();
    bool ok = stage_windows<A, A2, NTHR>(H, W, R, Rp, cx, cy, spx, trig, wins, rows);
    double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    printf("%dx%d R=%d A2=%d: planner %s in %.1f ms, %zu windows, %zu rows; kCap %d floats, LDS %zu B\n", H, W, R, A2,
           ok ? "ok" : "REFUSED", ms, wins.size(), rows.size(), CAP, FftLds<float, A, A2, NTHR, 1>::bytes);
    if (!ok) return 0;
    long bad = 0, staged = 0, samples = 0; int maxw = 0;
    std::vector<int> base(SS::kMaxRows);
    std::vector<char> written(CAP);
    for (int k = 0; k < Rp / (2 * P); ++k) {
        const int r0 = 2 * P * k;
        if (r0 >= R) continue;
        for (int j = 0; j < 16; ++j) {
            const StageWin& w = wins[(size_t)k * 16 + j];
            const int total = w.nrows * w.cmax, pitch = 4 * w.cmax;
            maxw = std::max(maxw, w.nrows * pitch);
            std::fill(written.begin(), written.end(), 0);
            for (int tid = 0; tid < NTHR; ++tid)
                for (int l = 0; l < SS::kLoads; ++l) {
                    const int c = tid + NTHR * l;
                    if (c >= total) continue;
                    const int row = (int)(((unsigned long long)(unsigned)c * w.magic) >> 32);
                    const int kk = c - row * w.cmax;
                    if (row != c / w.cmax || row >= w.nrows) { ++bad; continue; }
                    const int e = rows[w.rowoff + row];
                    const int xs = e >> 8, n = e & 255;
                    const int idx = row * pitch + 4 * kk;
                    if (idx < 0 || idx + 3 >= CAP) { ++bad; continue; }
                    if (kk < n) { for (int d = 0; d < 4; ++d) written[idx + d] = 1; staged += 4; }
                    if (kk == 0) base[row] = row * pitch - xs;
                }
            for (int f = 0; f < P; ++f)
                for (int h = 0; h < 2; ++h) {
                    const int r = r0 + 2 * f + h;
                    if (r >= R) continue;
                    for (int t = 0; t < NT; ++t) {
                        const int b = t + NT * (j & 3);
                        double cb, sb;
                        const int bi = 2 * (j & 3) + t / kStep;
                        rotate_pair(trig[2 * (t % kStep)], trig[2 * (t % kStep) + 1], trig[2 * kStep * bi],
                                    trig[2 * kStep * bi + 1], cb, sb);
                        if (bi * kStep + t % kStep != b) ++bad;
                        const TapPos<float> tp = sample_pos<float>(cx, cy, W, H, spx[r], cb, sb, j >> 2);
                        const int row = tp.y.i - w.imin;
                        ++samples;
                        if (row < 0 || row + 1 >= w.nrows) { ++bad; continue; }
                        for (int d = 0; d < 2; ++d) {
                            const int i0 = base[row + d] + tp.x.i;
                            if (i0 < 0 || i0 + 1 >= CAP || !written[i0] || !written[i0 + 1]) ++bad;
                            if (i0 < (row + d) * pitch || i0 + 1 >= (row + d + 1) * pitch) ++bad;
                        }
                    }
                }
        }
    }
    printf("   bad=%ld  staged px/sample=%.3f  max window %d floats\n", bad, (double)staged / samples, maxw);
    return bad != 0;
}

int main() {
    int fails = 0;
    fails += check<256>(2160, 3840, 1080);
    fails += check<16>(2160, 3840, 1080);
    fails += check<256>(1024, 1024, 512);
    fails += check<128>(4096, 4096, 300);
    fails += check<256>(1200, 1100, 550);
    fails += check<64>(2161, 2163, 1080);
    fails += check<256>(3000, 3000, 1300);
    printf("stage_windows_check: %d failure(s)\n", fails);
    return fails;
}
