// Runs the directed model's POSITIVE kernel (k_positive_dir, compiled for the
// host with the emulation header of this folder) on cases read from a file,
// for tests: the host side builds the kernel's inputs the way the library's
// positive() does (components of the assignment, flagged communities, member
// lists, cycle sizes), with the member and community order shuffled by a
// seed.  The level graph is S = W + W^T with the two strengths x and y of
// the directed model and the scale A of its edge term.  Every array has the
// exact size the kernel may use; scratch arrays start with junk.  A barrier
// that some threads pass and others never reach stops the run with each
// thread's barrier sequence (exit status 3).
//
// Input per case (little-endian): i64 n, nnz, A, seed, shuffle; i64
// rp[n+1]; i32 col[nnz], w[nnz], x[n], y[n], a[n].  Output per case: i64
// splits, err, nflag; i32 a[n] after the kernel.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <random>
#include <thread>
#include <unistd.h>

#include "k_positive_dir_emu.inc"

thread_local dim3 threadIdx;
thread_local dim3 blockIdx;
dim3 blockDim, gridDim;
std::barrier<> *emu_block_bar;
EmuWave *emu_waves;
std::vector<int> emu_seq[1024];
volatile long emu_progress;
int emu_skew_us;
thread_local uint64_t emu_rng;

void emu_sleep_us(int us) { std::this_thread::sleep_for(std::chrono::microseconds(us)); }

template <class T>
static std::vector<T> junk(size_t cnt, std::mt19937_64 &r)
{
    std::vector<T> v(cnt ? cnt : 1);
    unsigned char *b = (unsigned char *)v.data();
    for (size_t i = 0; i < v.size() * sizeof(T); i++) b[i] = (unsigned char)r();
    return v;
}

static void run_case(i64 n, const std::vector<i64> &rp, const std::vector<i32> &col,
                     const std::vector<i32> &w, const std::vector<i32> &x,
                     const std::vector<i32> &y, i64 A_sc, std::vector<i32> &a, u64 seed,
                     bool shuffle, i64 *splits_out, int *err_out, i64 *nflag_out)
{
    std::mt19937_64 rng(seed);
    const i64 nnz = rp[n];
    std::vector<int2> e(nnz ? nnz : 1);
    for (i64 j = 0; j < nnz; j++) e[j] = make_int2(col[j], w[j]);
    // components of u -> a(u): cycle flags, community = cycle minimum
    std::vector<int> state(n, 0);
    std::vector<i32> comp(n, -1), path;
    std::vector<uint8_t> cyc(n ? n : 1, 0);
    for (i64 s0 = 0; s0 < n; s0++) {
        if (state[s0]) continue;
        path.clear();
        i64 u = s0;
        while (state[u] == 0) {
            state[u] = 1;
            path.push_back((i32)u);
            u = a[u];
        }
        if (state[u] == 1) {
            i32 mn = (i32)u;
            i64 v = u;
            do {
                cyc[v] = 1;
                mn = std::min<i32>(mn, (i32)v);
                v = a[v];
            } while (v != u);
            do {
                comp[v] = mn;
                v = a[v];
            } while (v != u);
        }
        for (size_t i = path.size(); i-- > 0;) {
            if (comp[path[i]] < 0) comp[path[i]] = comp[a[path[i]]];
            state[path[i]] = 2;
        }
    }
    // communities holding a node of negative local gain
    //   g(u) = A w(u, C \ u) - x_u (X_C - x_u) + y_u (Y_C - y_u)
    std::vector<i64> sx(n, 0), sy(n, 0);
    for (i64 u = 0; u < n; u++) {
        sx[comp[u]] += x[u];
        sy[comp[u]] += y[u];
    }
    std::vector<i32> fidx(n, -1), flist;
    for (i64 u = 0; u < n; u++) {
        i64 wc = 0;
        for (i64 j = rp[u]; j < rp[u + 1]; j++)
            if (col[j] != u && comp[col[j]] == comp[u]) wc += w[j];
        const i64 c = comp[u];
        const i64 g = A_sc * wc - (i64)x[u] * (sx[c] - x[u]) + (i64)y[u] * (sy[c] - y[u]);
        if (g < 0 && fidx[c] < 0) {
            fidx[c] = (i32)flist.size();
            flist.push_back((i32)c);
        }
    }
    const i64 nflag = (i64)flist.size();
    *nflag_out = nflag;
    *splits_out = 0;
    *err_out = 0;
    if (nflag == 0) return;
    if (shuffle) {
        std::shuffle(flist.begin(), flist.end(), rng);
        for (i64 f = 0; f < nflag; f++) fidx[flist[f]] = (i32)f;
    }
    std::vector<std::vector<i32>> mems(nflag);
    std::vector<i32> flen(nflag, 0);
    for (i64 u = 0; u < n; u++) {
        const i32 f = fidx[comp[u]];
        if (f < 0) continue;
        mems[f].push_back((i32)u);
        if (cyc[u]) flen[f]++;
    }
    std::vector<i64> mem_off(nflag + 1, 0), woff(nflag + 1, 0), noff(nflag + 1, 0);
    std::vector<i32> mem(n);
    for (i64 f = 0; f < nflag; f++) {
        if (shuffle) std::shuffle(mems[f].begin(), mems[f].end(), rng);
        std::copy(mems[f].begin(), mems[f].end(), mem.begin() + mem_off[f]);
        mem_off[f + 1] = mem_off[f] + (i64)mems[f].size();
        const i64 l = flen[f];
        woff[f + 1] = woff[f] + (l >= 2 ? l * l : 0);
        noff[f + 1] = noff[f] + (l >= 2 ? l : 0);
    }
    std::vector<i32> part(comp);
    auto tmp = junk<i32>(n, rng), ord = junk<i32>(n, rng), chl = junk<i32>(2 * n, rng);
    auto dpre = junk<i64>(n + nflag, rng);
    auto lvl = junk<i32>(n + nflag, rng);
    auto stk = junk<int4>(n, rng);
    auto win = junk<i32>(n, rng), subk = junk<i32>(n, rng), cut = junk<i32>(n, rng);
    auto dep = junk<i32>(n, rng), root = junk<i32>(n, rng), chs = junk<i32>(n, rng);
    auto chc = junk<i32>(n, rng), cpos = junk<i32>(n, rng);
    auto cn = junk<i32>(noff[nflag], rng);
    auto W = junk<i64>(woff[nflag], rng);
    std::vector<i32> diag(n, 0);
    int err = 0;
    unsigned long long spl = 0;
    PosArgs A{};
    A.G.rp = rp.data();
    A.G.e = e.data();
    A.G.k = x.data();
    A.G.y = y.data();
    A.G.diag = diag.data();
    A.G.n = n;
    A.G.nnz = nnz;
    A.G.m2 = A_sc;
    A.a = a.data();
    A.cyc = cyc.data();
    A.flist = flist.data();
    A.mem_off = mem_off.data();
    A.mem = mem.data();
    A.tmp = tmp.data();
    A.ord = ord.data();
    A.chl = chl.data();
    A.dpre = dpre.data();
    A.lvl = lvl.data();
    A.stk = stk.data();
    A.part = part.data();
    A.win = win.data();
    A.subk = subk.data();
    A.cut = cut.data();
    A.dep = dep.data();
    A.root = root.data();
    A.chs = chs.data();
    A.chc = chc.data();
    A.cpos = cpos.data();
    A.lcyc = flen.data();
    A.woff = woff.data();
    A.W = W.data();
    A.noff = noff.data();
    A.cn = cn.data();
    A.splits = (i64 *)&spl;
    A.err = &err;

    std::barrier<> bb(PD_BS);
    emu_block_bar = &bb;
    emu_waves = new EmuWave[PD_NW];
    for (int q = 0; q < PD_NW; q++) emu_waves[q].bar = new std::barrier<>(64);
    blockDim.x = PD_BS;
    gridDim.x = (unsigned)nflag;
    std::atomic<bool> fin{false};
    std::thread dog([&] {
        long last = -1;
        int still = 0;
        while (!fin.load()) {
            std::this_thread::sleep_for(std::chrono::milliseconds(250));
            const long p = emu_progress;
            still = p == last ? still + 1 : 0;
            last = p;
            if (still >= 80) {  // 20 s without a barrier
                fprintf(stderr, "STUCK: barrier sequences (source lines) per thread\n");
                for (int t = 0; t < PD_BS; t++) {
                    const auto &q0 = emu_seq[0], &qt = emu_seq[t];
                    size_t i = 0;
                    while (i < q0.size() && i < qt.size() && q0[i] == qt[i]) i++;
                    fprintf(stderr, "  t%d: %zu barriers; first difference with t0 at %zu:", t,
                            qt.size(), i);
                    for (size_t j = i >= 3 ? i - 3 : 0; j < i + 3 && j < qt.size(); j++)
                        fprintf(stderr, " %d", qt[j]);
                    fprintf(stderr, "\n");
                }
                fflush(stderr);
                _exit(3);
            }
        }
    });
    std::vector<std::thread> th;
    for (int t = 0; t < PD_BS; t++)
        th.emplace_back([&, t] {
            threadIdx.x = t;
            emu_rng = (seed + 1) * 0x9E3779B97F4A7C15ull + (u64)t * 0xD1B54A32D192ED03ull + 1;
            emu_seq[t].clear();
            for (i64 b = 0; b < nflag; b++) {
                blockIdx.x = (unsigned)b;
                k_positive_dir(A);
                __syncthreads();
            }
        });
    for (auto &t : th) t.join();
    fin = true;
    dog.join();
    for (int q = 0; q < PD_NW; q++) delete emu_waves[q].bar;
    delete[] emu_waves;
    *splits_out = (i64)spl;
    *err_out = err;
}

int main(int argc, char **argv)
{
    if (argc < 4) return 2;
    FILE *in = fopen(argv[1], "rb"), *out = fopen(argv[2], "wb");
    if (!in || !out) return 2;
    emu_skew_us = atoi(argv[3]);
    i64 hdr[5];
    while (fread(hdr, sizeof(i64), 5, in) == 5) {
        const i64 n = hdr[0], nnz = hdr[1];
        std::vector<i64> rp(n + 1);
        std::vector<i32> col(nnz), w(nnz), x(n), y(n), a(n);
        if (fread(rp.data(), 8, n + 1, in) != (size_t)(n + 1)) return 2;
        if (nnz && fread(col.data(), 4, nnz, in) != (size_t)nnz) return 2;
        if (nnz && fread(w.data(), 4, nnz, in) != (size_t)nnz) return 2;
        if (n && fread(x.data(), 4, n, in) != (size_t)n) return 2;
        if (n && fread(y.data(), 4, n, in) != (size_t)n) return 2;
        if (n && fread(a.data(), 4, n, in) != (size_t)n) return 2;
        i64 res[3];
        int err = 0;
        run_case(n, rp, col, w, x, y, hdr[2], a, (u64)hdr[3], hdr[4] != 0, &res[0], &err,
                 &res[2]);
        res[1] = err;
        fwrite(res, 8, 3, out);
        fwrite(a.data(), 4, n, out);
    }
    fclose(out);
    return 0;
}
