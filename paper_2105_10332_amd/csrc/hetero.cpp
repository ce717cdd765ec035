// hetero.cpp -- heterogeneous swept advance (Sec. 3.2, Eq. 2): in every
// phase the shape instances of the tile rows jy < G run on the GPU (one
// launch of the phase kernel restricted to those rows) and the others on the
// host cores at the same time (host_swept.h), each side on its own copy of
// the two level-parity buffers.  After the phase the two copies are made to
// agree on the rows either side can read from the other's part:
//   1. the GPU's copy of those band rows is fetched into a pinned stage;
//   2. every band cell the host did not write in this phase takes the GPU's
//      value (the host marks the cells it writes), and the stage takes the
//      host's value of every cell it did write;
//   3. the merged stage goes back to the GPU, ahead of the next launch on
//      the stream.
// Both copies agree on the band after every phase (they agree at the start:
// the host copy of buffer 0 is fetched whole, and buffer 1 holds nothing that
// is read before it is written), and no instance reads a cell of the other
// side's part outside the band, so every read sees the value the all-GPU
// advance would see.  At the end the host's rows of the final level go to the
// GPU.  The band: rows within b of the two row boundaries of the split (0 and
// G b); a window reaches b/2 + n rows past its tile row, and b/2 + n < b.
#include "hetero.h"

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <new>
#include <thread>
#include <utility>

#include "host_swept.h"

namespace swept {

namespace {

// Fixed set of host worker threads; run() hands out items 0 .. n-1 from an
// atomic counter and returns when all are done.
class Pool {
   public:
    explicit Pool(int n)
    {
        for (int i = 0; i < n; ++i) th_.emplace_back([this, i] { loop(i); });
    }
    ~Pool()
    {
        {
            std::lock_guard<std::mutex> lk(m_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    int size() const { return (int)th_.size(); }
    void run(int items, const std::function<void(int, int)>& fn)
    {
        if (items <= 0) return;
        std::unique_lock<std::mutex> lk(m_);
        fn_ = &fn;
        items_ = items;
        next_.store(0);
        busy_ = (int)th_.size();
        ++gen_;
        cv_.notify_all();
        done_.wait(lk, [this] { return busy_ == 0; });
        fn_ = nullptr;
    }

   private:
    void loop(int w)
    {
        uint64_t seen = 0;
        for (;;) {
            const std::function<void(int, int)>* f;
            int items;
            {
                std::unique_lock<std::mutex> lk(m_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                f = fn_;
                items = items_;
            }
            for (int it; (it = next_.fetch_add(1)) < items;) (*f)(w, it);
            {
                std::lock_guard<std::mutex> lk(m_);
                if (--busy_ == 0) done_.notify_one();
            }
        }
    }
    std::vector<std::thread> th_;
    std::mutex m_;
    std::condition_variable cv_, done_;
    const std::function<void(int, int)>* fn_ = nullptr;
    int items_ = 0, busy_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
    std::atomic<int> next_{0};
};

}  // namespace

struct Hetero {
    HeteroSetup s;
    Pool* pool = nullptr;
    void* hb[2] = {nullptr, nullptr};  // host level-parity buffers (pinned), nvar * N * N values each
    void* stage = nullptr;             // pinned: 2 parities x nvar x band rows x N values
    size_t host_bytes = 0;
    std::vector<int> band;                   // band rows, ascending
    std::vector<int> row_band;               // N entries: index into band, or -1
    std::vector<std::pair<int, int>> runs;   // (first band index, count) of consecutive rows
    std::vector<uint8_t> mark;               // 2 x band rows x N
    std::vector<std::vector<double>> win_d;  // per-worker windows
    std::vector<std::vector<float>> win_f;
};

static size_t window_values(const HeteroSetup& s)
{
    const size_t W = (size_t)s.b + (s.kind == 0 ? 2 : 4);
    return s.kind == 0 ? 2 * W * W : 10 * W * W + 8 * (size_t)(s.b + 1);
}

void hetero_destroy(Hetero* h)
{
    if (!h) return;
    delete h->pool;
    for (void* p : {h->hb[0], h->hb[1], h->stage})
        if (p) (void)hipHostFree(p);
    delete h;
}

size_t hetero_host_bytes(const Hetero* h) { return h ? h->host_bytes : 0; }

hipError_t hetero_create(const HeteroSetup& s, Hetero** out)
{
    *out = nullptr;
    Hetero* h = new (std::nothrow) Hetero();
    if (!h) return hipErrorOutOfMemory;
    try {
        h->s = s;
        const int N = s.N, G = s.gpu_rows, T = s.tiles;
        h->row_band.assign(N, -1);
        if (G > 0 && G < T) {  // rows within b of the split's two row boundaries
            std::vector<char> in(N, 0);
            for (int Y : {0, G * s.b})
                for (int d = -s.b; d < s.b; ++d) in[((Y + d) % N + N) % N] = 1;
            for (int y = 0; y < N; ++y)
                if (in[y]) {
                    h->row_band[y] = (int)h->band.size();
                    h->band.push_back(y);
                }
            for (size_t i = 0; i < h->band.size();) {
                size_t j = i + 1;
                while (j < h->band.size() && h->band[j] == h->band[j - 1] + 1) ++j;
                h->runs.emplace_back((int)i, (int)(j - i));
                i = j;
            }
            h->mark.assign(2 * h->band.size() * (size_t)N, 0);
        }
        const int nw = std::max(1, s.threads);
        if (s.dtype == 0)
            h->win_d.assign(nw, std::vector<double>(window_values(s)));
        else
            h->win_f.assign(nw, std::vector<float>(window_values(s)));
        h->pool = new Pool(nw);
    } catch (...) {
        hetero_destroy(h);
        return hipErrorOutOfMemory;
    }
    const size_t S = s.dtype == 0 ? 8 : 4;
    const size_t stage_bytes = 2 * (size_t)s.nvar * h->band.size() * s.N * S;
    hipError_t e = hipHostMalloc(&h->hb[0], s.state_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&h->hb[1], s.state_bytes, hipHostMallocDefault);
    if (e == hipSuccess && stage_bytes) e = hipHostMalloc(&h->stage, stage_bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        hetero_destroy(h);
        return e;
    }
    h->host_bytes = 2 * s.state_bytes + stage_bytes;
    *out = h;
    return hipSuccess;
}

template <typename T>
static std::vector<std::vector<T>>& windows(Hetero& h);
template <>
std::vector<std::vector<double>>& windows<double>(Hetero& h)
{
    return h.win_d;
}
template <>
std::vector<std::vector<float>>& windows<float>(Hetero& h)
{
    return h.win_f;
}

template <typename T>
static void host_instance(const HeteroSetup& s, const HostPlan& P, int wx, int wy, int jx, int jy, T* const H[2],
                          std::vector<T>& win, const WriteLog& log)
{
    if (s.kind == 0) {
        host_heat_instance<T>(P, wx, wy, jx, jy, H, win, log);
        return;
    }
    switch (s.scheme) {
        case 1: host_euler_instance<T, 1>(P, wx, wy, jx, jy, H, win, log); break;
        case 2: host_euler_instance<T, 2>(P, wx, wy, jx, jy, H, win, log); break;
        case 3: host_euler_instance<T, 3>(P, wx, wy, jx, jy, H, win, log); break;
        default: host_euler_instance<T, 0>(P, wx, wy, jx, jy, H, win, log);
    }
}

// Steps 1-3 of the exchange (see the file comment).
template <typename T>
static hipError_t exchange(Hetero& h, T* const hb[2])
{
    const HeteroSetup& s = h.s;
    const size_t N = s.N, NN = N * N, nb = h.band.size();
    T* st = static_cast<T*>(h.stage);
    void* dp[2] = {s.d0, s.d1};
    hipError_t e = hipSuccess;
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < s.nvar; ++c)
            for (const auto& r : h.runs)
                if (e == hipSuccess)
                    e = hipMemcpyAsync(st + ((p * s.nvar + c) * nb + r.first) * N,
                                       static_cast<T*>(dp[p]) + c * NN + (size_t)h.band[r.first] * N,
                                       r.second * N * sizeof(T), hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    if (e != hipSuccess) return e;
    const uint8_t* mark = h.mark.data();
    h.pool->run((int)(2 * nb), [&](int, int it) {
        const int p = it / (int)nb, bi = it % (int)nb;
        const size_t y = h.band[bi];
        const uint8_t* mk = mark + ((size_t)p * nb + bi) * N;
        for (int c = 0; c < s.nvar; ++c) {
            T* hrow = hb[p] + c * NN + y * N;
            T* srow = st + ((p * s.nvar + c) * nb + bi) * N;
            for (size_t x = 0; x < N; ++x) {
                if (mk[x])
                    srow[x] = hrow[x];
                else
                    hrow[x] = srow[x];
            }
        }
    });
    for (int p = 0; p < 2; ++p)
        for (int c = 0; c < s.nvar; ++c)
            for (const auto& r : h.runs)
                if (e == hipSuccess)
                    e = hipMemcpyAsync(static_cast<T*>(dp[p]) + c * NN + (size_t)h.band[r.first] * N,
                                       st + ((p * s.nvar + c) * nb + r.first) * N, r.second * N * sizeof(T),
                                       hipMemcpyHostToDevice, s.stream);
    return e;
}

template <typename T>
static hipError_t advance_t(Hetero& h, long long n_steps)
{
    const HeteroSetup& s = h.s;
    if (n_steps <= 0) return hipSuccess;
    const int L = (int)(n_steps * s.lps), nwin = (L + s.h - 1) / s.h;
    const int N = s.N, T_ = s.tiles, G = s.gpu_rows;
    const size_t NN = (size_t)N * N;
    T* const hb[2] = {static_cast<T*>(h.hb[0]), static_cast<T*>(h.hb[1])};
    PhaseArgs a = s.base;
    a.L = L;
    a.jrows = G;
    HostPlan P{N, s.b, s.h, L, T_, s.tab.data(), {s.base.p[0], s.base.p[1], s.base.p[2], s.base.p[3], s.base.p[4]}};
    const size_t nb = h.band.size();
    const WriteLog log{h.mark.data(), h.row_band.data(), N, nb * (size_t)N};
    auto& wins = windows<T>(h);
    hipError_t e = hipSuccess;
    if (G < T_) {  // the host part starts from the whole level-0 state
        e = hipMemcpyAsync(hb[0], s.d0, s.state_bytes, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    }
    for (int ph = 0; ph <= 2 * nwin && e == hipSuccess; ++ph) {
        if (G > 0) {
            a.phase = ph;
            e = launch_phase(s.kind, s.dtype, a, s.wg, s.lds, s.stream);
            if (e != hipSuccess) break;
        }
        if (G < T_) {
            if (nb) memset(h.mark.data(), 0, h.mark.size());
            const int per = (T_ - G) * T_;
            const bool bridges = (ph & 1) != 0;
            const int w = (ph + 1) >> 1;
            h.pool->run(bridges ? 2 * per : per, [&](int wk, int it) {
                const int k = it >= per ? 1 : 0, r = it - k * per;
                const int jx = r % T_, jy = G + r / T_;
                int wx, wy;
                if (!bridges) {
                    wx = wy = ph >> 1;
                } else {
                    wx = k ? w - 1 : w;
                    wy = k ? w : w - 1;
                }
                host_instance<T>(s, P, wx, wy, jx, jy, hb, wins[wk], log);
            });
        }
        e = hipStreamSynchronize(s.stream);
        if (e == hipSuccess && G > 0 && G < T_) e = exchange<T>(h, hb);
    }
    if (e == hipSuccess && G < T_) {  // the host rows of level L
        void* dl = (L & 1) ? s.d1 : s.d0;
        const size_t y0 = (size_t)G * s.b;
        for (int c = 0; c < s.nvar && e == hipSuccess; ++c)
            e = hipMemcpyAsync(static_cast<T*>(dl) + c * NN + y0 * N, hb[L & 1] + c * NN + y0 * N,
                               (N - y0) * N * sizeof(T), hipMemcpyHostToDevice, s.stream);
    }
    if (e == hipSuccess && (L & 1)) e = hipMemcpyAsync(s.d0, s.d1, s.state_bytes, hipMemcpyDeviceToDevice, s.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s.stream);
    return e;
}

hipError_t hetero_advance(Hetero* h, long long n_steps, hipStream_t stream)
{
    h->s.stream = stream;
    return h->s.dtype == 0 ? advance_t<double>(*h, n_steps) : advance_t<float>(*h, n_steps);
}

}  // namespace swept
