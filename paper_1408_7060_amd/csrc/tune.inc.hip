// Autotuner of the batching form: FFT radix plans, launch shapes and the
// batched-GMRES schedule, timed on the context itself.  Every admissible
// setting computes the same operator; a candidate whose matvec departs from
// the current setting's by more than rounding is rejected.
// (Included by etaim.hip inside its anonymous namespace.)

bool radix_supported(int r) { return r == 2 || r == 3 || r == 4 || r == 6 || r == 8 || r == 12 || r == 16; }

// ordered factorisations of n into supported radices, at most maxp passes
void plans_of(int n, int maxp, const Radix& cur, std::vector<Radix>& out) {
    if (n == 1) {
        if (cur.n > 0) out.push_back(cur);
        return;
    }
    if (cur.n >= maxp) return;
    for (int r : {16, 12, 8, 6, 4, 3, 2})
        if (n % r == 0) {
            Radix nx = cur;
            nx.r[nx.n++] = r;
            plans_of(n / r, maxp, nx, out);
        }
}

std::vector<Radix> candidate_plans(int L) {
    const Radix def = make_radix(L);
    Radix empty{};
    empty.L = L;
    std::vector<Radix> all;
    plans_of(L, std::min(def.n + 1, 8), empty, all);
    return all;
}

bool radix_equal(const Radix& a, const Radix& b) {
    if (a.L != b.L || a.n != b.n) return false;
    for (int i = 0; i < a.n; ++i)
        if (a.r[i] != b.r[i]) return false;
    return true;
}

struct Shape {
    Radix rx, ry, rz;
    int mr = 0, mt = 0, waves = 4, sync = 1, graph = 0, engine = 0, xeng = 0, guess = kMaxGuess, precond = 1, dblock = 6,
        ieng = 0;
};

template <typename R>
int auto_gather_rows(const etaim_ctx* c, const Radix& rx) {
    int mr = sizeof(R) == 4 ? 16 : 8;
    const size_t lx = (size_t)rx.L;
    while (mr > 1 && (!plane_fits(4 * mr, rx) || (4 * (size_t)mr * (lx + 1) + lx) * sizeof(cplx<R>) > 160 * 1024))
        mr /= 2;
    return mr;
}

template <typename R>
bool shape_fits(const etaim_ctx* c, const Shape& s) {
    const GridDims& g = c->gd;
    const Radix* pl[3] = {&s.rx, &s.ry, &s.rz};
    for (int a = 0; a < 3; ++a) {
        if (pl[a]->L != g.L[a] || pl[a]->n < 1 || pl[a]->n > 8) return false;
        long prod = 1;
        for (int i = 0; i < pl[a]->n; ++i) {
            if (!radix_supported(pl[a]->r[i])) return false;
            prod *= pl[a]->r[i];
        }
        if (prod != g.L[a]) return false;
    }
    const int mr = s.mr > 0 ? s.mr : auto_gather_rows<R>(c, s.rx);
    const int mt = s.mt > 0 ? s.mt : lines_per_block<R>(s.rx);
    const size_t e = sizeof(cplx<R>), Lx = (size_t)g.L[0];
    const bool yz_fits =
        s.engine == 3 ? (line_fits<R>(s.ry) && line_fits<R>(s.rz))
                      : (plane_fits(g.N[2], s.ry) && plane_fits(g.L[1], s.rz) &&
                         (s.engine != 0 || ((size_t)g.L[2] * (g.L[1] + 1) + g.L[1] + g.L[2]) * sizeof(cplx<R>) <=
                                               (size_t)160 * 1024));
    const size_t nb = (size_t)c->B;
    if ((s.engine == 3 && 4 * nb * g.L[0] > kMaxGridY) || ((s.xeng == 0 || !xline_n(c)) && 4 * nb * g.N[2] > kMaxGridY))
        return false;
    return yz_fits && plane_fits(4 * mr, s.rx) &&
           plane_fits(mt, s.rx) && (4 * (size_t)mr * (Lx + 1) + Lx) * e <= 160 * 1024 &&
           ((size_t)mt * (Lx + 1) + Lx) * e <= (size_t)kLdsBudget && s.waves >= 1 && s.waves <= 4 &&
           s.sync >= 1 && s.sync <= c->prm.restart && (s.engine == 0 || s.engine == 3 || ((s.engine == 1 || s.engine == 2) && quad_n(c) > 0)) &&
           (s.xeng == 0 || (s.xeng == 1 && xreg_ok(c))) && s.guess >= 0 && s.guess <= kMaxGuess &&
           (s.precond == 0 || s.precond == 1) && s.dblock >= 1 && s.dblock <= kFarMaxBlock &&
           (s.ieng == 0 || (s.ieng == 1 && c->ntiles > 0 && interp_tile_lds<R>(c) <= 160 * 1024));
}

void drop_graphs(etaim_ctx* c) {
    for (auto& v : c->graphs) {
        for (auto& x : v)
            if (x) (void)hipGraphExecDestroy(x);
        v.clear();
    }
    for (auto& kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
    c->step_graphs.clear();
}

void put_shape(etaim_ctx* c, const Shape& s) {
    c->rx = s.rx;
    c->ry = s.ry;
    c->rz = s.rz;
    c->gather_rows_t = s.mr;
    c->lines_x_t = s.mt;
    c->interp_waves = s.waves;
    c->sync_every = s.sync;
    c->use_graph = s.graph == 1;
    c->step_graph = s.graph == 2;
    // the register engines lay the spectrum ring out by parity quadrants, the
    // LDS and line-pass engines plainly: a change between the two layouts
    // invalidates the history (and its block sums)
    auto quad = [](int e) { return e == 1 || e == 2; };
    if (quad(c->yz_engine) != quad(s.engine)) {
        c->next_step = -1;
        set_far_r0(c, -1);
    }
    c->yz_engine = s.engine;
    c->x_engine = s.xeng;
    c->guess_order = s.guess;
    c->precond = s.precond;
    c->interp_engine = s.ieng;
    if (c->delay_block != s.dblock) set_far_r0(c, -1);
    c->delay_block = s.dblock;
    drop_graphs(c);  // captured steps hold the old launch shapes
}

Shape get_shape(const etaim_ctx* c) {
    Shape s;
    s.rx = c->rx;
    s.ry = c->ry;
    s.rz = c->rz;
    s.mr = c->gather_rows_t;
    s.mt = c->lines_x_t;
    s.waves = c->interp_waves;
    s.sync = c->sync_every;
    s.graph = c->step_graph ? 2 : (c->use_graph ? 1 : 0);
    s.engine = c->yz_engine;
    s.xeng = c->x_engine;
    s.guess = c->guess_order;
    s.precond = c->precond;
    s.dblock = c->delay_block;
    s.ieng = c->interp_engine;
    return s;
}

template <typename R>
void shape_to_c(const etaim_ctx* c, const Shape& s, etaim_tuning* t) {
    std::memset(t->radix, 0, sizeof(t->radix));
    const Radix* pl[3] = {&s.rx, &s.ry, &s.rz};
    for (int a = 0; a < 3; ++a)
        for (int i = 0; i < pl[a]->n && i < 8; ++i) t->radix[a][i] = pl[a]->r[i];
    t->gather_rows = s.mr > 0 ? s.mr : auto_gather_rows<R>(c, s.rx);
    t->lines_per_block = s.mt > 0 ? s.mt : lines_per_block<R>(s.rx);
    t->interp_waves = s.waves;
    t->sync_every = s.sync;
    t->graph = s.graph;
    t->yz_engine = s.engine;
    t->x_engine = s.xeng;
    t->guess_order = s.guess;
    t->precond = s.precond;
    t->delay_block = s.dblock;
    t->interp_engine = s.ieng;
}

// EINVAL for malformed plans; shape_fits decides EUNSUPPORTED afterwards
int shape_from_c(const etaim_ctx* c, const etaim_tuning* t, Shape& s) {
    Radix* pl[3] = {&s.rx, &s.ry, &s.rz};
    for (int a = 0; a < 3; ++a) {
        *pl[a] = Radix{};
        pl[a]->L = c->gd.L[a];
        long prod = 1;
        for (int i = 0; i < 8 && t->radix[a][i] != 0; ++i) {
            if (!radix_supported(t->radix[a][i]))
                return fail(ETAIM_EINVAL, "radix " + std::to_string(t->radix[a][i]) + " is not supported");
            pl[a]->r[pl[a]->n++] = t->radix[a][i];
            prod *= t->radix[a][i];
        }
        if (prod != c->gd.L[a])
            return fail(ETAIM_EINVAL, "radix plan of axis " + std::to_string(a) + " does not multiply to " +
                                          std::to_string(c->gd.L[a]));
    }
    if (t->gather_rows < 1 || t->lines_per_block < 1 || t->interp_waves < 1 || t->sync_every < 1)
        return fail(ETAIM_EINVAL, "gather_rows, lines_per_block, interp_waves and sync_every must be >= 1");
    if (t->graph < 0 || t->graph > 2) return fail(ETAIM_EINVAL, "graph must be 0, 1 or 2");
    s.mr = t->gather_rows;
    s.mt = t->lines_per_block;
    s.waves = t->interp_waves;
    s.sync = t->sync_every;
    s.graph = t->graph;
    s.engine = t->yz_engine;
    s.xeng = t->x_engine;
    s.guess = t->guess_order;
    s.precond = t->precond;
    s.dblock = t->delay_block;
    s.ieng = t->interp_engine;
    return ETAIM_OK;
}

std::string tune_key(const etaim_ctx* c) {
    char k[256];
    std::snprintf(k, sizeof k, "etaim-gfx950 prec=%d B=%d ns=%d nnz=%d grid=%dx%dx%d ng=%d mn=%d restart=%d%s",
                  c->prec, c->B, c->ns, c->nnz, c->gd.N[0], c->gd.N[1], c->gd.N[2], c->st.ng, c->st.mn,
                  c->prm.restart, c->st.cfie ? " cfie" : "");
    return k;
}

// ---- JSON-lines cache (one flat object per line, written by cache_append)
bool json_int(const std::string& line, const char* name, long& v) {
    const std::string pat = std::string("\"") + name + "\":";
    size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    p += pat.size();
    while (p < line.size() && line[p] == ' ') ++p;
    char* end = nullptr;
    v = std::strtol(line.c_str() + p, &end, 10);
    return end != line.c_str() + p;
}

bool json_ints(const std::string& line, const char* name, int* out, int cap) {
    const std::string pat = std::string("\"") + name + "\": [";
    size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    p += pat.size();
    for (int i = 0; i < cap; ++i) out[i] = 0;
    int n = 0;
    while (p < line.size() && line[p] != ']' && n < cap) {
        char* end = nullptr;
        const long v = std::strtol(line.c_str() + p, &end, 10);
        if (end == line.c_str() + p) return false;
        out[n++] = (int)v;
        p = (size_t)(end - line.c_str());
        while (p < line.size() && (line[p] == ',' || line[p] == ' ')) ++p;
    }
    return n > 0;
}

bool cache_lookup(const char* path, const std::string& key, etaim_tuning& t) {
    std::FILE* f = std::fopen(path, "r");
    if (!f) return false;
    std::string line;
    bool found = false;
    char buf[4096];
    while (std::fgets(buf, sizeof buf, f)) {
        line = buf;
        if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
        std::memset(&t, 0, sizeof t);
        long v[11];
        if (json_ints(line, "radix_x", t.radix[0], 8) && json_ints(line, "radix_y", t.radix[1], 8) &&
            json_ints(line, "radix_z", t.radix[2], 8) && json_int(line, "gather_rows", v[0]) &&
            json_int(line, "lines_per_block", v[1]) && json_int(line, "interp_waves", v[2]) &&
            json_int(line, "sync_every", v[3]) && json_int(line, "graph", v[4]) &&
            json_int(line, "yz_engine", v[5]) && json_int(line, "x_engine", v[6]) &&
            json_int(line, "guess_order", v[7]) && json_int(line, "precond", v[8]) &&
            json_int(line, "delay_block", v[9]) && json_int(line, "interp_engine", v[10])) {
            t.gather_rows = (int)v[0];
            t.lines_per_block = (int)v[1];
            t.interp_waves = (int)v[2];
            t.sync_every = (int)v[3];
            t.graph = (int)v[4];
            t.yz_engine = (int)v[5];
            t.x_engine = (int)v[6];
            t.guess_order = (int)v[7];
            t.precond = (int)v[8];
            t.delay_block = (int)v[9];
            t.interp_engine = (int)v[10];
            found = true;  // the last matching record wins
        }
    }
    std::fclose(f);
    return found;
}

int cache_append(const char* path, const std::string& key, const etaim_tuning& t) {
    std::FILE* f = std::fopen(path, "a");
    if (!f) return fail(ETAIM_EINVAL, std::string("cannot write the tuning cache ") + path);
    auto arr = [](const int32_t* r) {
        std::string s = "[";
        for (int i = 0; i < 8 && r[i]; ++i) s += (i ? ", " : "") + std::to_string(r[i]);
        return s + "]";
    };
    std::fprintf(f,
                 "{\"key\": \"%s\", \"radix_x\": %s, \"radix_y\": %s, \"radix_z\": %s, \"gather_rows\": %d, "
                 "\"lines_per_block\": %d, \"interp_waves\": %d, \"sync_every\": %d, \"graph\": %d, "
                 "\"yz_engine\": %d, \"x_engine\": %d, \"guess_order\": %d, \"precond\": %d, \"delay_block\": %d, "
                 "\"interp_engine\": %d, \"apply_ms\": %.4f, \"solve_ms\": %.3f}\n",
                 key.c_str(), arr(t.radix[0]).c_str(), arr(t.radix[1]).c_str(), arr(t.radix[2]).c_str(),
                 t.gather_rows, t.lines_per_block, t.interp_waves, t.sync_every, t.graph, t.yz_engine, t.x_engine, t.guess_order, t.precond, t.delay_block, t.interp_engine, t.apply_ms,
                 t.solve_ms);
    std::fclose(f);
    return ETAIM_OK;
}

// ---- timing
struct TuneBufs {
    zd *x = nullptr, *y = nullptr, *rhs = nullptr, *sol = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~TuneBufs() {
        for (zd* p : {x, y, rhs, sol})
            if (p) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

template <typename R>
int time_apply(etaim_ctx* c, TuneBufs& b, int reps, double& ms) {
    CHK(Ops<R>::apply(c, 0, b.x, nullptr, b.y, 0));
    HIPCHK(hipEventRecord(b.e0, c->stream));
    for (int i = 0; i < reps; ++i) CHK(Ops<R>::apply(c, 0, b.x, nullptr, b.y, 0));
    HIPCHK(hipEventRecord(b.e1, c->stream));
    HIPCHK(hipEventSynchronize(b.e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, b.e0, b.e1));
    ms = t / reps;
    return ETAIM_OK;
}

template <typename R>
int time_solve(etaim_ctx* c, TuneBufs& b, double& ms, int& iters) {
    const size_t nB = (size_t)c->B * c->ns;
    HIPCHK(hipMemsetAsync(b.sol, 0, nB * sizeof(zd), c->stream));
    HIPCHK(hipEventRecord(b.e0, c->stream));
    StepResult res;
    CHK(gmres<R>(c, b.rhs, b.sol, 0, res));
    HIPCHK(hipEventRecord(b.e1, c->stream));
    HIPCHK(hipEventSynchronize(b.e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, b.e0, b.e1));
    ms = t;
    iters = res.iters;
    return ETAIM_OK;
}

// history sums at 24 consecutive steps past N_g (every block length up to 8
// but 5 and 7 divides 24) over the ring as it stands; the block sums are
// dropped before and after, so a march that follows starts its own
template <typename R>
int time_delayed(etaim_ctx* c, TuneBufs& b, double& ms) {
    const int ng = c->st.ng, k = 24;
    set_far_r0(c, -1);
    CHK(Ops<R>::delayed(c, ng + 1, c->zero, b.y, 0));
    HIPCHK(hipEventRecord(b.e0, c->stream));
    for (int i = 0; i < k; ++i) CHK(Ops<R>::delayed(c, ng + 2 + i, c->zero, b.y, 0));
    HIPCHK(hipEventRecord(b.e1, c->stream));
    HIPCHK(hipEventSynchronize(b.e1));
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, b.e0, b.e1));
    ms = t / k;
    set_far_r0(c, -1);
    return ETAIM_OK;
}

int fetch(etaim_ctx* c, const zd* d, std::vector<zd>& h) {
    h.resize((size_t)c->B * c->ns);
    HIPCHK(hipMemcpyAsync(h.data(), d, h.size() * sizeof(zd), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return ETAIM_OK;
}

double rel_l2(const std::vector<zd>& a, const std::vector<zd>& b) {
    double num = 0, den = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double dx = a[i].x - b[i].x, dy = a[i].y - b[i].y;
        if (!std::isfinite(dx) || !std::isfinite(dy)) return INFINITY;
        num += dx * dx + dy * dy;
        den += b[i].x * b[i].x + b[i].y * b[i].y;
    }
    return den > 0 ? std::sqrt(num / den) : std::sqrt(num);
}

template <typename R>
int autotune_impl(etaim_ctx* c, int budget_ms, etaim_tuning* out) {
    const size_t nB = (size_t)c->B * c->ns;
    const double tol = sizeof(R) == 4 ? 1e-4 : 1e-10;
    const bool prof = c->prof;
    c->prof = false;
    c->iter_hint = 0;
    TuneBufs b;
    HIPCHK(hipMalloc(&b.x, nB * sizeof(zd)));
    HIPCHK(hipMalloc(&b.y, nB * sizeof(zd)));
    HIPCHK(hipMalloc(&b.rhs, nB * sizeof(zd)));
    HIPCHK(hipMalloc(&b.sol, nB * sizeof(zd)));
    HIPCHK(hipEventCreate(&b.e0));
    HIPCHK(hipEventCreate(&b.e1));
    {
        // seeded uniform(-1, 1) entries (64-bit LCG, Knuth's MMIX constants)
        std::vector<zd> h(nB);
        uint64_t st = 0x9E3779B97F4A7C15ull;
        auto u = [&]() {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            return (double)(st >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        };
        for (auto& v : h) v = zd{u(), u()};
        HIPCHK(hipMemcpy(b.x, h.data(), nB * sizeof(zd), hipMemcpyHostToDevice));
        for (auto& v : h) v = zd{u(), u()};
        HIPCHK(hipMemcpy(b.rhs, h.data(), nB * sizeof(zd), hipMemcpyHostToDevice));
    }
    const auto t_start = std::chrono::steady_clock::now();
    auto spent = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    };
    Shape best = get_shape(c);
    best.graph = 0;
    best.sync = 1;
    put_shape(c, best);
    std::vector<zd> yref, y;
    double t_best = 0;
    CHK(time_apply<R>(c, b, 3, t_best));
    CHK(fetch(c, b.y, yref));
    // one candidate: time it if it fits, keep it if faster and equal to the reference
    auto trial = [&](const Shape& s) -> int {
        if (!shape_fits<R>(c, s) || spent() > budget_ms) return ETAIM_OK;
        put_shape(c, s);
        double t = 0;
        CHK(time_apply<R>(c, b, 3, t));
        CHK(fetch(c, b.y, y));
        if (rel_l2(y, yref) <= tol && t < t_best) {
            t_best = t;
            best = s;
        }
        put_shape(c, best);
        return ETAIM_OK;
    };
    for (int eng : {0, 1, 2, 3})
        if (eng != best.engine) {
            Shape s = best;
            s.engine = eng;
            CHK(trial(s));
        }
    for (int eng : {0, 1})
        if (eng != best.xeng) {
            Shape s = best;
            s.xeng = eng;
            CHK(trial(s));
        }
    for (const Radix& p : candidate_plans(c->gd.L[0]))
        if (!radix_equal(p, best.rx)) {
            Shape s = best;
            s.rx = p;
            s.mr = s.mt = 0;
            CHK(trial(s));
        }
    for (const Radix& p : candidate_plans(c->gd.L[1]))
        if (!radix_equal(p, best.ry)) {
            Shape s = best;
            s.ry = p;
            CHK(trial(s));
        }
    for (const Radix& p : candidate_plans(c->gd.L[2]))
        if (!radix_equal(p, best.rz)) {
            Shape s = best;
            s.rz = p;
            CHK(trial(s));
        }
    for (int mr : {1, 2, 4, 8, 16, 32}) {
        Shape s = best;
        s.mr = mr;
        CHK(trial(s));
    }
    for (int mt : {2, 4, 8, 16, 32, 64}) {
        Shape s = best;
        s.mt = mt;
        CHK(trial(s));
    }
    for (int w : {1, 2, 4}) {
        Shape s = best;
        s.waves = w;
        CHK(trial(s));
    }
    {
        Shape s = best;
        s.ieng = 1 - best.ieng;
        CHK(trial(s));
    }
    // freeze the automatic choices so that the record is explicit
    if (best.mr == 0) best.mr = auto_gather_rows<R>(c, best.rx);
    if (best.mt == 0) best.mt = lines_per_block<R>(best.rx);
    put_shape(c, best);
    // time blocks of the delayed field (register and line-pass engines)
    if ((best.engine == 1 || best.engine == 2 || best.engine == 3) && c->st.ng > 2) {
        double d_best = 0;
        CHK(time_delayed<R>(c, b, d_best));
        for (int pb : {1, 2, 3, 4, 5, 6, 7, 8}) {
            Shape s = best;
            s.dblock = pb;
            if (pb == best.dblock || !shape_fits<R>(c, s) || spent() > budget_ms) continue;
            put_shape(c, s);
            double t = 0;
            CHK(time_delayed<R>(c, b, t));
            if (t < d_best) {
                d_best = t;
                best.dblock = pb;
            }
        }
        put_shape(c, best);
    }
    // GMRES schedule: solves of the seeded right-hand side (identical
    // iterates whatever the schedule; only the time differs)
    double s_best = 0;
    int it_ref = 0;
    CHK(time_solve<R>(c, b, s_best, it_ref));
    for (int graph : {0, 1})
        for (int sync : {1, 2, 3, 4, 6, 8}) {
            Shape s = best;
            s.graph = graph;
            s.sync = sync;
            if ((graph == 0 && sync == 1) || !shape_fits<R>(c, s) || spent() > budget_ms) continue;
            put_shape(c, s);
            double t = 0;
            int it = 0;
            if (graph) CHK(time_solve<R>(c, b, t, it));  // first solve captures the steps
            CHK(time_solve<R>(c, b, t, it));
            if (it == it_ref && t < s_best) {
                s_best = t;
                best.graph = graph;
                best.sync = sync;
            }
        }
    put_shape(c, best);
    c->prof = prof;
    if (out) {
        shape_to_c<R>(c, best, out);
        out->apply_ms = t_best;
        out->solve_ms = s_best;
    }
    return ETAIM_OK;
}
