// Host replay of the tile engine's index arithmetic for every precision (FP64 included), tile
// width and the network shapes of the workloads: the LDS layout's regions stay inside the
// layout and do not overlap, every fragment-ordered and D-slot index of the activation, delta,
// weight and partial-sum buffers stays inside its buffer, fragment offsets are a bijection,
// and the activation scratch index stays inside one workgroup's stride.  Built with hipcc and
// run by tests/test_layout_cpu.py; prints the number of checks or the first failure.
#include <cstdio>
#include <vector>

#include "../paper_2606_04895_amd/csrc/layout.hpp"

using namespace best;

static long n_checks = 0;
static int failed = 0;

#define CHECK(cond, ...)                                                      \
  do {                                                                        \
    ++n_checks;                                                               \
    if (!(cond) && !failed) {                                                 \
      failed = 1;                                                             \
      std::printf("FAIL %s:%d: %s | ", __FILE__, __LINE__, #cond);            \
      std::printf(__VA_ARGS__);                                               \
      std::printf("\n");                                                      \
    }                                                                         \
  } while (0)

struct Shape {
  int d, H, nh;
};

// fragment-order bijection on a rows x (KS * KSTEP) matrix
template <class P>
static void check_frag(int rows, int KS) {
  const int64_t n = (int64_t)rows * KS * P::KSTEP;
  std::vector<char> seen(n, 0);
  for (int r = 0; r < rows; ++r)
    for (int k = 0; k < KS * P::KSTEP; ++k) {
      const int64_t o = frag_offset<P>(r, k, KS);
      CHECK(o >= 0 && o < n, "frag row %d k %d KS %d -> %ld of %ld", r, k, KS, (long)o, (long)n);
      if (o >= 0 && o < n) {
        CHECK(!seen[o], "frag offset %ld hit twice", (long)o);
        seen[o] = 1;
      }
    }
}

// D-slot accesses of lds_store4 / lds_load4 into an M x H B-fragment buffer: rows
// rt*16 + drow(g, r) (the FP32-class instructions store rows 4g .. 4g + 3 as one vector)
template <class P>
static void check_dslots(int M, int H) {
  const int KS = H / P::KSTEP;
  for (int rt = 0; rt < H / 16; ++rt)
    for (int g = 0; g < 4; ++g)
      for (int c = 0; c < M; ++c)
        for (int r = 0; r < 4; ++r) {
          const int row = P::ROWS4 ? rt * 16 + 4 * g + r : rt * 16 + P::drow(g, r);
          const int o = P::ROWS4 ? lds_off<P>(rt * 16 + 4 * g, c, KS) + r : lds_off<P>(row, c, KS);
          CHECK(o >= 0 && o < M * H, "dslot rt %d g %d c %d r %d -> %d of %d", rt, g, c, r, o, M * H);
          CHECK(o == lds_off<P>(row, c, KS), "dslot vector layout rt %d g %d r %d", rt, g, r);
        }
}

struct Region {
  const char* name;
  int lo, hi;
};

template <class P>
static void check_config(int prec, int MT, const Shape& s, int lds_h, int st_lds, int w1) {
  using IP = typename InPrec<P>::type;
  const int M = 16 * MT, H = s.H, d = s.d, nh = s.nh;
  const LdsLayout L = layout_for(prec, MT, H, d, nh, lds_h, st_lds, w1);
  const int ts = tsize(prec), va = vasize(prec), waves = tile_waves(ts);
  const int MH = M * H * ts;
  const int mlp_bytes = (lds_h ? nh + 2 : 2) * MH;
  const int asm_bytes = 8 * (2 * d * M + M + M * d + kMaxD + 3 * kMaxTerms + waves * 32);
  std::vector<Region> rg;
  rg.push_back({"big", L.big, L.big + (mlp_bytes > asm_bytes ? mlp_bytes : asm_bytes)});
  rg.push_back({"th", L.th, L.th + M * in_ksteps(prec, d) * in_kstep(prec) * in_size(prec)});
  rg.push_back({"gth", L.gth, L.gth + M * d * va});
  const int red_bytes = waves * M * d * va;
  const int dlt0 = lds_h ? nh * MH : ((nh - 1) & 1) * MH;
  const int dlt1 = lds_h ? (nh + 1) * MH : (nh & 1) * MH;
  const int d1_buf = ((nh - 1) & 1) == 0 ? dlt0 : dlt1;  // the delta buffer holding delta_1
  if (L.red >= L.big && L.red < L.big + mlp_bytes) {
    // inside the delta buffer that does not hold delta_1
    const int other = d1_buf == dlt0 ? dlt1 : dlt0;
    CHECK(L.red == L.big + other, "red not at the free delta buffer");
    CHECK(red_bytes <= MH, "red %d larger than a delta buffer %d", red_bytes, MH);
  } else {
    rg.push_back({"red", L.red, L.red + red_bytes});
  }
  rg.push_back({"outp", L.outp, L.outp + waves * M * va});
  rg.push_back({"out", L.out, L.out + M * va});
  rg.push_back({"up", L.up, L.up + M * va});
  rg.push_back({"mi", L.mi, L.mi + 4 * M * 4});
  rg.push_back({"md", L.md, L.md + 8 * M * 8});
  if (st_lds == 1) {
    CHECK(L.st >= 0 && L.cst >= 0, "st_lds without regions");
    rg.push_back({"st", L.st, L.st + (7 * d * M + M) * 8});
    rg.push_back({"cst", L.cst, L.cst + (2 * d * d + 8 * d) * 8});
  } else if (st_lds == 2) {  // the launch constants alone
    CHECK(L.st < 0 && L.cst >= 0, "constants-only layout");
    rg.push_back({"cst", L.cst, L.cst + (2 * d * d + 8 * d) * 8});
  } else {
    CHECK(L.st < 0 && L.cst < 0, "regions without st_lds");
  }
  if (w1) {
    CHECK(L.w1 >= 0 && L.w1f_bytes == (int)w1f_bytes(prec, H, d) &&
              L.w1t_bytes == (int)w1t_bytes(prec, H, d), "w1 region sizes");
    rg.push_back({"w1", L.w1, L.w1 + L.w1f_bytes + L.w1t_bytes});
  } else {
    CHECK(L.w1 < 0, "w1 region without residency");
  }
  for (size_t i = 0; i < rg.size(); ++i) {
    CHECK(rg[i].lo >= 0 && rg[i].lo % 16 == 0 && rg[i].hi <= L.total, "region %s [%d, %d) of %d",
          rg[i].name, rg[i].lo, rg[i].hi, L.total);
    for (size_t j = i + 1; j < rg.size(); ++j)
      CHECK(rg[i].hi <= rg[j].lo || rg[j].hi <= rg[i].lo, "regions %s and %s overlap",
            rg[i].name, rg[j].name);
  }
  // activation / delta buffers: every D-slot access in an M x H buffer; the buffers are
  // consecutive M x H slices of big
  check_dslots<P>(M, H);
  CHECK(dlt0 + MH <= mlp_bytes && dlt1 + MH <= mlp_bytes, "delta buffers inside big");
  // input layer B fragments (M chains x K1 inputs) inside th
  {
    const int ks1 = in_ksteps(prec, d);
    for (int c = 0; c < M; ++c)
      for (int i = 0; i < ks1 * IP::KSTEP; ++i) {
        const int64_t o = frag_offset<IP>(c, i, ks1);
        CHECK(o >= 0 && o < (int64_t)M * ks1 * IP::KSTEP, "th c %d i %d", c, i);
      }
  }
  // input-gradient partial sums red[(wv * M + ct * 16 + cl) * d + i] and their sum into gth
  {
    int64_t mx = 0;
    for (int wv = 0; wv < waves; ++wv)
      for (int ct = 0; ct < MT; ++ct)
        for (int cl = 0; cl < 16; ++cl)
          for (int i = 0; i < d; ++i) {
            const int64_t o = ((int64_t)wv * M + ct * 16 + cl) * d + i;
            mx = o > mx ? o : mx;
          }
    CHECK((mx + 1) * va <= red_bytes, "red index %ld", (long)mx);
  }
  // activation scratch of one workgroup: [layer][rt][ct][lane][4], stride nh H 16 MT
  {
    const int RT = H / 16;
    const int64_t stride = (int64_t)nh * H * 16 * MT;
    const int64_t o = hsave_index<1>(0, 0, 0, 0, 0);
    CHECK(o == 0, "hsave origin");
    int64_t mx = 0;
    for (int l = 0; l < nh; ++l)
      for (int rt = 0; rt < RT; rt += RT - 1 > 0 ? RT - 1 : 1)
        for (int ct = 0; ct < MT; ++ct)
          for (int lane = 0; lane < 64; lane += 63) {
            int64_t v = 0;
            switch (MT) {
              case 1: v = hsave_index<1>(l, RT, rt, ct, lane); break;
              case 2: v = hsave_index<2>(l, RT, rt, ct, lane); break;
              default: v = hsave_index<4>(l, RT, rt, ct, lane); break;
            }
            mx = v > mx ? v : mx;
          }
    CHECK(mx + 3 < stride, "hsave index %ld of stride %ld", (long)mx, (long)stride);
  }
}

template <class P>
static void check_prec(int prec, const std::vector<Shape>& shapes) {
  for (const Shape& s : shapes) {
    const int KS = s.H / P::KSTEP;
    check_frag<P>(s.H, KS);                                     // W_l and W_l^T
    check_frag<P>(16 * grad_rtiles(s.d), KS);                    // W_1^T
    using IP = typename InPrec<P>::type;
    check_frag<IP>(s.H, in_ksteps(prec, s.d));                   // W_1
    CHECK(w1f_bytes(prec, s.H, s.d) ==
              (size_t)s.H * in_ksteps(prec, s.d) * IP::KSTEP * sizeof(typename IP::T),
          "w1f bytes");
    CHECK(w1t_bytes(prec, s.H, s.d) == (size_t)16 * grad_rtiles(s.d) * s.H * sizeof(typename P::T),
          "w1t bytes");
    for (int MT = 1; MT <= mt_max(prec); MT *= 2)
      for (int lds_h = 0; lds_h <= 1; ++lds_h)
        for (int st = 0; st <= 2; ++st)
          for (int w1 = 0; w1 <= 1; ++w1) check_config<P>(prec, MT, s, lds_h, st, w1);
  }
}

int main() {
  // the workloads' networks (C1 .. C5), the test problems and the extremes of the API
  const std::vector<Shape> shapes = {{5, 128, 3},  {3, 128, 1},  {4, 128, 2},  {6, 128, 2},
                                     {6, 512, 4},  {12, 1024, 4}, {27, 1024, 5}, {32, 2048, 2},
                                     {1, 128, 16}};
  check_prec<Prec<double>>(BEST_FP64, shapes);
  check_prec<Prec<float>>(BEST_FP32, shapes);
  check_prec<Prec<_Float16>>(BEST_FP16, shapes);
  check_prec<Prec<__bf16>>(BEST_BF16, shapes);
  if (failed) return 1;
  std::printf("ok %ld checks\n", n_checks);
  return 0;
}
