// Host build of one generated level program, checked against central differences.
// Compiled and run by tests/test_codegen_host.py; prints "name max_rel_err" lines.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#define __device__
#define __forceinline__ inline
#define __restrict__
#define MTP_BLOCK_FENCE()
using std::fma;
#include MTP_LEVEL_HEADER

using L = MTP_LEVEL_STRUCT;

struct RegM {
  const double* m;
  double operator()(int e) const { return m[e]; }
};

static std::mt19937_64 rng(12345);
static double unif(double a, double b) { return std::uniform_real_distribution<double>(a, b)(rng); }

static double relerr(const std::vector<double>& a, const std::vector<double>& b) {
  double num = 0, den = 1e-300;
  for (size_t k = 0; k < a.size(); ++k) {
    num = std::fmax(num, std::fabs(a[k] - b[k]));
    den = std::fmax(den, std::fabs(b[k]));
  }
  return num / den;
}

// smooth stand-ins for the radial functions
static void radial(double r, double* f, double* fp) {
  for (int mu = 0; mu < L::NMU; ++mu) {
    f[mu] = std::sin(0.7 * (mu + 1) * r) + 0.3;
    fp[mu] = 0.7 * (mu + 1) * std::cos(0.7 * (mu + 1) * r);
  }
}

static void moments_of(const std::vector<double>& d, std::vector<double>& m) {
  m.assign(L::NMOM, 0.0);
  const int np = (int)d.size() / 3;
  for (int p = 0; p < np; ++p) {
    double x = d[3 * p], y = d[3 * p + 1], z = d[3 * p + 2];
    double r = std::sqrt(x * x + y * y + z * z), f[L::NMU], fp[L::NMU];
    radial(r, f, fp);
    double part[L::NMOM];
    for (int g = 0; g < L::NGROUP; ++g) {
      for (int e = 0; e < L::NMOM; ++e) part[e] = 0.0;
      const int lo = L::GROUP_LO[g];
      if (g == 0) L::acc_moments<0>(part, f, x, y, z);
#if MTP_NGROUP > 1
      if (g == 1) L::acc_moments<1>(part, f, x, y, z);
#endif
#if MTP_NGROUP > 2
      if (g == 2) L::acc_moments<2>(part, f, x, y, z);
#endif
      for (int e = lo; e < L::GROUP_HI[g]; ++e) m[e] += part[e - lo];
    }
  }
}

template <int G>
static void tan_range(const std::vector<double>& d, const std::vector<double>& dl, std::vector<double>& md) {
  const int np = (int)d.size() / 3;
  const int lo = L::TGROUP_LO[G];
  for (int p = 0; p < np; ++p) {
    double x = d[3 * p], y = d[3 * p + 1], z = d[3 * p + 2];
    double r = std::sqrt(x * x + y * y + z * z), f[L::NMU], fp[L::NMU];
    radial(r, f, fp);
    const double rdot = (x * dl[3 * p] + y * dl[3 * p + 1] + z * dl[3 * p + 2]) / r;
    double part[L::NMOM] = {0};
    L::tan_moments<G>(part, f, fp, x, y, z, dl[3 * p], dl[3 * p + 1], dl[3 * p + 2], rdot);
    for (int e = lo; e < L::TGROUP_HI[G]; ++e) md[e] += part[e - lo];
  }
}

// tangent of the moments over every moment-tangent range of the level
template <int G>
static void tan_group(const std::vector<double>& d, const std::vector<double>& dl, std::vector<double>& md) {
  if constexpr (G < L::NTGROUP) {
    tan_range<G>(d, dl, md);
    tan_group<G + 1>(d, dl, md);
  }
}

// every adjoint group of the level, each over its own moment range
template <int G>
static void adj_pair_groups(const double* mb, const double* mbd, double x, double y, double z, double ex,
                            double ey, double ez, double* S, double* A) {
  if constexpr (G < L::NAGROUP) {
    L::adj_pair<G>(mb + L::AGROUP_LO[G], mbd + L::AGROUP_LO[G], x, y, z, ex, ey, ez, S, A);
    adj_pair_groups<G + 1>(mb, mbd, x, y, z, ex, ey, ez, S, A);
  }
}

// every part of the reverse-tangent program, in order, into one output vector
template <int P>
static void rev_tan_parts(const double* m, const double* md, const double* Cb, const double* Cbd, double* out) {
  if constexpr (P < L::NRTPART) {
    L::rev_tan<P, double>(RegM{m}, RegM{md}, Cb, Cbd, out, 1);
    rev_tan_parts<P + 1>(m, md, Cb, Cbd, out);
  }
}

int main() {
  const int np = 6;
  std::vector<double> d(3 * np), dl(3 * np);
  for (int p = 0; p < np; ++p) {
    double r = unif(2.2, 4.5), th = unif(0, 3.14159), ph = unif(0, 6.28318);
    d[3 * p] = r * std::sin(th) * std::cos(ph);
    d[3 * p + 1] = r * std::sin(th) * std::sin(ph);
    d[3 * p + 2] = r * std::cos(th);
    for (int k = 0; k < 3; ++k) dl[3 * p + k] = unif(-1, 1);
  }
  const double h = 1e-6;
  // ---- tangent of the moments
  std::vector<double> m, mp, mm, md(L::NMOM, 0.0), fd(L::NMOM);
  moments_of(d, m);
  {
    std::vector<double> dp = d, dm = d;
    for (size_t k = 0; k < d.size(); ++k) { dp[k] += h * dl[k]; dm[k] -= h * dl[k]; }
    moments_of(dp, mp);
    moments_of(dm, mm);
    for (int e = 0; e < L::NMOM; ++e) fd[e] = (mp[e] - mm[e]) / (2 * h);
    tan_group<0>(d, dl, md);
    std::printf("tan_moments %.3e\n", relerr(md, fd));
  }
  // ---- forward tangent of the contractions
  std::vector<double> C(L::NCOMP), Cd(L::NCOMP), Cp(L::NCOMP), Cm(L::NCOMP), fdC(L::NCOMP);
  {
    L::fwd_tan<double>(RegM{m.data()}, RegM{md.data()}, C.data(), Cd.data());
    std::vector<double> mpl(L::NMOM), mmi(L::NMOM);
    for (int e = 0; e < L::NMOM; ++e) { mpl[e] = m[e] + h * md[e]; mmi[e] = m[e] - h * md[e]; }
    L::fwd<double>(RegM{mpl.data()}, Cp.data());
    L::fwd<double>(RegM{mmi.data()}, Cm.data());
    for (int q = 0; q < L::NCOMP; ++q) fdC[q] = (Cp[q] - Cm[q]) / (2 * h);
    std::vector<double> C0(L::NCOMP);
    L::fwd<double>(RegM{m.data()}, C0.data());
    std::printf("fwd_value %.3e\n", relerr(C, C0));
    std::printf("fwd_tan %.3e\n", relerr(Cd, fdC));
  }
  // ---- products with tangents
  std::vector<double> xi(L::NALPHA);
  for (auto& v : xi) v = unif(-1, 1);
  const double ebar = 0.37;
  std::vector<double> Cb(L::NCOMP), Cbd(L::NCOMP), out(L::NALPHA);
  {
    L::products_tan<double>(C.data(), Cd.data(), xi.data(), ebar, Cb.data(), Cbd.data(), out.data(), 1);
    std::vector<double> Bp(L::NALPHA), Bm(L::NALPHA), B0(L::NALPHA), Cbp(L::NCOMP), Cbm(L::NCOMP), Cb0(L::NCOMP);
    std::vector<double> Cpl(L::NCOMP), Cmi(L::NCOMP);
    for (int q = 0; q < L::NCOMP; ++q) { Cpl[q] = C[q] + h * Cd[q]; Cmi[q] = C[q] - h * Cd[q]; }
    L::products<true, double>(Cpl.data(), xi.data(), Cbp.data(), Bp.data(), 1);
    L::products<true, double>(Cmi.data(), xi.data(), Cbm.data(), Bm.data(), 1);
    L::products<true, double>(C.data(), xi.data(), Cb0.data(), B0.data(), 1);
    std::vector<double> want(L::NALPHA), cbdw(L::NCOMP);
    for (int a = 0; a < L::NALPHA; ++a) want[a] = ebar * B0[a] - (Bp[a] - Bm[a]) / (2 * h);
    for (int q = 0; q < L::NCOMP; ++q) cbdw[q] = (Cbp[q] - Cbm[q]) / (2 * h);
    std::printf("products_out %.3e\n", relerr(out, want));
    std::printf("products_cb %.3e\n", relerr(Cb, Cb0));
    std::printf("products_cbd %.3e\n", relerr(Cbd, cbdw));
  }
  // ---- reverse tangent
  {
    std::vector<double> mbd(L::NMOM, 0.0), want(L::NMOM);
    std::vector<double> mpl(L::NMOM), mmi(L::NMOM), cbp(L::NCOMP), cbm(L::NCOMP);
    for (int e = 0; e < L::NMOM; ++e) { mpl[e] = m[e] + h * md[e]; mmi[e] = m[e] - h * md[e]; }
    for (int q = 0; q < L::NCOMP; ++q) { cbp[q] = Cb[q] + h * Cbd[q]; cbm[q] = Cb[q] - h * Cbd[q]; }
    std::vector<double> rp(L::NMOM, 0.0), rm(L::NMOM, 0.0);
    // the parts store or add their entries; poison mbd first so that a missed store shows
    for (auto& v : mbd) v = 1e300;
    rev_tan_parts<0>(m.data(), md.data(), Cb.data(), Cbd.data(), mbd.data());
    for (int g = 0; g < L::NGROUP; ++g) {
      const int lo = L::GROUP_LO[g];
      double* pp = rp.data() + lo;
      double* pm = rm.data() + lo;
      if (g == 0) {
        L::rev<0>(RegM{mpl.data()}, cbp.data(), pp);
        L::rev<0>(RegM{mmi.data()}, cbm.data(), pm);
      }
#if MTP_NGROUP > 1
      if (g == 1) {
        L::rev<1>(RegM{mpl.data()}, cbp.data(), pp);
        L::rev<1>(RegM{mmi.data()}, cbm.data(), pm);
      }
#endif
#if MTP_NGROUP > 2
      if (g == 2) {
        L::rev<2>(RegM{mpl.data()}, cbp.data(), pp);
        L::rev<2>(RegM{mmi.data()}, cbm.data(), pm);
      }
#endif
    }
    for (int e = 0; e < L::NMOM; ++e) want[e] = (rp[e] - rm[e]) / (2 * h);
    std::printf("rev_tan %.3e\n", relerr(mbd, want));
  }
  // ---- pair gradient: grad_d of sum_e mb_e f_mu(r) mono_e(d) against central differences
  {
    std::vector<double> mb(L::NMOM);
    for (auto& v : mb) v = unif(-1, 1);
    auto energy = [&](double x, double y, double z) {
      double r = std::sqrt(x * x + y * y + z * z), f[L::NMU], fp[L::NMU];
      radial(r, f, fp);
      std::vector<double> m(L::NMOM, 0.0);
      for (int g = 0; g < L::NGROUP; ++g) {
        double part[L::NMOM] = {0};
        const int lo = L::GROUP_LO[g];
        if (g == 0) L::acc_moments<0>(part, f, x, y, z);
#if MTP_NGROUP > 1
        if (g == 1) L::acc_moments<1>(part, f, x, y, z);
#endif
#if MTP_NGROUP > 2
        if (g == 2) L::acc_moments<2>(part, f, x, y, z);
#endif
        for (int e = lo; e < L::GROUP_HI[g]; ++e) m[e] = part[e - lo];
      }
      double e = 0;
      for (int k = 0; k < L::NMOM; ++k) e += mb[k] * m[k];
      return e;
    };
    double x = d[3], y = d[4], z = d[5];
    double r = std::sqrt(x * x + y * y + z * z), f[L::NMU], fp[L::NMU];
    radial(r, f, fp);
    double gx = 0, gy = 0, gz = 0, u = 0;
    // pair_grad takes the adjoints multiplied by a! b! c! of each entry
    std::vector<double> mbs(L::NMOM);
    for (int k = 0; k < L::NMOM; ++k) mbs[k] = mb[k] * L::MFACT[k];
    for (int g = 0; g < L::NGROUP; ++g) {
      const int lo = L::GROUP_LO[g];
      if (g == 0) L::pair_grad<0>(mbs.data() + lo, f, fp, x, y, z, gx, gy, gz, u);
#if MTP_NGROUP > 1
      if (g == 1) L::pair_grad<1>(mbs.data() + lo, f, fp, x, y, z, gx, gy, gz, u);
#endif
#if MTP_NGROUP > 2
      if (g == 2) L::pair_grad<2>(mbs.data() + lo, f, fp, x, y, z, gx, gy, gz, u);
#endif
    }
    std::vector<double> got = {gx + u * x / r, gy + u * y / r, gz + u * z / r}, want(3);
    want[0] = (energy(x + h, y, z) - energy(x - h, y, z)) / (2 * h);
    want[1] = (energy(x, y + h, z) - energy(x, y - h, z)) / (2 * h);
    want[2] = (energy(x, y, z + h) - energy(x, y, z - h)) / (2 * h);
    std::printf("pair_grad %.3e\n", relerr(got, want));
  }
  // ---- adjoint pair sums against the plain definition
  {
    std::vector<double> mb(L::NMOM), mbd(L::NMOM);
    for (int e = 0; e < L::NMOM; ++e) { mb[e] = unif(-1, 1); mbd[e] = unif(-1, 1); }
    double x = d[0], y = d[1], z = d[2], ex = dl[0], ey = dl[1], ez = dl[2];
    std::vector<double> S(L::NMU, 0.0), A(L::NMU, 0.0), Sw(L::NMU, 0.0), Aw(L::NMU, 0.0);
    adj_pair_groups<0>(mb.data(), mbd.data(), x, y, z, ex, ey, ez, S.data(), A.data());
    for (int e = 0; e < L::NMOM; ++e) {
      const int mu = L::ENTRIES[e][0], a = L::ENTRIES[e][1], b = L::ENTRIES[e][2], c = L::ENTRIES[e][3];
      const double mono = std::pow(x, a) * std::pow(y, b) * std::pow(z, c);
      const double dm = (a ? a * std::pow(x, a - 1) * std::pow(y, b) * std::pow(z, c) * ex : 0.0) +
                        (b ? b * std::pow(x, a) * std::pow(y, b - 1) * std::pow(z, c) * ey : 0.0) +
                        (c ? c * std::pow(x, a) * std::pow(y, b) * std::pow(z, c - 1) * ez : 0.0);
      Sw[mu] += mb[e] * mono;
      Aw[mu] += mbd[e] * mono + mb[e] * dm;
    }
    std::printf("adj_pair_S %.3e\n", relerr(S, Sw));
    std::printf("adj_pair_A %.3e\n", relerr(A, Aw));
  }
  return 0;
}
