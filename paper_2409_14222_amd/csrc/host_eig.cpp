// Eigenvalues of a small upper Hessenberg matrix (host).  The Chebyshev
// smoother of Sec. 3 needs the largest eigenvalue of the relaxation-
// preconditioned operator on each level; the Arnoldi vectors are formed on the
// device and only the k x k Hessenberg matrix of the recurrence (k = 10 by
// default) comes here.
//
// Method: the shifted QR algorithm on the Hessenberg form in complex
// arithmetic.  One step on the active window [l, hi] subtracts the shift mu,
// factors H - mu I = Q R by Givens rotations G_l .. G_{hi-1} (each zeroing one
// subdiagonal entry), and forms R Q + mu I, which is again Hessenberg and
// unitarily similar to H.  The shift is the eigenvalue of the trailing 2 x 2
// block nearer to its last diagonal entry (Wilkinson); a window whose last
// subdiagonal entry has not become negligible after 10 steps gets one
// exceptional shift.  A subdiagonal entry is negligible when it is at most the
// unit roundoff times the two adjacent diagonal magnitudes; the matrix then
// splits and the bottom entry of a 1 x 1 window is an eigenvalue.  Only the
// active window is updated: the off-window blocks do not change eigenvalues.
#include <cfloat>
#include <cmath>
#include <complex>
#include <vector>

#include "vk_internal.hpp"

namespace vk {

using cplx = std::complex<double>;

bool hessenberg_eigs(int n, const double* Hrm, std::vector<cplx>& ev) {
  ev.clear();
  if (n <= 0) return true;
  std::vector<cplx> A((size_t)n * n, 0.0);
  double scale = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = std::max(0, i - 1); j < n; ++j) {
      const double v = Hrm[(size_t)i * n + j];
      if (!std::isfinite(v)) return false;
      A[(size_t)i * n + j] = v;
      scale = std::max(scale, std::fabs(v));
    }
  auto a = [&](int i, int j) -> cplx& { return A[(size_t)i * n + j]; };
  const double eps = DBL_EPSILON;
  std::vector<cplx> gc(n), gs(n);
  int hi = n - 1, since = 0, total = 0;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = std::abs(a(l, l)) + std::abs(a(l - 1, l - 1));
      if (s == 0.0) s = scale;
      if (std::abs(a(l, l - 1)) <= eps * s) {
        a(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {
      ev.push_back(a(hi, hi));
      --hi;
      since = 0;
      continue;
    }
    if (++total > 100 * n) return false;
    ++since;
    // shift: eigenvalue of the trailing 2 x 2 block nearer to its last diagonal entry
    const cplx p = a(hi - 1, hi - 1), q = a(hi - 1, hi), r = a(hi, hi - 1), t = a(hi, hi);
    const cplx half = 0.5 * (p - t);
    const cplx root = std::sqrt(half * half + q * r);
    const cplx m1 = 0.5 * (p + t) + root, m2 = 0.5 * (p + t) - root;
    cplx mu = std::abs(m1 - t) < std::abs(m2 - t) ? m1 : m2;
    if (since % 11 == 10) mu = t + 0.75 * std::abs(r) * cplx(1.0, 0.5);  // exceptional shift
    for (int i = l; i <= hi; ++i) a(i, i) -= mu;
    // H - mu I = Q R: rotations from the left zero the subdiagonal of the window
    for (int k = l; k < hi; ++k) {
      const cplx x = a(k, k), y = a(k + 1, k);
      const double nr = std::hypot(std::abs(x), std::abs(y));
      cplx c = 1.0, s = 0.0;
      if (nr > 0.0) {
        c = x / nr;
        s = y / nr;
      }
      gc[k] = c;
      gs[k] = s;
      for (int j = k; j <= hi; ++j) {
        const cplx u = a(k, j), v = a(k + 1, j);
        a(k, j) = std::conj(c) * u + std::conj(s) * v;
        a(k + 1, j) = -s * u + c * v;
      }
    }
    // R Q: the same rotations from the right, then add the shift back
    for (int k = l; k < hi; ++k) {
      const cplx c = gc[k], s = gs[k];
      const int iend = std::min(k + 2, hi);
      for (int i = l; i <= iend; ++i) {
        const cplx u = a(i, k), v = a(i, k + 1);
        a(i, k) = u * c + v * s;
        a(i, k + 1) = -u * std::conj(s) + v * std::conj(c);
      }
    }
    for (int i = l; i <= hi; ++i) a(i, i) += mu;
  }
  return true;
}

}  // namespace vk

extern "C" vk_status vk_hessenberg_eigenvalues(int n, const double* h_H, double* h_re, double* h_im) {
  if (n < 1 || n > 512 || !h_H || !h_re || !h_im) return VK_EINVAL;
  std::vector<vk::cplx> ev;
  if (!vk::hessenberg_eigs(n, h_H, ev)) return VK_ENAN;
  for (int i = 0; i < n; ++i) {
    h_re[i] = ev[i].real();
    h_im[i] = ev[i].imag();
  }
  return VK_OK;
}
