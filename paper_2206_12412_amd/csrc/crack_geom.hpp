// Geometry of a straight crack that grows along a prescribed direction
// (Alg. 1 takes the direction d as an input).  Host and device use the same
// functions: the host severs the links of the initial crack, the crack step
// those of each increment.
//
// The crack lies on the line through S = (x0, yc) along the unit vector u; a
// tip is given by its line coordinate a, the point S + (a - x0) u (along +x,
// u = (1, 0), simply (a, yc)).  A link is severed when the closed segment
// between two line coordinates touches it (Sec. 4.1: links intersected by the
// crack carry no information; touching counts).  All arithmetic is FP64
// without contraction, so that host, device and every run agree bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace lbmk {
namespace geom {

struct Line {
  int aligned;       // u = (1, 0): the crack row y = yc, a = x
  double x0, yc;     // S
  double ux, uy;     // u
};

__host__ __device__ inline void point_at(const Line &L, double a, double *x, double *y) {
#pragma clang fp contract(off)
  if (L.aligned) {
    *x = a;
    *y = L.yc;
    return;
  }
  const double d = a - L.x0;
  *x = L.x0 + d * L.ux;
  *y = L.yc + d * L.uy;
}

// sign of the cross product (q - p) x (r - p)
__host__ __device__ inline int turn(double px, double py, double qx, double qy, double rx,
                                    double ry) {
#pragma clang fp contract(off)
  const double c = (qx - px) * (ry - py) - (qy - py) * (rx - px);
  return (c > 0.0) - (c < 0.0);
}

// r (collinear with p, q) inside the box spanned by p and q
__host__ __device__ inline bool in_box(double px, double py, double qx, double qy, double rx,
                                       double ry) {
  return (px < qx ? px : qx) <= rx && rx <= (px < qx ? qx : px) &&
         (py < qy ? py : qy) <= ry && ry <= (py < qy ? qy : py);
}

// closed segments a-b and c-d share a point
__host__ __device__ inline bool closed_segments_meet(double ax, double ay, double bx, double by,
                                                     double cx, double cy, double dx, double dy) {
  const int t1 = turn(cx, cy, dx, dy, ax, ay), t2 = turn(cx, cy, dx, dy, bx, by);
  const int t3 = turn(ax, ay, bx, by, cx, cy), t4 = turn(ax, ay, bx, by, dx, dy);
  if (t1 * t2 < 0 && t3 * t4 < 0) return true;
  return (t1 == 0 && in_box(cx, cy, dx, dy, ax, ay)) || (t2 == 0 && in_box(cx, cy, dx, dy, bx, by)) ||
         (t3 == 0 && in_box(ax, ay, bx, by, cx, cy)) || (t4 == 0 && in_box(ax, ay, bx, by, dx, dy));
}

// Does the crack between line coordinates a and b touch the link from site
// (i, j) to (i + di, j + dj)?
__host__ __device__ inline bool touches_link(const Line &L, double a, double b, int i, int j,
                                             int di, int dj) {
  double ax, ay, bx, by;
  point_at(L, a, &ax, &ay);
  point_at(L, b, &bx, &by);
  return closed_segments_meet(ax, ay, bx, by, (double)i, (double)j, (double)(i + di),
                              (double)(j + dj));
}

// Arc length from (x, y) along (ux, uy) to the wall rectangle
// [-1/2, nx - 1/2] x [-1/2, ny - 1/2] that (x, y) lies in.
inline double wall_distance(int nx, int ny, double x, double y, double ux, double uy) {
  double t = HUGE_VAL;
  if (ux > 0) t = std::fmin(t, (nx - 0.5 - x) / ux);
  if (ux < 0) t = std::fmin(t, (-0.5 - x) / ux);
  if (uy > 0) t = std::fmin(t, (ny - 0.5 - y) / uy);
  if (uy < 0) t = std::fmin(t, (-0.5 - y) / uy);
  return t;
}

}  // namespace geom
}  // namespace lbmk
