// Contour geometry on the host: validation, the enclosed-point test applied to candidate
// eigenvalues, and a circle that encloses the contour.
#pragma once

#include <complex>

#include "../../include/feast_mi355x.h"

// 0 when *C describes a valid contour and quadrature (either the ellipse or a glued contour), -1
// otherwise.
int contour_check(const feast_contour* C);

// True when lam lies inside C: inside the ellipse, or a nonzero winding number of the glued
// contour about lam (the value the exact Cauchy integral of eqn:cauchy_contour takes).
bool contour_inside(const feast_contour& C, std::complex<double> lam);

// Center and radius of a circle containing the contour: the ellipse's center and larger semi-axis,
// or the mean of the glued pieces' end points and the largest distance from it to any point of the
// contour.
void contour_circle(const feast_contour& C, double* c_re, double* c_im, double* radius);
