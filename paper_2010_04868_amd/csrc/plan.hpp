// Host-side planning (no device calls).
#pragma once

#include <string>

#include "kernels.hpp"

namespace tvs {

const char* last_error();
int validate(Problem* pr, int ndim, const int64_t* dims, int dtype, int shape, int order,
             int dependence, int boundary);
int validate_life(Problem* pr, int ndim, const int64_t* dims, int boundary);
int parse_tuning(const char* str, Schedule* s, bool* has_method);
std::string format_tuning(const Problem& p, const Schedule& s);
Schedule default_schedule(const Problem& p);
int check_schedule(const Problem& p, const Schedule& s);
void choose_segment(const Problem& p, Schedule* s, bool vc = false);
Schedule varcoef_schedule(const Problem& p, const Schedule& s, bool given);
int wgs_per_cu(const BandGeom& g);
double band_cost(const Problem& p, const BandGeom& g);

}  // namespace tvs
