// Readers of the docking program's input files (include/mdock.h, "file front end"): AutoGrid
// map files, PDBQT ligands and the atom_par lines of an AutoDock parameter file.  The paper
// docks real ligands against real receptor maps (Background, "Design and Structure of
// MiniMDock"); these readers turn such files into the arrays md_receptor_create and
// md_ligand_create take.  Host code only.
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "mdock.h"

namespace mdock {
md_status api_fail(md_status st, const std::string& msg);
}  // namespace mdock

using namespace mdock;

namespace {

// The text's lines (without their end-of-line characters).
std::vector<std::string> lines_of(const char* text, long long length) {
  std::vector<std::string> out;
  std::string cur;
  for (long long i = 0; i < length; ++i) {
    const char c = text[i];
    if (c == '\n') {
      if (!cur.empty() && cur.back() == '\r') cur.pop_back();
      out.push_back(cur);
      cur.clear();
    } else {
      cur.push_back(c);
    }
  }
  if (!cur.empty()) {
    if (cur.back() == '\r') cur.pop_back();
    out.push_back(cur);
  }
  return out;
}

std::vector<std::string> tokens(const std::string& s) {
  std::vector<std::string> t;
  size_t i = 0;
  while (i < s.size()) {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    size_t j = i;
    while (j < s.size() && !std::isspace((unsigned char)s[j])) ++j;
    if (j > i) t.push_back(s.substr(i, j - i));
    i = j;
  }
  return t;
}

bool to_double(const std::string& s, double* v) {
  if (s.empty()) return false;
  char* end = nullptr;
  *v = std::strtod(s.c_str(), &end);
  while (end && *end && std::isspace((unsigned char)*end)) ++end;
  return end && *end == '\0' && std::isfinite(*v);
}

bool to_int(const std::string& s, long* v) {
  if (s.empty()) return false;
  char* end = nullptr;
  *v = std::strtol(s.c_str(), &end, 10);
  while (end && *end && std::isspace((unsigned char)*end)) ++end;
  return end && *end == '\0';
}

std::string trim(const std::string& s) {
  size_t a = 0, b = s.size();
  while (a < b && std::isspace((unsigned char)s[a])) ++a;
  while (b > a && std::isspace((unsigned char)s[b - 1])) --b;
  return s.substr(a, b - a);
}

// Single-bond covalent radii (Angstrom) of the elements AutoDock atom types name.
double covalent_radius(const std::string& element) {
  static const struct {
    const char* e;
    double r;
  } table[] = {{"H", 0.31}, {"C", 0.76}, {"N", 0.71}, {"O", 0.66}, {"F", 0.57},  {"P", 1.07},
               {"S", 1.05}, {"Cl", 1.02}, {"Br", 1.20}, {"I", 1.39}, {"Si", 1.11}, {"B", 0.84}};
  for (const auto& x : table)
    if (element == x.e) return x.r;
  return -1.0;
}

// The element of an AutoDock atom type: the type's own element, with the usual aliases
// (A aromatic carbon, NA / NS nitrogen acceptors, OA / OS oxygen acceptors, SA sulfur acceptor,
// HD / HS polar hydrogens).
std::string element_of(const std::string& type) {
  if (type == "A") return "C";
  if (type == "NA" || type == "NS") return "N";
  if (type == "OA" || type == "OS") return "O";
  if (type == "SA") return "S";
  if (type == "HD" || type == "HS") return "H";
  if (type == "CL") return "Cl";
  if (type == "BR") return "Br";
  return type;
}

std::string at_line(size_t k) { return "line " + std::to_string(k + 1) + ": "; }

}  // namespace

extern "C" {

md_status md_autogrid_map_parse(const char* text, long long length, md_grid_desc* desc, float* values,
                                long long capacity, long long* n_values) {
  if (!text || length < 0 || !desc) return api_fail(MD_EINVAL, "md_autogrid_map_parse: null argument");
  const std::vector<std::string> ls = lines_of(text, length);
  double spacing = -1.0, center[3] = {0, 0, 0};
  long ne[3] = {-1, -1, -1};
  bool have_center = false;
  size_t k = 0;
  // header: keyword lines until the first line that is a plain number
  for (; k < ls.size(); ++k) {
    const std::vector<std::string> t = tokens(ls[k]);
    if (t.empty()) continue;
    double v;
    if (t.size() == 1 && to_double(t[0], &v)) break;
    if (t[0] == "SPACING") {
      if (t.size() != 2 || !to_double(t[1], &spacing) || !(spacing > 0))
        return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) + "bad SPACING");
    } else if (t[0] == "NELEMENTS") {
      if (t.size() != 4) return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) + "bad NELEMENTS");
      for (int a = 0; a < 3; ++a)
        if (!to_int(t[1 + a], &ne[a]) || ne[a] < 2 || ne[a] % 2 != 0 || ne[a] > 100000)
          return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) +
                                         "NELEMENTS must be even interval counts >= 2");
    } else if (t[0] == "CENTER") {
      if (t.size() != 4) return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) + "bad CENTER");
      for (int a = 0; a < 3; ++a)
        if (!to_double(t[1 + a], &center[a]))
          return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) + "bad CENTER");
      have_center = true;
    } else if (t[0] == "GRID_PARAMETER_FILE" || t[0] == "GRID_DATA_FILE" || t[0] == "MACROMOLECULE") {
      // file names: informational
    } else {
      return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) + "unknown header record " + t[0]);
    }
  }
  if (spacing <= 0 || ne[0] < 0 || !have_center)
    return api_fail(MD_EINVAL, "md_autogrid_map_parse: the header needs SPACING, NELEMENTS and CENTER");
  const long long nodes = (long long)(ne[0] + 1) * (ne[1] + 1) * (ne[2] + 1);
  long long count = 0;
  for (; k < ls.size(); ++k) {
    const std::vector<std::string> t = tokens(ls[k]);
    if (t.empty()) continue;
    double v;
    if (t.size() != 1 || !to_double(t[0], &v))
      return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + at_line(k) + "expected one map value");
    if (values && count < capacity) values[count] = (float)v;
    ++count;
  }
  if (count != nodes)
    return api_fail(MD_EINVAL, "md_autogrid_map_parse: " + std::to_string(count) + " values for " +
                                   std::to_string(nodes) + " grid nodes");
  if (n_values) *n_values = count;
  if (values && capacity < count)
    return api_fail(MD_ERANGE, "md_autogrid_map_parse: values capacity below " + std::to_string(count));
  desc->nx = (int)ne[0] + 1;
  desc->ny = (int)ne[1] + 1;
  desc->nz = (int)ne[2] + 1;
  desc->spacing = (float)spacing;
  for (int a = 0; a < 3; ++a) desc->origin[a] = (float)(center[a] - spacing * (double)(ne[a] / 2));
  desc->n_types = kTypes;
  return MD_OK;
}

md_status md_pdbqt_parse(const char* text, long long length, int n_types, const char* const* type_names,
                         md_pdbqt_ligand* out) {
  if (!text || length < 0 || !out || n_types < 1 || !type_names)
    return api_fail(MD_EINVAL, "md_pdbqt_parse: null argument");
  const std::vector<std::string> ls = lines_of(text, length);
  struct Atom {
    long serial;
    double x, y, z, q;
    int type;
    std::string element;
  };
  std::vector<Atom> atoms;
  std::vector<std::pair<long, long>> branches;   // (root-side serial, far-side serial)
  int depth = 0;
  bool in_root = false, root_seen = false;
  for (size_t k = 0; k < ls.size(); ++k) {
    const std::string& l = ls[k];
    const std::vector<std::string> t = tokens(l);
    if (t.empty()) continue;
    const std::string rec = t[0];
    if (rec == "ROOT") {
      if (root_seen) return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "second ROOT");
      in_root = root_seen = true;
    } else if (rec == "ENDROOT") {
      in_root = false;
    } else if (rec == "BRANCH" || rec == "ENDBRANCH") {
      long a, b;
      if (t.size() != 3 || !to_int(t[1], &a) || !to_int(t[2], &b))
        return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "bad " + rec + " record");
      if (rec == "BRANCH") {
        branches.push_back({a, b});
        ++depth;
      } else {
        if (--depth < 0) return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "unmatched ENDBRANCH");
      }
    } else if (rec == "ATOM" || rec == "HETATM") {
      // fixed columns for the serial number and coordinates; the partial charge and the
      // AutoDock type are the record's last two fields
      if (l.size() < 54) return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "short atom record");
      Atom a;
      double v;
      if (!to_int(trim(l.substr(6, 5)), &a.serial) || !to_double(trim(l.substr(30, 8)), &a.x) ||
          !to_double(trim(l.substr(38, 8)), &a.y) || !to_double(trim(l.substr(46, 8)), &a.z))
        return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "bad serial number or coordinates");
      const std::vector<std::string> tail = tokens(l.substr(54));
      if (tail.size() < 2 || !to_double(tail[tail.size() - 2], &v))
        return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "missing partial charge or atom type");
      a.q = v;
      const std::string& ty = tail.back();
      a.type = -1;
      for (int i = 0; i < n_types; ++i)
        if (type_names[i] && ty == type_names[i]) a.type = i;
      if (a.type < 0)
        return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "atom type " + ty +
                                       " has no map among the receptor's types");
      a.element = element_of(ty);
      if (covalent_radius(a.element) < 0)
        return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "no covalent radius for atom type " + ty);
      for (const Atom& b : atoms)
        if (b.serial == a.serial)
          return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "serial number used twice");
      atoms.push_back(a);
    } else if (rec == "TORSDOF" || rec == "REMARK" || rec == "MODEL" || rec == "ENDMDL" || rec == "TER" ||
               rec == "END" || rec == "USER" || rec == "COMPND") {
      // not needed: the rotatable bonds are the BRANCH records
    } else {
      return api_fail(MD_EINVAL, "md_pdbqt_parse: " + at_line(k) + "unknown record " + rec);
    }
  }
  (void)in_root;
  if (depth != 0) return api_fail(MD_EINVAL, "md_pdbqt_parse: unmatched BRANCH");
  if (!root_seen || atoms.empty()) return api_fail(MD_EINVAL, "md_pdbqt_parse: no ROOT or no atoms");
  const int n = (int)atoms.size();
  auto index_of = [&](long serial) {
    for (int i = 0; i < n; ++i)
      if (atoms[i].serial == serial) return i;
    return -1;
  };
  // bonds: atom pairs closer than 1.2 x the sum of their covalent radii, plus every BRANCH bond
  std::vector<std::pair<int, int>> bonds;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const double dx = atoms[i].x - atoms[j].x, dy = atoms[i].y - atoms[j].y, dz = atoms[i].z - atoms[j].z;
      const double lim = 1.2 * (covalent_radius(atoms[i].element) + covalent_radius(atoms[j].element));
      if (dx * dx + dy * dy + dz * dz <= lim * lim) bonds.push_back({i, j});
    }
  std::vector<int> torsions;
  for (const auto& br : branches) {
    const int a = index_of(br.first), b = index_of(br.second);
    if (a < 0 || b < 0) return api_fail(MD_EINVAL, "md_pdbqt_parse: BRANCH names an atom that is not in the file");
    int found = -1;
    for (size_t k = 0; k < bonds.size(); ++k)
      if ((bonds[k].first == std::min(a, b) && bonds[k].second == std::max(a, b))) found = (int)k;
    if (found < 0) {
      bonds.push_back({std::min(a, b), std::max(a, b)});
      found = (int)bonds.size() - 1;
    }
    torsions.push_back(found);
  }
  out->n_atoms = n;
  out->n_bonds = (int)bonds.size();
  out->n_torsions = (int)torsions.size();
  out->root_atom = 0;
  if (n > out->max_atoms || out->n_bonds > out->max_bonds || out->n_torsions > out->max_torsions)
    return api_fail(MD_ERANGE, "md_pdbqt_parse: capacities below the ligand's " + std::to_string(n) + " atoms, " +
                                   std::to_string(out->n_bonds) + " bonds, " + std::to_string(out->n_torsions) +
                                   " torsions (counts are set)");
  if (!out->xyz || !out->charge || !out->type || (out->n_bonds && !out->bonds) || (out->n_torsions && !out->torsions))
    return api_fail(MD_EINVAL, "md_pdbqt_parse: null output array");
  for (int i = 0; i < n; ++i) {
    out->xyz[3 * i] = (float)atoms[i].x;
    out->xyz[3 * i + 1] = (float)atoms[i].y;
    out->xyz[3 * i + 2] = (float)atoms[i].z;
    out->charge[i] = (float)atoms[i].q;
    out->type[i] = atoms[i].type;
    if (out->serial) out->serial[i] = (int)atoms[i].serial;
  }
  for (size_t k = 0; k < bonds.size(); ++k) {
    out->bonds[2 * k] = bonds[k].first;
    out->bonds[2 * k + 1] = bonds[k].second;
  }
  for (size_t k = 0; k < torsions.size(); ++k) out->torsions[k] = torsions[k];
  return MD_OK;
}

md_status md_atom_par_parse(const char* text, long long length, int n_types, const char* const* type_names,
                            float* type_params) {
  if (!text || length < 0 || n_types < 1 || !type_names || !type_params)
    return api_fail(MD_EINVAL, "md_atom_par_parse: null argument");
  const std::vector<std::string> ls = lines_of(text, length);
  std::vector<char> found(n_types, 0);
  for (size_t k = 0; k < ls.size(); ++k) {
    const std::vector<std::string> t = tokens(ls[k]);
    if (t.empty() || t[0] != "atom_par") continue;
    if (t.size() < 9) return api_fail(MD_EINVAL, "md_atom_par_parse: " + at_line(k) + "short atom_par record");
    int ti = -1;
    for (int i = 0; i < n_types; ++i)
      if (type_names[i] && t[1] == type_names[i]) ti = i;
    if (ti < 0) continue;
    double v[7];
    long hb;
    for (int c = 0; c < 6; ++c)
      if (!to_double(t[2 + c], &v[c]))
        return api_fail(MD_EINVAL, "md_atom_par_parse: " + at_line(k) + "bad number");
    if (!to_int(t[8], &hb) || hb < 0 || hb > 5)
      return api_fail(MD_EINVAL, "md_atom_par_parse: " + at_line(k) + "bad hbond code");
    // columns: Rii, epsii, vol, solpar, Rij_hb, epsij_hb, hbond; hbond 1-2 donor, 3-5 acceptor
    float* row = type_params + 7 * ti;
    row[0] = (float)v[0];
    row[1] = (float)v[1];
    row[2] = (float)v[2];
    row[3] = (float)v[3];
    row[4] = hb == 0 ? 0.f : (hb <= 2 ? 1.f : 2.f);
    row[5] = (float)v[4];
    row[6] = (float)v[5];
    found[ti] = 1;
  }
  for (int i = 0; i < n_types; ++i)
    if (!found[i])
      return api_fail(MD_EINVAL, std::string("md_atom_par_parse: no atom_par record for type ") +
                                     (type_names[i] ? type_names[i] : "(null)"));
  return MD_OK;
}

}  // extern "C"
