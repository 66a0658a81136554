// Learned strategy predictor (Sec. III-H, Listing 5; Table IV): a
// gradient-boosted tree ensemble over the features (n, k, H) evaluated on
// the host.  The file format is the project's own text format, documented
// in ahs.h.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ahs.h"

struct ahs_model {
  struct Node {
    bool leaf = false;
    int feature = 0;
    double thr = 0.0;
    int left = -1, right = -1;
    double value = 0.0;
  };
  struct Tree {
    int cls = 0;
    std::vector<Node> nodes;
  };
  double base[3] = {0, 0, 0};
  std::vector<Tree> trees;
};

extern "C" ahs_status ahs_model_load(const char* path, ahs_model** out) {
  if (!path || !out) return AHS_E_INVALID_ARG;
  *out = nullptr;
  std::ifstream in(path);
  if (!in) return AHS_E_INVALID_ARG;
  auto m = new (std::nothrow) ahs_model();
  if (!m) return AHS_E_OOM;
  std::string tok;
  int ver = 0, ncls = 0, ntrees = -1;
  auto bad = [&]() {
    delete m;
    return AHS_E_PARSE;
  };
  if (!(in >> tok >> ver) || tok != "ahs-gbt" || ver != 1) return bad();
  if (!(in >> tok >> ncls) || tok != "num_class" || ncls != 3) return bad();
  if (!(in >> tok >> m->base[0] >> m->base[1] >> m->base[2]) || tok != "base_score") return bad();
  if (!(in >> tok >> ntrees) || tok != "num_trees" || ntrees < 0 || ntrees > 100000) return bad();
  m->trees.resize((size_t)ntrees);
  for (auto& t : m->trees) {
    int nn = 0;
    if (!(in >> tok >> t.cls >> nn) || tok != "tree" || t.cls < 0 || t.cls > 2 || nn < 1 || nn > 1000000)
      return bad();
    t.nodes.resize((size_t)nn);
    std::vector<char> seen((size_t)nn, 0);
    for (int i = 0; i < nn; ++i) {
      int id = -1;
      if (!(in >> id >> tok) || id < 0 || id >= nn || seen[(size_t)id]) return bad();
      seen[(size_t)id] = 1;
      ahs_model::Node& nd = t.nodes[(size_t)id];
      if (tok == "split") {
        if (!(in >> nd.feature >> nd.thr >> nd.left >> nd.right)) return bad();
        // children strictly after the parent: no cycles
        if (nd.feature < 0 || nd.feature > 2 || nd.left <= id || nd.right <= id || nd.left >= nn || nd.right >= nn)
          return bad();
      } else if (tok == "leaf") {
        nd.leaf = true;
        if (!(in >> nd.value)) return bad();
      } else {
        return bad();
      }
    }
  }
  *out = m;
  return AHS_OK;
}

extern "C" void ahs_model_free(ahs_model* m) { delete m; }

extern "C" ahs_status ahs_model_predict(const ahs_model* m, const ahs_feature_vector* f, ahs_strategy* out) {
  if (!m || !f || !out) return AHS_E_INVALID_ARG;
  const double x[3] = {(double)f->n, (double)f->span + 1.0, f->entropy_bits};
  double score[3] = {m->base[0], m->base[1], m->base[2]};
  for (const auto& t : m->trees) {
    size_t id = 0;
    while (!t.nodes[id].leaf) {
      const auto& nd = t.nodes[id];
      id = (size_t)(x[nd.feature] < nd.thr ? nd.left : nd.right);
    }
    score[t.cls] += t.nodes[id].value;
  }
  int best = 0;
  for (int c = 1; c < 3; ++c)
    if (score[c] > score[best]) best = c;
  *out = (ahs_strategy)(AHS_COUNTING + best);
  return AHS_OK;
}
