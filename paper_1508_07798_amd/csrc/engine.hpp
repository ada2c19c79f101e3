// Non-template interface between the C ABI and the device engine.
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hss.h"
#include "planner.hpp"

namespace hss {

struct EngineBase {
  virtual ~EngineBase() {}
  virtual void factor(const hss_block_op_t* A, double tol) = 0;
  virtual void apply(int nrhs, const void* x, int64_t ldx, void* y, int64_t ldy, bool on_device) = 0;
  virtual int gmres(int nrhs, const void* b, void* x, int64_t ld, double tol, int restart, int maxit,
                    bool on_device, hss_gmres_info_t* info) = 0;
  virtual bool query(const std::string& key, std::vector<double>& out) = 0;
};

std::unique_ptr<EngineBase> make_engine(std::shared_ptr<const Plan> plan, const hss_opts_t& opts, bool cplx);

}  // namespace hss
