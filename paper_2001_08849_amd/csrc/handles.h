// Definitions of the opaque ABI handles (internal).
#pragma once
#include "gnn.h"

struct sfem_ctx {
  sfem::Ctx c;
};

struct sfem_gnn {
  sfem::Gnn g;
};
