// Single translation unit of libspoly.so: the persistent mixed kernel calls
// the one-vertex and two-vertex solve bodies as device functions, so every
// module is compiled together.
#include "api.hip"
#include "cull.hip"
#include "onebounce.hip"
#include "twobounce.hip"
#include "pruner.hip"
#include "mixed.hip"
#include "tail.hip"
#include "order.hip"
