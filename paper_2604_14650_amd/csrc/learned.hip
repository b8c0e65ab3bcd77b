// Learned position model (filled in below).
#include "api_internal.hpp"

namespace planb {
struct LearnedModel {
    int unused = 0;
};
void release_learned(planb_fib_t* f)
{
    delete f->learned;
    f->learned = nullptr;
}
}  // namespace planb
