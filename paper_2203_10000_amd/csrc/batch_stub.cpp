// Placeholder for the batched form until its kernel lands.
#include "runtime.h"

using namespace sal;

extern "C" sal_status sal_label_batch(sal_context *, const sal_instance *, int32_t,
                                      const sal_label_options *, sal_label_stats *) {
    return set_error(SAL_ERR_INTERNAL, "batched form not available in this build");
}
