// Entry points not yet implemented in this build return QSV_E_UNSUPPORTED.
#include "device.hpp"

extern "C" {


}
