// 3-D grid kernels (the d = 3 case of the method of section 3).
#pragma once
