"""CPU oracle (test infrastructure only): see ipb_oracle."""
from .ipb_oracle import (Params, complete, complete_map, structuring_element, dilate, erode,
                         gaussian_taps, gaussian_sum, bilateral_sum, reflect101, N_STAGES,
                         SE_FULL, SE_CROSS, SE_DIAMOND, SE_CIRCLE, BLUR_GAUSSIAN, BLUR_BILATERAL)
