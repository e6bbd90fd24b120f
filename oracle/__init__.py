"""FP64 CPU oracle for GlassNet (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  It shares no code with the HIP library and never imports it.
"""
from .glassnet_oracle import (adam_step, alpha_blend, all_slot_orders, dssim_loss,  # noqa: F401
                              encode, forward, ssim_map, ssim_window,
                              forward_bruteforce, grad, grad_from_dy, l1_loss, n_params, pack,
                              relu_margins, relu_signature, unpack)
from .sr_oracle import (sr_forward, sr_forward_bruteforce, sr_grad, sr_n_params,  # noqa: F401
                        sr_unpack, upsample2x)
