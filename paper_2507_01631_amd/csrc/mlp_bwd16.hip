// The BF16 pipelined adjoint of the networks in a translation unit of its own,
// compiled with the register-minimising scheduler (see launch_bwd_pipe_bf16).
#define SNAKE_MLP_BWD16 1
#include "mlp.hip"
