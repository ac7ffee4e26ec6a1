// kernels.h -- all device kernels of the collective multigrid library.
#pragma once
#include "common.h"
#include "smoother.h"
#include "jacobi.h"
#include "residual.h"
#include "transfer.h"
#include "coarse.h"
#include "krylov.h"
#include "ssn.h"
#include "cvar.h"
#include "batch.h"
#include "netio.h"
